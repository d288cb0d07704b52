"""Host-side checks of the C ABI (no GPU work): symbols and validation."""
import re
import os

import numpy as np
import pytest

from paper_2010_13213_amd import lgf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "lgf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lgf_[a-z_]+)\s*\(", text)))


def test_header_declares_the_binding_symbols():
    assert set(_declared()) == set(lgf.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = lgf.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_status_strings():
    L = lgf.lib()
    assert L.lgf_status_string(0) == b"LGF_OK"
    assert L.lgf_status_string(1) == b"LGF_E_INVALID"
    assert L.lgf_table_radius() == 128


def test_build_id_names_the_sources_in_the_tree():
    from paper_2010_13213_amd import build
    bid = lgf.build_id()
    assert re.fullmatch(r"sha256=[0-9a-f]{64} arch=gfx950", bid), bid
    assert bid.split()[0] == "sha256=" + build.source_digest()


def test_stale_library_is_refused():
    with pytest.raises(RuntimeError, match="built from other sources"):
        lgf._check_build("sha256=" + "0" * 64 + " arch=gfx950")


def _cube(n, lo=0):
    return np.array([(x, y, z) for z in range(lo, lo + n) for y in range(lo, lo + n)
                     for x in range(lo, lo + n)])


def test_problem_check_accepts_valid_problems():
    st, msg = lgf.problem_check([_cube(2)], 8, 1.0)
    assert st == lgf.LGF_OK, msg
    coarse, fine = _cube(4), _cube(2, lo=2)   # fine blocks 2,3 -> parents 1
    st, msg = lgf.problem_check([coarse, fine], 16, 0.5, 3)
    assert st == lgf.LGF_OK, msg


@pytest.mark.parametrize("case", ["dup", "nb", "dx", "comp", "nest", "empty", "prec"])
def test_problem_check_rejects_malformed_problems(case):
    args = dict(level_blocks=[_cube(2)], nb=8, dx0=1.0, n_components=1, precision="fp64")
    if case == "dup":
        args["level_blocks"] = [np.array([[0, 0, 0], [1, 0, 0], [0, 0, 0]])]
    elif case == "nb":
        args["nb"] = 12
    elif case == "dx":
        args["dx0"] = -1.0
    elif case == "comp":
        args["n_components"] = 9
    elif case == "nest":
        args["level_blocks"] = [_cube(2), np.array([[9, 0, 0]])]
    elif case == "empty":
        args["level_blocks"] = [np.zeros((0, 3), dtype=np.int32)]
    elif case == "prec":
        args["precision"] = 7
    st, msg = lgf.problem_check(**args)
    assert st == lgf.LGF_E_INVALID and msg


def test_null_arguments_are_rejected_without_a_device():
    import ctypes
    L = lgf.lib()
    assert L.lgf_plan_create(None, None, None) == lgf.LGF_E_INVALID
    assert L.lgf_solve(None, None, None, None, None) == lgf.LGF_E_INVALID
    out = ctypes.c_void_p()
    assert L.lgf_context_create(0, 0, None) == lgf.LGF_E_INVALID


def test_problem_check_cell_masks():
    coarse, fine = _cube(2), _cube(2, lo=2)           # fine blocks 2,3 refine coarse block (1,1,1)
    nb = 8
    m0 = np.ones((len(coarse), nb, nb, nb), dtype=np.uint8)
    i = [tuple(b) for b in coarse.tolist()].index((1, 1, 1))
    m0[i] = 0                                          # the refined block dropped entirely: valid
    m0[0, :2] = 0                                      # and some uncovered cells: valid
    st, msg = lgf.problem_check([coarse, fine], nb, 1.0, cell_masks=[m0, None])
    assert st == lgf.LGF_OK, msg
    bad = m0.copy()
    bad[i, 7, 7, 7] = 1                                # a covered cell kept: the levels overlap
    st, msg = lgf.problem_check([coarse, fine], nb, 1.0, cell_masks=[bad, None])
    assert st == lgf.LGF_E_INVALID and "overlap" in msg
    two = m0.copy()
    two[0, 5, 5, 5] = 2
    st, msg = lgf.problem_check([coarse, fine], nb, 1.0, cell_masks=[two, None])
    assert st == lgf.LGF_E_INVALID and "0 or 1" in msg
