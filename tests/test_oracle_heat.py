"""Pins of the integrating-factor oracle (paper Sec. 2.3, Sec. 3.5).

* mass: sum_n E(n) = 1 (exp(a L) conserves the sum: L annihilates constants);
* semigroup: H(b) H(a) f = H(a + b) f;
* the heat equation itself: d/da H(a) f = L H(a) f (central difference in a,
  second-order convergence in the step);
* a -> 0: H(a) = 1 + a L + O(a^2);
* composite (eq. FIF-AMR): one level reduces to the plain convolution; a
  coarse-only source whose interpolation lies inside the extended region
  gives phi_1 = H(4 a0) P f^_0 exactly; a fine-only source gives
  phi_1 = H(4 a0) f^_1 and phi_0 = H(a0) (mean of the 8 children of f^_1).
"""
import numpy as np
import pytest

from oracle import composite as C, heat


def _cube(lo, n):
    ax = np.arange(lo, lo + n)
    g = np.meshgrid(ax, ax, ax, indexing="ij")
    return np.stack([v.ravel() for v in g], axis=1)


@pytest.mark.parametrize("a", [0.05, 0.7, 3.0])
def test_kernel_conserves_mass(a):
    B = heat.kernel_row(a, 60)
    assert abs((B[0] + 2.0 * B[1:].sum()) ** 3 - 1.0) < 1e-14


def test_semigroup():
    rng = np.random.default_rng(0)
    src = _cube(-2, 5)
    f = rng.standard_normal(len(src))
    mid = _cube(-22, 45)
    tgt = _cube(-4, 9)
    one = heat.apply(mid, heat.apply(src, f, mid, 0.8), tgt, 1.3)
    two = heat.apply(src, f, tgt, 2.1)
    assert np.abs(one - two).max() < 1e-13 * np.abs(two).max()


def test_solves_the_heat_equation():
    rng = np.random.default_rng(1)
    src = _cube(-2, 5)
    f = rng.standard_normal(len(src))
    tgt = _cube(-3, 7)
    nbr = [np.array(o) for o in [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)]]
    a = 0.9
    Hf = lambda c, aa: heat.apply(src, f, c, aa)
    LHf = sum(Hf(tgt + o, a) for o in nbr) - 6.0 * Hf(tgt, a)
    errs = []
    for h in (1e-2, 5e-3):
        d = (Hf(tgt, a + h) - Hf(tgt, a - h)) / (2 * h)
        errs.append(np.abs(d - LHf).max() / np.abs(LHf).max())
    assert errs[0] < 1e-3 and 3.5 < errs[0] / errs[1] < 4.5, errs


def test_small_a_is_identity_plus_a_laplacian():
    rng = np.random.default_rng(2)
    src = _cube(0, 4)
    f = rng.standard_normal(len(src))
    tgt = _cube(-1, 6)
    a = 1e-4
    u = heat.apply(src, f, tgt, a)
    fa = dict(zip(map(tuple, src.tolist()), f))
    val = lambda c: fa.get(tuple(c), 0.0)
    ref = np.array([val(c) + a * (sum(val(c + o) for o in np.vstack([np.eye(3, dtype=int), -np.eye(3, dtype=int)]))
                                  - 6 * val(c)) for c in tgt])
    assert np.abs(u - ref).max() < 5 * a * a * 36 * np.abs(f).max()


def _bump(cells, ctr, R):
    t2 = (((cells + 0.5) - ctr) ** 2).sum(axis=1) / (R * R)
    out = np.zeros(len(cells))
    m = t2 < 1
    out[m] = np.exp(-4.0 / (1.0 - t2[m]))
    return out


def test_composite_one_level_is_the_plain_convolution():
    b = _cube(0, 2)
    orc = C.CompositeOracle(4, 1.0, [b])
    f = np.random.default_rng(3).standard_normal(len(orc.cells[0]))
    phi = heat.fif_solve(4, 1.0, [b], [f], 0.6)[0]
    assert np.array_equal(phi, heat.apply(orc.cells[0], f, orc.cells[0], 0.6))


def _two_level():
    coarse = _cube(0, 4)                  # 4^3 blocks of 4^3: coarse cells [0, 16)^3
    fine = _cube(2, 2)                    # level-1 cells [8, 16)^3 = coarse [4, 8)^3
    return 4, [coarse, fine]


def test_composite_coarse_source_is_interpolated_then_convolved():
    nb, blocks = _two_level()
    orc = C.CompositeOracle(nb, 1.0, blocks, ext_layers=3)
    f0 = _bump(orc.cells[0], np.array([10.0, 6.0, 6.0]), 2.2)       # coarse x in (7.8, 12.2): Omega_0
    assert np.all(orc.mask[0][f0 != 0])
    f1 = np.zeros(len(orc.cells[1]))
    a0 = 0.3
    phi = heat.fif_solve(nb, 1.0, blocks, [f0, f1], a0, ext_layers=3)
    m0 = orc.mask[0]
    assert np.abs(phi[0][m0] - heat.apply(orc.cells[0], f0, orc.cells[0][m0], a0)).max() < 1e-15
    box = C.Box(np.array([-2] * 3), np.array([18] * 3))
    arr = box.zeros()
    i, j, k = box.idx(orc.cells[0])
    arr[i, j, k] = f0
    fine = C.Box(np.array([0] * 3), np.array([32] * 3)).cells()
    Pf = C.interp_trilinear(box, arr, fine)
    # R_1 (level-1 blocks dilated by 3 blocks: cells [-4, 28)^3) holds the whole of P f^_0
    assert np.all(np.all((fine[Pf != 0] >= -4) & (fine[Pf != 0] < 28), axis=1))
    assert Pf.reshape(32, 32, 32)[-1].max() == 0.0
    ref1 = heat.apply(fine, Pf, orc.cells[1], 4 * a0)
    assert np.abs(phi[1] - ref1).max() < 1e-14 * np.abs(ref1).max()


def test_composite_fine_source_is_coarsened_below_and_convolved_above():
    nb, blocks = _two_level()
    orc = C.CompositeOracle(nb, 1.0, blocks)
    f1 = _bump(orc.cells[1], np.array([12.0, 12.0, 12.0]), 3.5)
    f0 = np.zeros(len(orc.cells[0]))
    a0 = 0.25
    phi = heat.fif_solve(nb, 1.0, blocks, [f0, f1], a0)
    ref1 = heat.apply(orc.cells[1], f1, orc.cells[1], 4 * a0)
    assert np.abs(phi[1] - ref1).max() < 1e-15
    # the 8-children mean by reshaping the fine block cube, independent of the oracle's helper
    fa = np.zeros((8, 8, 8))
    c = orc.cells[1] - 8
    fa[c[:, 0], c[:, 1], c[:, 2]] = f1
    F = fa.reshape(4, 2, 4, 2, 4, 2).mean(axis=(1, 3, 5)).ravel()
    cc = C.Box(np.array([4] * 3), np.array([8] * 3)).cells()
    m0 = orc.mask[0]
    ref0 = heat.apply(cc, F, orc.cells[0][m0], a0)
    assert np.abs(phi[0][m0] - ref0).max() < 1e-15
