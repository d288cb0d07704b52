"""Vector solves and extent limits.

Components run through the MAC in groups of up to three (one launch serves
every component of a group).  Each component of a vector solve has the same
arithmetic, in the same order, as a scalar solve of that component alone,
so the results must be equal bit for bit, for any number of components
(here 4 and 5: a full group plus a partial one).  Extents: 64 blocks along
an axis is the largest supported (checked against the oracle on sampled
cells), 65 is refused with LGF_E_UNSUPPORTED.
"""
import numpy as np
import pytest

from oracle import direct
from paper_2010_13213_amd import inputs
from helpers import rel_l2

pytestmark = pytest.mark.gpu


def _cube(n, lo=(0, 0, 0)):
    return np.array([(lo[0] + x, lo[1] + y, lo[2] + z) for z in range(n) for y in range(n)
                     for x in range(n)], dtype=np.int32)


def _solve(ctx, blocks, nb, dx0, fields, precision):
    """fields: (n_comp, n_cells_total) numpy -> same shape."""
    import torch
    from paper_2010_13213_amd import lgf
    plan = lgf.Plan(ctx, blocks, nb, dx0, fields.shape[0], precision)
    u = plan.solve(torch.from_numpy(np.ascontiguousarray(fields).reshape(-1)).cuda())
    out = u.cpu().numpy().reshape(fields.shape)
    plan.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_five_components_equal_five_scalar_solves(gpu_ctx, precision):
    p = inputs.single_ring(components=(0,))
    blocks = [p.levels[0].blocks]
    n = len(blocks[0]) * p.nb ** 3
    rng = np.random.default_rng(31)
    base = p.levels[0].values.reshape(-1)
    fields = np.stack([base * (1 + c) + 1e-3 * rng.standard_normal(n) for c in range(5)])
    vec = _solve(gpu_ctx, blocks, p.nb, p.dx0, fields, precision)
    for c in range(5):
        one = _solve(gpu_ctx, blocks, p.nb, p.dx0, fields[c:c + 1], precision)
        assert np.array_equal(vec[c], one[0]), (precision, c)


def test_four_component_composite_equals_scalar_solves(gpu_ctx):
    nb = 8
    blocks = [_cube(4), _cube(2, lo=(1, 2, 1))]
    n = sum(len(b) for b in blocks) * nb ** 3
    rng = np.random.default_rng(32)
    fields = rng.standard_normal((4, n))
    vec = _solve(gpu_ctx, blocks, nb, 0.25, fields, "fp64")
    for c in range(4):
        one = _solve(gpu_ctx, blocks, nb, 0.25, fields[c:c + 1], "fp64")
        assert np.array_equal(vec[c], one[0]), c


@pytest.mark.parametrize("axis", [0, 2])
def test_extent_of_64_blocks_is_supported(gpu_ctx, axis):
    nb = 8
    rng = np.random.default_rng(33 + axis)
    line = np.zeros((64, 3), dtype=np.int32)
    line[:, axis] = np.arange(64) - 20
    extra = line[rng.uniform(size=64) < 0.25].copy()
    extra[:, (axis + 1) % 3] += 1
    blocks = np.concatenate([line, extra])
    c = inputs.cell_coords(blocks, nb)
    f = rng.standard_normal(len(c))
    u = _solve(gpu_ctx, [blocks], nb, 0.4, f[None], "fp64")[0]
    tgt = rng.choice(len(c), 2000, replace=False)
    ref = direct.direct_sum(c, f, c[tgt], 0.4)
    assert rel_l2(u[tgt], ref) < 1e-12


def test_extent_of_65_blocks_is_refused(gpu_ctx):
    from paper_2010_13213_amd import lgf
    blocks = np.zeros((65, 3), dtype=np.int32)
    blocks[:, 1] = np.arange(65)
    with pytest.raises(lgf.LgfError) as e:
        lgf.Plan(gpu_ctx, [blocks], 8, 1.0, 1, "fp64")
    assert e.value.status == lgf.LGF_E_UNSUPPORTED
