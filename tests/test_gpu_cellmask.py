"""Cell masks of lgf_level (the partition of Sec. 3.1 stated cell by cell)
on the GPU against the oracle with the same masks."""
import numpy as np
import pytest

from oracle import composite as C, direct
from paper_2010_13213_amd import inputs
from helpers import rel_l2

pytestmark = pytest.mark.gpu


def _cube(n, lo=(0, 0, 0)):
    return np.array([(lo[0] + x, lo[1] + y, lo[2] + z) for z in range(n) for y in range(n)
                     for x in range(n)], dtype=np.int32)


def _solve(ctx, prob, precision="fp64"):
    import torch
    from paper_2010_13213_amd import lgf
    plan = lgf.Plan.for_problem(ctx, prob, precision)
    u = plan.solve(torch.from_numpy(prob.flat_source()).cuda()).cpu().numpy().reshape(prob.n_components, -1)
    plan.close()
    return u


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_refine", 1e-10)])
def test_single_level_mask(gpu_ctx, precision, tol):
    nb = 8
    b = _cube(3)
    rng = np.random.default_rng(3)
    c = inputs.cell_coords(b, nb)
    f = np.exp(-(((c - 12.0) / 5.0) ** 2).sum(1)) + 0.01 * rng.standard_normal(len(c))
    mask = (((c - 12.0) ** 2).sum(1) < 11.5 ** 2).astype(np.uint8)     # a ball inside the box of blocks
    prob = inputs.Problem(nb=nb, dx0=0.5, levels=[inputs.Level(
        blocks=b, values=f.reshape(1, len(b), nb, nb, nb), cell_mask=mask.reshape(len(b), nb, nb, nb))])
    u = _solve(gpu_ctx, prob, precision)[0]
    keep = mask.astype(bool)
    ref = direct.direct_sum(c[keep], f[keep], c[keep], 0.5)
    assert rel_l2(u[keep], ref) < tol
    assert np.all(u[~keep] == 0.0)


def test_two_level_hand_masked_coarse_block(gpu_ctx):
    nb = 8
    blocks = [_cube(4), _cube(2, lo=(2, 2, 2))]
    rng = np.random.default_rng(5)
    orc0 = C.CompositeOracle(nb, 1.0, blocks)
    masks = [orc0.mask[0].copy(), orc0.mask[1].copy()]
    # drop a corner slab of an uncovered coarse block and a few fine cells
    cells0 = orc0.cells[0]
    masks[0] &= ~((cells0[:, 0] < 6) & (cells0[:, 1] < 6))
    masks[1][::5] = False
    vals = [rng.standard_normal((2, len(b), nb, nb, nb)) for b in blocks]
    prob = inputs.Problem(nb=nb, dx0=1.0, levels=[
        inputs.Level(blocks=blocks[k], values=vals[k], cell_mask=masks[k].astype(np.uint8).reshape(-1, nb, nb, nb))
        for k in range(2)])
    u = _solve(gpu_ctx, prob)
    orc = C.CompositeOracle(nb, 1.0, blocks, cell_masks=masks)
    n0 = len(orc.cells[0])
    for comp in range(2):
        ref = orc.solve([vals[k][comp].reshape(-1) for k in range(2)])
        for k, part in enumerate([u[comp][:n0], u[comp][n0:]]):
            m = orc.mask[k]
            assert rel_l2(part[m], ref[k][m]) < 1e-12, (comp, k)
            assert np.all(part[~m] == 0.0)


def test_mask_equal_to_the_cover_changes_nothing_and_batches(gpu_ctx):
    import torch
    from paper_2010_13213_amd import lgf
    nb = 8
    blocks = [_cube(3), _cube(2, lo=(1, 1, 1))]
    orc = C.CompositeOracle(nb, 1.0, blocks)
    rng = np.random.default_rng(7)
    vals = [rng.standard_normal((1, len(b), nb, nb, nb)) for b in blocks]
    plain = inputs.Problem(nb=nb, dx0=1.0, levels=[inputs.Level(blocks=blocks[k], values=vals[k]) for k in range(2)])
    masked = inputs.Problem(nb=nb, dx0=1.0, levels=[
        inputs.Level(blocks=blocks[k], values=vals[k], cell_mask=orc.mask[k].astype(np.uint8).reshape(-1, nb, nb, nb))
        for k in range(2)])
    assert np.array_equal(_solve(gpu_ctx, plain), _solve(gpu_ctx, masked))
    one = inputs.Problem(nb=nb, dx0=1.0, levels=[inputs.Level(
        blocks=blocks[0], values=vals[0], cell_mask=(rng.uniform(size=(len(blocks[0]), nb, nb, nb)) < 0.7).astype(np.uint8))])
    cases = [masked, one, inputs.gaussian_box()]
    plans = [lgf.Plan.for_problem(gpu_ctx, p) for p in cases]
    fs = [torch.from_numpy(p.flat_source()).cuda() for p in cases]
    alone = [pl.solve(f).cpu().numpy() for pl, f in zip(plans, fs)]
    us = [torch.empty_like(f) for f in fs]
    lgf.solve_batch(gpu_ctx, plans, fs, us)
    torch.cuda.synchronize()
    for a, u in zip(alone, us):
        assert np.array_equal(a, u.cpu().numpy())
    for pl in plans:
        pl.close()
