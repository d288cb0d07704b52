"""Integrating factor H(a) = exp(a L) on the GPU (paper Sec. 2.3, eq.
IF-single; Sec. 3.5, eq. FIF-AMR) against the oracle, through
lgf_plan_create_if: one level with both block sizes and several a, a
two-level and the three-level colliding-ring mesh, and batched = alone."""
import numpy as np
import pytest

from oracle import heat
from paper_2010_13213_amd import inputs
from helpers import rel_l2

pytestmark = pytest.mark.gpu


def _solve(ctx, prob, a0):
    import torch
    from paper_2010_13213_amd import lgf
    plan = lgf.Plan.for_problem(ctx, prob, if_a0=a0)
    u = plan.solve(torch.from_numpy(prob.flat_source()).cuda()).cpu().numpy().reshape(prob.n_components, -1)
    plan.close()
    return u


def _random_box(n_blk, nb, seed, nc=1, dx=1.0):
    b = np.array([(x, y, z) for z in range(n_blk) for y in range(n_blk) for x in range(n_blk)], dtype=np.int32)
    vals = np.random.default_rng(seed).standard_normal((nc, len(b), nb, nb, nb))
    return inputs.Problem(nb=nb, dx0=dx, levels=[inputs.Level(blocks=b, values=vals)])


@pytest.mark.parametrize("a", [0.05, 1.0, 6.0])
def test_single_level_full_parity(gpu_ctx, a):
    prob = _random_box(2, 8, 1)
    c = inputs.cell_coords(prob.levels[0].blocks, 8)
    got = _solve(gpu_ctx, prob, a)[0]
    ref = heat.apply(c, prob.flat_source(), c, a)
    assert rel_l2(got, ref) < 1e-12


def test_single_level_16_blocks_sampled(gpu_ctx):
    prob = _random_box(3, 16, 2, nc=2)
    c = inputs.cell_coords(prob.levels[0].blocks, 16)
    got = _solve(gpu_ctx, prob, 2.5)
    idx = np.random.default_rng(3).choice(len(c), 400, replace=False)
    f = prob.flat_source().reshape(2, -1)
    for comp in range(2):
        assert rel_l2(got[comp][idx], heat.apply(c, f[comp], c[idx], 2.5)) < 1e-12


def _two_level(nc=2, seed=4):
    rng = np.random.default_rng(seed)
    b0 = np.array([(x, y, z) for z in range(3) for y in range(3) for x in range(3)], dtype=np.int32)
    b1 = np.array([(2, 2, 2), (3, 2, 2), (2, 3, 3), (3, 3, 3)], dtype=np.int32)
    return inputs.Problem(nb=8, dx0=0.5, levels=[
        inputs.Level(blocks=b0, values=rng.standard_normal((nc, len(b0), 8, 8, 8))),
        inputs.Level(blocks=b1, values=rng.standard_normal((nc, len(b1), 8, 8, 8)))])


def _check_composite(got, prob, a0, n_sample, seed):
    """Sampled phi_k of every level against the oracle.  H(a) is positive
    and conserves the sum, so |H f| <= max|f|: the error is measured against
    max|f| (on coarse levels far from the refined sources phi_k is many
    orders below it, and a relative error there would measure only the
    rounding of the nearby large values)."""
    rng = np.random.default_rng(seed)
    blocks = [lv.blocks for lv in prob.levels]
    from oracle import composite as C
    orc = C.CompositeOracle(prob.nb, prob.dx0, blocks)
    samp = [np.sort(rng.choice(np.nonzero(orc.mask[k])[0], min(n_sample, int(orc.mask[k].sum())), replace=False))
            for k in range(len(blocks))]
    for c in range(prob.n_components):
        ref = heat.fif_solve(prob.nb, prob.dx0, blocks, [lv.values[c].reshape(-1) for lv in prob.levels], a0,
                             sample=samp)
        scale = max(np.abs(lv.values[c]).max() for lv in prob.levels)
        base = 0
        for k, lv in enumerate(prob.levels):
            n = len(lv.blocks) * prob.nb ** 3
            assert np.abs(got[c][base:base + n][samp[k]] - ref[k][samp[k]]).max() < 1e-13 * scale, (c, k)
            if np.abs(ref[k][samp[k]]).max() > 1e-3 * scale:
                assert rel_l2(got[c][base:base + n][samp[k]], ref[k][samp[k]]) < 1e-12, (c, k)
            base += n


def test_two_level_composite_against_oracle(gpu_ctx):
    prob = _two_level()
    got = _solve(gpu_ctx, prob, 0.4)
    _check_composite(got, prob, 0.4, 600, 5)


def test_three_level_colliding_rings_against_oracle(gpu_ctx):
    prob = inputs.colliding_rings(nb=8, dx0=1.0 / 8, components=(0,))
    got = _solve(gpu_ctx, prob, 0.3)
    _check_composite(got, prob, 0.3, 150, 6)


def test_batch_with_integrating_factor_plans_equals_alone(gpu_ctx):
    import torch
    from paper_2010_13213_amd import lgf
    cases = [(_two_level(), 0.4), (_random_box(2, 8, 7), 1.5), (inputs.gaussian_box(), None), (_two_level(1, 8), None)]
    plans = [lgf.Plan.for_problem(gpu_ctx, p, if_a0=a) for p, a in cases]
    fs = [torch.from_numpy(p.flat_source()).cuda() for p, _ in cases]
    alone = [pl.solve(f).cpu().numpy() for pl, f in zip(plans, fs)]
    us = [torch.full_like(f, float("nan")) for f in fs]
    lgf.solve_batch(gpu_ctx, plans, fs, us)
    torch.cuda.synchronize()
    for a, u in zip(alone, us):
        assert np.array_equal(a, u.cpu().numpy())
    for pl in plans:
        pl.close()


def test_integrating_factor_refuses_mixed_precision(gpu_ctx):
    from paper_2010_13213_amd import lgf
    with pytest.raises(lgf.LgfError) as e:
        lgf.Plan.for_problem(gpu_ctx, _random_box(1, 8, 0), precision="fp32_refine", if_a0=0.5)
    assert e.value.status == lgf.LGF_E_UNSUPPORTED
