"""Two-grid fast-LGF approximation on the GPU (lgf_plan_create_flgf)
against the oracle's same approximation (parity), and its error against
the exact sum (the approximation's budget)."""
import numpy as np
import pytest

from oracle import flgf
from paper_2010_13213_amd import inputs
from helpers import rel_l2

pytestmark = pytest.mark.gpu


def _solve(ctx, prob, near=None):
    import torch
    from paper_2010_13213_amd import lgf
    plan = lgf.Plan.for_problem(ctx, prob, flgf_near=near)
    u = plan.solve(torch.from_numpy(prob.flat_source()).cuda()).cpu().numpy().reshape(prob.n_components, -1)
    plan.close()
    return u


def _box(ex, ey, ez, seed, nc=2):
    b = np.array([(x, y, z) for z in range(ez) for y in range(ey) for x in range(ex)], dtype=np.int32)
    c = inputs.cell_coords(b, 16).astype(float)
    rng = np.random.default_rng(seed)
    vals = []
    for _ in range(nc):
        ctr = rng.uniform(8, 16 * np.array([ex, ey, ez]) - 8)
        vals.append(np.exp(-((c - ctr) ** 2).sum(1) / (2 * 9.0 ** 2)) + 0.05 * rng.standard_normal(len(c)))
    return inputs.Problem(nb=16, dx0=0.5, levels=[inputs.Level(blocks=b, values=np.stack(vals).reshape(nc, len(b), 16, 16, 16))])


@pytest.mark.parametrize("near", [0, 1])
def test_flgf_matches_oracle_approximation(gpu_ctx, near):
    prob = _box(4, 3, 2, 1)
    u = _solve(gpu_ctx, prob, near)
    c = inputs.cell_coords(prob.levels[0].blocks, 16)
    idx = np.random.default_rng(2).choice(len(c), 150, replace=False)
    f = prob.flat_source().reshape(2, -1)
    for comp in range(2):
        ref = flgf.flgf(c, f[comp], c[idx], prob.dx0, 16, near)
        assert rel_l2(u[comp][idx], ref) < 1e-12, (near, comp)


def test_flgf_error_budget_on_the_ring(gpu_ctx):
    """Config 2's ring (208 blocks of 16^3): the approximation against the
    exact GPU sum for near radii 1 and 2."""
    prob = inputs.single_ring(components=(0, 1))
    exact = _solve(gpu_ctx, prob)
    errs = []
    for near in (1, 2):
        u = _solve(gpu_ctx, prob, near)
        errs.append(max(rel_l2(u[c], exact[c]) for c in range(2)))
    print("fast-LGF rel L2 vs exact, near radius 1, 2:", errs, flush=True)
    assert errs[0] < 2e-5 and errs[1] < 2e-6, errs
