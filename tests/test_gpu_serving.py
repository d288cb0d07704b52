"""Batched and served solves: every result equals the request solved alone.

lgf_solve_batch runs the block FFTs and spectral products of all requests in
shared launches; each request's reduction order is fixed by its own plan,
so the batched result must match lgf_solve bit for bit (and the oracle to
the path's tolerance).
"""
import numpy as np
import pytest

from oracle import direct
from paper_2010_13213_amd import inputs
from helpers import rel_l2

pytestmark = pytest.mark.gpu


def _alone(ctx, reqs):
    import torch
    from paper_2010_13213_amd import lgf
    out = []
    for r in reqs:
        plan = lgf.Plan.for_problem(ctx, r.problem, r.precision)
        out.append(plan.solve(torch.from_numpy(r.problem.flat_source()).cuda()).cpu().numpy())
        plan.close()
    return out


def test_batch_equals_alone_bitwise(gpu_ctx):
    import torch
    from paper_2010_13213_amd import lgf
    reqs = inputs.served_stream(10, seed=21, sizes=[16, 24, 40, 64, 96])
    alone = _alone(gpu_ctx, reqs)
    plans = [lgf.Plan.for_problem(gpu_ctx, r.problem, r.precision) for r in reqs]
    fs = [torch.from_numpy(r.problem.flat_source()).cuda() for r in reqs]
    us = [torch.empty_like(f) for f in fs]
    lgf.solve_batch(gpu_ctx, plans, fs, us)
    torch.cuda.synchronize()
    for a, u in zip(alone, us):
        assert np.array_equal(a, u.cpu().numpy())
    # and the batched results meet the oracle
    for r, u in list(zip(reqs, us))[:4]:
        c = inputs.cell_coords(r.problem.levels[0].blocks, r.problem.nb)
        rng = np.random.default_rng(0)
        idx = rng.choice(len(c), min(400, len(c)), replace=False)
        ref = direct.direct_sum(c, r.problem.flat_source(), c[idx], 1.0)
        tol = 1e-12 if r.precision == "fp64" else 1e-10
        assert rel_l2(u.cpu().numpy()[idx], ref) < tol, r.precision
    for p in plans:
        p.close()


def test_served_stream_results_match_alone(gpu_ctx):
    from paper_2010_13213_amd import serve
    reqs = inputs.served_stream(24, seed=22, sizes=[16, 32, 48, 64])
    alone = _alone(gpu_ctx, reqs)
    cap = serve.serve(gpu_ctx, reqs, None)
    res = serve.serve(gpu_ctx, reqs, 0.8 * cap["requests_per_s"], keep_results=True, max_batch=8)
    assert res["p50_ms"] > 0 and res["p99_ms"] >= res["p50_ms"]
    for a, u in zip(alone, res["u"]):
        assert np.array_equal(a, u)


def test_hbm_budget_refuses_an_oversized_plan():
    import torch
    from paper_2010_13213_amd import lgf
    ctx = lgf.Context(0, hbm_budget_bytes=128 << 20)      # the LGF table alone is ~17 MB
    p = inputs.blob_cube(128, 8, np.random.default_rng(0))
    with pytest.raises(lgf.LgfError) as e:
        lgf.Plan.for_problem(ctx, p)
    assert e.value.status == lgf.LGF_E_NOMEM
    small = lgf.Plan.for_problem(ctx, inputs.blob_cube(16, 8, np.random.default_rng(1)))
    small.close()
    ctx.close()
    torch.cuda.synchronize()
