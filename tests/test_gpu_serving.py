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


def _two_level_small(nc, seed):
    rng = np.random.default_rng(seed)
    b0 = np.array([(x, y, z) for z in range(3) for y in range(3) for x in range(3)], dtype=np.int32)
    b1 = np.array([(2, 2, 2), (3, 2, 2), (2, 3, 3)], dtype=np.int32)
    return inputs.Problem(nb=8, dx0=0.5, levels=[
        inputs.Level(blocks=b0, values=rng.standard_normal((nc, len(b0), 8, 8, 8))),
        inputs.Level(blocks=b1, values=rng.standard_normal((nc, len(b1), 8, 8, 8)))])


def test_composite_batch_equals_alone_bitwise(gpu_ctx):
    """Composite plans of 2 and 3 levels (FP64 and FP32+refine, 2 and 4
    components) batched level by level with a single-level plan: each result
    equals its lgf_solve, bit for bit, and the three-level ones meet the
    stored oracle samples."""
    import os
    import torch
    from paper_2010_13213_amd import lgf
    rings = inputs.colliding_rings(nb=8, dx0=1.0 / 8, components=(0, 2))
    cases = [(rings, "fp64"), (_two_level_small(4, 3), "fp32_refine"), (rings, "fp32_refine"),
             (inputs.gaussian_box(), "fp64"), (_two_level_small(1, 4), "fp64")]
    plans = [lgf.Plan.for_problem(gpu_ctx, p, prec) for p, prec in cases]
    fs = [torch.from_numpy(p.flat_source()).cuda() for p, _ in cases]
    alone = [pl.solve(f).cpu().numpy() for pl, f in zip(plans, fs)]
    us = [torch.full_like(f, float("nan")) for f in fs]
    print("batch: 3-level rings fp64/fp32_refine, 2-level 4 comps, single level", flush=True)
    lgf.solve_batch(gpu_ctx, plans, fs, us)
    torch.cuda.synchronize()
    for (p, prec), a, u in zip(cases, alone, us):
        assert np.array_equal(a, u.cpu().numpy()), (p.name, prec)
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "colliding_rings_quarter_samples.npz"))
    for i, tol in ((0, 1e-12), (2, 1e-10)):
        got = us[i].cpu().numpy().reshape(2, -1)
        base = 0
        for k, lv in enumerate(rings.levels):
            n = len(lv.blocks) * rings.nb ** 3
            for c in range(2):
                idx = gold["sample%d" % k]
                assert rel_l2(got[c][base:base + n][idx], gold["phi%d_c%d" % (k, c)]) < tol, (i, k, c)
            base += n
    for pl in plans:
        pl.close()


def _cube_req(L, seed, precision="fp64", rid=0):
    p = inputs.blob_cube(L, 8, np.random.default_rng(seed))
    return inputs.Request(rid=rid, problem=p, precision=precision, arrival=0.0)


def test_plans_of_equal_block_count_and_other_shape_are_not_shared(gpu_ctx):
    """2x4x1 and 8x1x1 blocks (8 each) in one served stream: each result
    meets the oracle (a pool keyed by block count would hand one the
    other's plan)."""
    from paper_2010_13213_amd import serve
    rng = np.random.default_rng(9)
    reqs = []
    for i, blocks in enumerate([[(x, y, 0) for y in range(4) for x in range(2)], [(x, 0, 0) for x in range(8)]] * 2):
        b = np.array(blocks, dtype=np.int32)
        p = inputs.Problem(nb=8, dx0=1.0, levels=[inputs.Level(blocks=b, values=rng.standard_normal((1, 8, 8, 8, 8)))])
        reqs.append(inputs.Request(rid=i, problem=p, precision="fp64", arrival=0.0))
    res = serve.serve(gpu_ctx, reqs, None, keep_results=True, max_batch=1, n_streams=1)
    assert res["plans_created"] == 2
    for r, u in zip(reqs, res["u"]):
        c = inputs.cell_coords(r.problem.levels[0].blocks, 8)
        ref = direct.direct_sum(c, r.problem.flat_source(), c, 1.0)
        assert rel_l2(u, ref) < 1e-12


def test_request_waits_for_memory_and_the_budget_holds():
    """A context budget that holds the table, the spectra and one large plan
    but not two: the second shape waits until the first completes and its
    idle plan is freed; the context never exceeds the budget, and every
    result equals the request solved alone."""
    import torch
    from paper_2010_13213_amd import lgf, serve
    big, other = _cube_req(104, 1), _cube_req(96, 2)
    probe = lgf.Context(0)
    alone = {}
    ws = []
    for r in (big, other):
        pl = lgf.Plan.for_problem(probe, r.problem, r.precision)
        ws.append(pl.workspace_bytes())
        alone[r.problem.name] = pl.solve(torch.from_numpy(r.problem.flat_source()).cuda()).cpu().numpy()
        pl.close()
    base = probe.bytes()                       # table and spectra, no plan
    probe.close()
    budget = base + max(ws) + min(ws) // 2
    ctx = lgf.Context(0, hbm_budget_bytes=budget)
    reqs = [_cube_req(104, 1, rid=0), _cube_req(96, 2, rid=1), _cube_req(104, 1, rid=2), _cube_req(96, 2, rid=3)]
    print("serving 4 requests under a budget of %d bytes (base %d, plans %s)" % (budget, base, ws), flush=True)
    res = serve.serve(ctx, reqs, None, keep_results=True)
    assert res["deferred"] > 0 and res["plans_evicted"] > 0
    assert res["peak_context_bytes"] <= budget
    for r, u in zip(reqs, res["u"]):
        assert np.array_equal(u, alone[r.problem.name])
    ctx.close()
    torch.cuda.synchronize()
