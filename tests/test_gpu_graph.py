"""lgf_graph_create / lgf_graph_launch: one solve captured as a HIP graph.

Every replay must equal the eager lgf_solve result bit for bit (the graph
holds the same launches in the same order).  Between replays the program
runs its own eager work (solves of the same plan into other buffers, torch
fills) and synchronises, and each replay is checked on its own.  The
inputs are refreshed in place between replays, which the graph must see.
"""
import numpy as np
import pytest

from paper_2010_13213_amd import inputs

pytestmark = pytest.mark.gpu


def _cube(n, lo=(0, 0, 0)):
    return np.array([(lo[0] + x, lo[1] + y, lo[2] + z) for z in range(n) for y in range(n)
                     for x in range(n)], dtype=np.int32)


def _two_level():
    nb = 8
    blocks = [_cube(4), _cube(2, lo=(1, 1, 1))]
    rng = np.random.default_rng(21)
    levels = [inputs.Level(blocks=b, values=rng.standard_normal((2, len(b), nb, nb, nb))) for b in blocks]
    return inputs.Problem(nb=nb, dx0=0.5, levels=levels, name="two-level cubes")


@pytest.mark.parametrize("case,precision", [("box", "fp64"), ("box", "fp32_refine"),
                                            ("two_level", "fp64"), ("two_level", "fp32_refine")])
def test_graph_replays_equal_eager_solves(gpu_ctx, case, precision):
    import torch
    from paper_2010_13213_amd import lgf
    p = inputs.gaussian_box() if case == "box" else _two_level()
    plan = lgf.Plan.for_problem(gpu_ctx, p, precision)
    f0 = torch.from_numpy(p.flat_source()).cuda()
    f1 = torch.flip(f0, dims=[0]).contiguous() * 0.5
    ref0 = plan.solve(f0)
    ref1 = plan.solve(f1)
    torch.cuda.synchronize()
    assert not torch.equal(ref0, ref1)

    f = f0.clone()
    u = torch.empty_like(f0)
    g = lgf.Graph(plan, f, u)
    scratch = torch.empty_like(f0)
    for rep, (src, ref) in enumerate([(f0, ref0), (f1, ref1), (f0, ref0), (f1, ref1)]):
        f.copy_(src)                       # refresh the bound input in place
        u.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(u, ref), (case, precision, rep)
        # eager work of the program between replays, on the same plan
        plan.solve(f1 if rep % 2 == 0 else f0, scratch)
        torch.cuda.synchronize()
        assert torch.equal(scratch, ref1 if rep % 2 == 0 else ref0)
    g.close()
    # eager solves after the graph is gone still agree
    assert torch.equal(plan.solve(f0), ref0)
    plan.close()


def test_batch_graph_replays_equal_eager_batches(gpu_ctx):
    """lgf_graph_create_batch: one graph holds a whole batch -- single-level
    FP64 and FP32+refine, a composite FP64 and a composite FP32+refine plan,
    an integrating-factor plan.  Each replay (inputs refreshed in place,
    eager batches of the same plans between replays) equals the eager
    lgf_solve_batch bit for bit."""
    import torch
    from paper_2010_13213_amd import lgf
    reqs = inputs.served_stream(4, seed=31, sizes=[16, 24, 40])
    cases = [(r.problem, r.precision, None) for r in reqs] + \
            [(_two_level(), "fp64", None), (_two_level(), "fp32_refine", None), (_two_level(), "fp64", 0.7)]
    plans = [lgf.Plan.for_problem(gpu_ctx, p, prec, if_a0=a) for p, prec, a in cases]
    f0 = [torch.from_numpy(p.flat_source()).cuda() for p, _, _ in cases]
    f1 = [torch.flip(f, dims=[0]).contiguous() * -0.25 for f in f0]
    refs = []
    for src in (f0, f1):
        us = [torch.empty_like(f) for f in src]
        lgf.solve_batch(gpu_ctx, plans, src, us)
        torch.cuda.synchronize()
        refs.append([u.clone() for u in us])
    fb = [f.clone() for f in f0]
    ub = [torch.empty_like(f) for f in f0]
    print("capturing a batch of %d plans" % len(plans), flush=True)
    g = lgf.BatchGraph(gpu_ctx, plans, fb, ub)
    scratch = [torch.empty_like(f) for f in f0]
    for rep in range(4):
        src, ref = (f0, refs[0]) if rep % 2 == 0 else (f1, refs[1])
        for a, b in zip(fb, src):
            a.copy_(b)
        for u in ub:
            u.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        for i, (u, r) in enumerate(zip(ub, ref)):
            assert torch.equal(u, r), (rep, i)
        lgf.solve_batch(gpu_ctx, plans, f1 if rep % 2 == 0 else f0, scratch)
        torch.cuda.synchronize()
        for u, r in zip(scratch, refs[1] if rep % 2 == 0 else refs[0]):
            assert torch.equal(u, r)
    g.close()
    for p in plans:
        p.close()
