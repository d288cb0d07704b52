"""lgf_solve_scratch (the entry point for callers that cannot allocate)
against lgf_solve on the same plans: bit for bit, and against the oracle.

Two calls in a row share the library's static scratch; the second is
smaller, so stale contents of the first must not leak into it."""
import numpy as np
import pytest

from oracle import direct
from paper_2010_13213_amd import inputs, lgf
from helpers import rel_l2

pytestmark = pytest.mark.gpu


def _pair(ctx, prob, precision="fp64"):
    import torch
    plan = lgf.Plan.for_problem(ctx, prob, precision)
    f = torch.from_numpy(prob.flat_source()).cuda()
    ref = plan.solve(f)
    got = torch.full_like(f, float("nan"))
    return plan, f, ref, got


def _oracle(prob):
    c = inputs.cell_coords(prob.levels[0].blocks, prob.nb)
    return direct.direct_sum(c, prob.levels[0].values[0].reshape(-1), c, prob.dx0)


def test_scratch_solve_equals_solve_two_calls_second_smaller(gpu_ctx):
    import torch
    big, small = inputs.gaussian_box(n_blk=4, nb=8), inputs.gaussian_box(n_blk=2, nb=8, seed=2)
    pb, fb, rb, gb = _pair(gpu_ctx, big)
    ps, fs, rs, gs = _pair(gpu_ctx, small)
    print("scratch: 32^3 then 16^3 Gaussian boxes", flush=True)
    pb.solve_scratch(fb, gb)
    ps.solve_scratch(fs, gs)
    torch.cuda.synchronize()
    for prob, got, ref in ((big, gb, rb), (small, gs, rs)):
        g, r = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(g, r)
        assert rel_l2(g, _oracle(prob)) < 1e-12
    pb.close()
    ps.close()


def test_scratch_solve_refined_vector_and_composite(gpu_ctx):
    import torch
    vec = inputs.gaussian_box(n_blk=2, nb=8)
    vals = vec.levels[0].values
    vec.levels[0].values = np.concatenate([vals, 0.5 * vals[:, ::-1], -vals], axis=0)   # 3 components
    two = inputs.Problem(nb=8, dx0=1.0, levels=[
        inputs.Level(blocks=np.array([(x, y, z) for z in range(3) for y in range(3) for x in range(3)], dtype=np.int32),
                     values=np.random.default_rng(7).standard_normal((1, 27, 8, 8, 8))),
        inputs.Level(blocks=np.array([(2, 2, 2), (3, 2, 2)], dtype=np.int32),
                     values=np.random.default_rng(8).standard_normal((1, 2, 8, 8, 8)))])
    cases = [(vec, "fp32_refine"), (two, "fp64"), (vec, "fp64")]
    made = [_pair(gpu_ctx, p, prec) for p, prec in cases]
    print("scratch: refined vector, two-level composite, plain vector", flush=True)
    for plan, f, ref, got in made:
        plan.solve_scratch(f, got)
    torch.cuda.synchronize()
    for plan, f, ref, got in made:
        assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy())
        plan.close()


def test_scratch_solve_refuses_plans_beyond_the_array(gpu_ctx):
    import torch
    ring = inputs.single_ring(components=(0,))          # 208 blocks of 16^3 in a 8^3-block box
    plan = lgf.Plan.for_problem(gpu_ctx, ring)
    f = torch.from_numpy(ring.flat_source()).cuda()
    u = torch.zeros_like(f)
    with pytest.raises(lgf.LgfError) as e:
        plan.solve_scratch(f, u)
    assert e.value.status == lgf.LGF_E_INVALID and "static scratch" in str(e.value)
    assert float(u.abs().max()) == 0.0
    plan.close()
