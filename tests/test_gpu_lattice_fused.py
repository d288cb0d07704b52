"""The lattice MAC in one pass per block frequency (lengths 32 x 32 x 32).

Where every lattice DFT length of a convolution is 32 (boxes of 9 to 16
blocks along each axis), the one-pass split (lgf_context_set_lattice_passes
1) does the x DFTs, the y/z slabs and the inverse x DFTs of one frequency in
one workgroup, and hands the terms of the even and the odd lattice x
frequencies to the inverse block FFT, which adds them.  These tests compare it with the three-pass split
(the same sum, rounding apart) on dense, sparse, vector and mixed-precision
solves, with the oracle's direct sum on sampled targets, check which
kernels ran, and that a batch equals its requests alone bit for bit.
"""
import numpy as np
import pytest

from oracle import direct
from paper_2010_13213_amd import inputs
from helpers import gpu_solve, rel_l2

pytestmark = pytest.mark.gpu


def _ctx(passes):
    from paper_2010_13213_amd import lgf
    ctx = lgf.Context(0)
    ctx.set_mac_method("lattice")
    ctx.set_lattice_passes(passes)
    return ctx


@pytest.fixture(scope="module")
def ctx1():
    import torch
    ctx = _ctx(1)
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


@pytest.fixture(scope="module")
def ctx3():
    import torch
    ctx = _ctx(3)
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


def _box(ex, ey, ez, lo=(0, 0, 0)):
    return np.array([(lo[0] + x, lo[1] + y, lo[2] + z) for z in range(ez) for y in range(ey) for x in range(ex)],
                    dtype=np.int32)


def _problem(ext, nb, n_comp, keep, seed, dx=0.5):
    rng = np.random.default_rng(seed)
    blocks = _box(*ext, lo=(2, -4, 7))
    if keep < 1.0:
        blocks = blocks[rng.random(len(blocks)) < keep]
    vals = rng.standard_normal((n_comp, len(blocks), nb, nb, nb))
    return inputs.Problem(nb=nb, dx0=dx, levels=[inputs.Level(blocks=blocks, values=vals)], name="fused")


def _stages(ctx, prob, precision):
    ctx.set_timing(True)
    ctx.stage_times()
    u = gpu_solve(ctx, prob, precision)
    st = ctx.stage_times()
    ctx.set_timing(False)
    return u, st


CASES = [((16, 16, 16), 16, 1, 1.0, "fp64", 1e-13),     # the dense 256^3 box
         ((9, 13, 11), 8, 3, 0.6, "fp64", 1e-13),       # ragged extents, empty slots, three components
         ((12, 10, 16), 16, 2, 1.0, "fp32_refine", 1e-11),
         ((16, 9, 14), 8, 1, 0.3, "fp32_refine", 1e-11)]


@pytest.mark.parametrize("ext,nb,n_comp,keep,precision,tol", CASES)
def test_one_pass_matches_three_passes(ctx1, ctx3, ext, nb, n_comp, keep, precision, tol):
    prob = _problem(ext, nb, n_comp, keep, seed=sum(ext) + nb)
    print("case", ext, nb, n_comp, keep, precision, flush=True)
    u1, st1 = _stages(ctx1, prob, precision)
    u3, st3 = _stages(ctx3, prob, precision)
    assert st1["lat_fused"][1] > 0 and st1["lat_x"][1] == 0 and st1["lat_yz"][1] == 0, st1
    assert st3["lat_fused"][1] == 0 and st3["lat_yz"][1] > 0, st3
    for c in range(n_comp):
        assert rel_l2(u1[c], u3[c]) < tol, (c, rel_l2(u1[c], u3[c]))


@pytest.mark.parametrize("ext,nb,keep", [((10, 9, 12), 8, 0.4), ((16, 16, 9), 8, 1.0)])
def test_one_pass_vs_oracle_sampled(ctx1, ext, nb, keep):
    """FP64 against the direct sum on 1500 sampled targets, a third of them
    on block faces (where the block FFT's zero padding and the lattice
    offsets meet)."""
    prob = _problem(ext, nb, 1, keep, seed=3 * sum(ext))
    print("case", ext, nb, keep, flush=True)
    u = gpu_solve(ctx1, prob)[0]
    c = inputs.cell_coords(prob.levels[0].blocks, nb)
    f = prob.flat_source()
    rng = np.random.default_rng(11)
    local = c % nb
    face = np.nonzero(((local == 0) | (local == nb - 1)).any(1))[0]
    idx = np.concatenate([rng.choice(face, 500, replace=False), rng.choice(len(c), 1000, replace=False)])
    ref = direct.direct_sum(c, f, c[idx], prob.dx0)
    err = rel_l2(u[idx], ref)
    print("rel L2 vs oracle", err, flush=True)
    assert err < 1e-12


def test_one_pass_batch_equals_alone(ctx1):
    import torch
    from paper_2010_13213_amd import lgf
    probs = [_problem((16, 12, 10), 8, 1, 1.0, seed=5), _problem((9, 16, 16), 8, 2, 0.5, seed=6)]
    alone = [gpu_solve(ctx1, p) for p in probs]
    plans = [lgf.Plan.for_problem(ctx1, p) for p in probs]
    fs = [torch.from_numpy(p.flat_source()).cuda() for p in probs]
    us = [torch.empty_like(f) for f in fs]
    lgf.solve_batch(ctx1, plans, fs, us)
    torch.cuda.synchronize()
    for p, a, u in zip(probs, alone, us):
        got = u.cpu().numpy().reshape(p.n_components, -1)
        assert np.array_equal(got, a)
    for pl in plans:
        pl.close()
