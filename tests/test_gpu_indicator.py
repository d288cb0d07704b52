"""Refinement indicator and AMR convergence on the GPU (paper Sec. 3.4 test,
Sec. 4.2).

* lgf_solve_indicator's per-block RMS and max of the combined source S_k
  (eq. combined_source) against the composite oracle's, on two- and
  three-level meshes.
* The manufactured ring streamfunction of Sec. 3.4 (c1 = 1e3, c2 = 10,
  R = 0.125) solved on meshes refined by the criterion
  |omega^k| > alpha^(L_R - k) max|omega| (alpha = 1/6) for L_R = 0..3: the
  error on the finest level against the exact Psi falls with every level
  (second order in the finest spacing), as in the paper's convergence
  figure; the indicator flags of eqs. refine1 / refine2 follow from the
  statistics.
"""
import numpy as np
import pytest

from oracle import composite as C
from paper_2010_13213_amd import amr, inputs

pytestmark = pytest.mark.gpu


def _stats_oracle(orc, k, nb):
    cells, vals = orc.combined[k]
    blk = np.floor_divide(cells, nb)
    out = {}
    keys, inv = np.unique(blk, axis=0, return_inverse=True)
    inv = inv.ravel()
    ss = np.bincount(inv, weights=vals * vals, minlength=len(keys))
    mx = np.zeros(len(keys))
    np.maximum.at(mx, inv, np.abs(vals))
    cnt = np.bincount(inv, minlength=len(keys))
    for i, key in enumerate(map(tuple, keys.tolist())):
        out[key] = (np.sqrt(ss[i] / cnt[i]), mx[i])
    return out


def _check_indicator(ctx, prob, fft):
    import torch
    from paper_2010_13213_amd import lgf
    plan = lgf.Plan.for_problem(ctx, prob)
    f = torch.from_numpy(prob.flat_source()).cuda()
    u, rms, mx = plan.solve_indicator(f)
    u_plain = plan.solve(f)
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), u_plain.cpu().numpy())
    blocks = [lv.blocks for lv in prob.levels]
    orc = C.CompositeOracle(prob.nb, prob.dx0, blocks, fft_min_targets=fft)
    for c in range(prob.n_components):
        orc.solve([lv.values[c].reshape(-1) for lv in prob.levels], sample=[np.arange(4)] * len(blocks))
        for k in range(len(blocks)):
            ref = _stats_oracle(orc, k, prob.nb)
            got_b = [tuple(b) for b in plan.source_blocks(k).tolist()]
            assert set(got_b) == set(ref), (c, k)
            r = np.array([ref[b][0] for b in got_b])
            m = np.array([ref[b][1] for b in got_b])
            scale = max(np.abs(r).max(), 1e-300)
            assert np.abs(rms[c][k] - r).max() <= 1e-12 * scale, (c, k)
            assert np.abs(mx[c][k] - m).max() <= 1e-12 * max(np.abs(m).max(), 1e-300), (c, k)
    plan.close()


def test_indicator_statistics_two_levels(gpu_ctx):
    rng = np.random.default_rng(13)
    b0 = np.array([(x, y, z) for z in range(3) for y in range(3) for x in range(3)], dtype=np.int32)
    b1 = np.array([(2, 2, 2), (3, 2, 2), (2, 3, 3)], dtype=np.int32)
    prob = inputs.Problem(nb=8, dx0=0.5, levels=[
        inputs.Level(blocks=b0, values=rng.standard_normal((2, len(b0), 8, 8, 8))),
        inputs.Level(blocks=b1, values=rng.standard_normal((2, len(b1), 8, 8, 8)))])
    print("indicator: two levels, 27 + 3 blocks of 8^3", flush=True)
    _check_indicator(gpu_ctx, prob, None)


def test_indicator_statistics_three_level_rings(gpu_ctx):
    prob = inputs.colliding_rings(nb=8, dx0=1.0 / 8, components=(0,))
    print("indicator: quarter-size colliding rings", flush=True)
    _check_indicator(gpu_ctx, prob, 20000)


def _ring_mesh(n_refine, nb=8):
    dx0 = 0.5 / 32
    base = np.array([(x, y, z) for z in range(-2, 2) for y in range(-2, 2) for x in range(-2, 2)])
    fn = lambda p: np.abs(amr.manufactured_ring(p)[1]).max(axis=0)
    return amr.refine_by_field(fn, nb, dx0, base, n_refine, 1.0 / 6.0), dx0


def test_manufactured_ring_converges_with_refinement_levels(gpu_ctx):
    import torch
    from paper_2010_13213_amd import lgf
    errs = []
    for LR in range(4):
        levels, dx0 = _ring_mesh(LR)
        nb = 8
        vals = []
        for k, b in enumerate(levels):
            p = inputs.cell_centres(b, nb, dx0 / 2 ** k, (0.0, 0.0, 0.0)).reshape(-1, 3)
            vals.append(amr.manufactured_ring(p)[1][:2].reshape(2, len(b), nb, nb, nb))
        prob = inputs.Problem(nb=nb, dx0=dx0, levels=[inputs.Level(blocks=b, values=v) for b, v in zip(levels, vals)])
        plan = lgf.Plan.for_problem(gpu_ctx, prob)
        f = torch.from_numpy(prob.flat_source()).cuda()
        u, rms, mx = plan.solve_indicator(f)
        u = u.cpu().numpy().reshape(2, -1)
        plan.close()
        # finest level against the exact Psi on its Omega (all of it: nothing finer)
        kf = len(levels) - 1
        base = sum(len(b) for b in levels[:kf]) * nb ** 3
        p = inputs.cell_centres(levels[kf], nb, dx0 / 2 ** kf, (0.0, 0.0, 0.0)).reshape(-1, 3)
        psi = amr.manufactured_ring(p)[0][:2]
        err = np.abs(u[:, base:] - psi).max() / np.abs(psi).max()
        errs.append(err)
        # the indicator: the finest level's blocks are where the criterion asks for refinement
        s_max = max(float(r.max()) for r in rms[0])
        flags = amr.indicator_flags(mx[0][kf], kf, len(levels) - 1, s_max, 1.0 / 6.0, 0.75)
        print("L_R = %d: blocks %s, L_inf error on the finest level %.3e, refine/keep/coarsen %s"
              % (LR, [len(b) for b in levels], err, [int((flags == v).sum()) for v in (1, 0, -1)]), flush=True)
    for a, b in zip(errs, errs[1:]):
        assert b < 0.5 * a, errs
    assert errs[-1] < errs[0] / 16, errs
