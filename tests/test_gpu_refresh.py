"""Velocity refresh u = -C^dagger L_E^-1 omega on the GPU (paper Sec. 4.1,
eq. vel_update), through lgf_velocity_refresh.

* A compact edge field A gives u = C^dagger A and omega = C u (the
  oracle's curls, pinned on the CPU); the refresh must return u exactly
  (up to rounding) wherever its backward stencil lies in the support, and
  NaN where it does not.
* The thin ring's vorticity: sampled cells against the oracle's refresh
  (direct sums for psi, then the backward curl).
* psi equals lgf_solve of omega bit for bit.
"""
import numpy as np
import pytest

from oracle import refresh
from paper_2010_13213_amd import inputs
from helpers import rel_l2

pytestmark = pytest.mark.gpu


def _box_problem(n_blk, nb, dx, field):
    b = np.array([(x, y, z) for z in range(n_blk) for y in range(n_blk) for x in range(n_blk)], dtype=np.int32)
    c = inputs.cell_coords(b, nb)
    vals = field[:, c[:, 0], c[:, 1], c[:, 2]].reshape(3, len(b), nb, nb, nb)
    return inputs.Problem(nb=nb, dx0=dx, levels=[inputs.Level(blocks=b, values=vals)]), c


def _bump3(shape, ctr, R):
    ax = [np.arange(n) + 0.5 for n in shape]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    out = []
    for c, amp in enumerate((1.0, -0.7, 1.3)):
        cc = np.asarray(ctr, dtype=float) + (c - 1) * 0.8
        t2 = ((X - cc[0]) ** 2 + (Y - cc[1]) ** 2 + (Z - cc[2]) ** 2) / R ** 2
        f = np.zeros(shape)
        m = t2 < 1
        f[m] = amp * np.exp(-4.0 / (1.0 - t2[m]))
        out.append(f)
    return np.stack(out)


def _refresh(ctx, prob):
    import torch
    from paper_2010_13213_amd import lgf
    plan = lgf.Plan.for_problem(ctx, prob)
    w = torch.from_numpy(prob.flat_source()).cuda()
    psi, u = lgf.velocity_refresh(plan, w)
    solo = plan.solve(w)
    torch.cuda.synchronize()
    out = psi.cpu().numpy().reshape(3, -1), u.cpu().numpy().reshape(3, -1), solo.cpu().numpy().reshape(3, -1)
    plan.close()
    return out


def test_refresh_recovers_compact_velocity(gpu_ctx):
    n_blk, nb, dx = 4, 8, 0.25
    L = n_blk * nb
    A = _bump3((L, L, L), (L / 2, L / 2, L / 2), 9.0)
    u_ex = refresh.curl_backward(A, dx)
    w = refresh.curl_forward(u_ex, dx)
    prob, c = _box_problem(n_blk, nb, dx, w)
    print("refresh: compact field on 4^3 blocks of 8^3", flush=True)
    psi, u, solo = _refresh(gpu_ctx, prob)
    assert np.array_equal(psi, solo)
    want = u_ex[:, c[:, 0], c[:, 1], c[:, 2]]
    # u_x needs the cells one back along y and z, u_y along z and x, u_z along x and y
    need = [(1, 2), (2, 0), (0, 1)]
    for comp in range(3):
        inside = np.all(c[:, list(need[comp])] >= 1, axis=1)
        assert np.all(np.isnan(u[comp][~inside]))
        assert np.all(np.isfinite(u[comp][inside]))
        assert np.abs(u[comp][inside] - want[comp][inside]).max() < 1e-12 * np.abs(u_ex).max()


def test_refresh_of_ring_vorticity_against_oracle(gpu_ctx):
    prob = inputs.single_ring()                  # 208 blocks of 16^3 at dx = R/32
    c = inputs.cell_coords(prob.levels[0].blocks, prob.nb)
    print("refresh: ring vorticity, 208 blocks of 16^3", flush=True)
    psi, u, solo = _refresh(gpu_ctx, prob)
    assert np.array_equal(psi, solo)
    blocks = {tuple(b) for b in prob.levels[0].blocks.tolist()}
    back_ok = np.ones(len(c), dtype=bool)
    for a in range(3):
        q = c.copy()
        q[:, a] -= 1
        back_ok &= np.array([tuple(v) in blocks for v in np.floor_divide(q, prob.nb).tolist()])
    idx = np.random.default_rng(5).choice(np.nonzero(back_ok)[0], 300, replace=False)
    w = prob.flat_source().reshape(3, -1)
    ref = refresh.velocity_refresh(c, w, c[idx], prob.dx0)
    for comp in range(3):
        assert rel_l2(u[comp][idx], ref[comp]) < 1e-12, comp
