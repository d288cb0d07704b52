"""Three-level colliding-ring workload on the GPU.

* Quarter-size geometry (R/8, R/16, R/32 with 8^3 blocks): sampled values of
  every level against the composite oracle, stored by
  tests/golden/make_colliding_rings_quarter.py (calls only oracle/).
* Full size (R/32, R/64, R/128 with 16^3 blocks, 992 / 2137 / 4776 blocks):
  a manufactured source on the finest level only, f_2 = L_2 Psi with a
  compact Psi.  The recursion of the paper's Sec. 3.4 then gives exactly
  psi_0 = psi_1 = 0, S = 0, phi_2 = Psi on the finest level, and
  phi_k = L_k^-1 F_k (F_k the mean-8 coarsening of f_2) on the coarser
  levels, which the oracle evaluates by direct sums over the small support.
  F_k is the coarsened Laplacian of a compact function: its mass and low
  moments cancel, so phi_k on the coarse levels is about 1e-6 of the sum
  sum |G| |F_k| that both sides round against.  The coarse check therefore
  bounds the error by tol times that conditioning scale, not by tol times
  the (cancelled) values.
"""
import os

import numpy as np
import pytest

from oracle import composite as C, direct
from paper_2010_13213_amd import inputs
from helpers import rel_l2

pytestmark = pytest.mark.gpu


def _solve(ctx, p, precision, fields):
    import torch
    from paper_2010_13213_amd import lgf
    plan = lgf.Plan(ctx, [lv.blocks for lv in p.levels], p.nb, p.dx0, len(fields[0]), precision)
    flat = np.concatenate([np.concatenate([fk[c] for fk in fields]) for c in range(len(fields[0]))])
    u = plan.solve(torch.from_numpy(flat).cuda()).cpu().numpy().reshape(len(fields[0]), -1)
    plan.close()
    out, base = [], 0
    for lv in p.levels:
        n = len(lv.blocks) * p.nb ** 3
        out.append(u[:, base:base + n])
        base += n
    return out


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_refine", 1e-10)])
def test_quarter_size_colliding_rings_against_stored_oracle(gpu_ctx, precision, tol):
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "colliding_rings_quarter_samples.npz"))
    p = inputs.colliding_rings(nb=8, dx0=1.0 / 8, components=(0, 2))
    assert [len(lv.blocks) for lv in p.levels] == list(gold["n_blocks"])
    fields = [lv.values.reshape(2, -1) for lv in p.levels]
    got = _solve(gpu_ctx, p, precision, fields)
    for c in range(2):
        for k in range(3):
            idx = gold["sample%d" % k]
            assert rel_l2(got[k][c][idx], gold["phi%d_c%d" % (k, c)]) < tol, (c, k)


def _bump(cells, ctr, R):
    t2 = (((cells + 0.5) - ctr) ** 2).sum(axis=1) / (R * R)
    out = np.zeros(len(cells))
    m = t2 < 1
    out[m] = np.exp(-10.0 / (1.0 - t2[m]))
    return out


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_refine", 1e-10)])
def test_full_size_colliding_rings_finest_manufactured_source(gpu_ctx, precision, tol):
    p = inputs.colliding_rings(nb=16, dx0=1.0 / 32, components=(), with_values=False)
    nb = p.nb
    blocks = [lv.blocks for lv in p.levels]
    dx = [p.dx0 / 2 ** k for k in range(3)]
    # a fine block whose 26 neighbours are all fine blocks: Psi lives inside
    fine = {tuple(b) for b in blocks[2].tolist()}
    inner = [b for b in blocks[2].tolist()
             if all((b[0] + i, b[1] + j, b[2] + k) in fine
                    for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1))]
    b0 = np.array(inner[len(inner) // 2])
    ctr = (b0 + 0.5) * nb
    cells2 = C.block_cells(blocks[2], nb)
    box = C.Box(b0 * nb - 12, b0 * nb + nb + 12)
    psi_box = _bump(box.cells(), ctr, 9.5).reshape(box.shape)
    lap_box = C.laplacian7(psi_box, dx[2])
    near = np.all((cells2 >= box.lo) & (cells2 < box.hi), axis=1)
    f2 = np.zeros(len(cells2))
    i, j, k = box.idx(cells2[near])
    f2[near] = lap_box[i, j, k]
    fields = [np.zeros((1, len(b) * nb ** 3)) for b in blocks[:2]] + [f2[None]]
    got = _solve(gpu_ctx, p, precision, fields)
    # finest level: phi_2 = Psi
    psi2 = np.zeros(len(cells2))
    psi2[near] = psi_box[i, j, k]
    assert np.abs(got[2][0] - psi2).max() < tol * np.abs(psi2).max()
    # coarser levels: phi_k = L_k^-1 F_k on sampled Omega_k cells, with F_k
    # the mean-8 coarsening of the finer cumulative source (oracle steps)
    Fb, F_fine = box, lap_box
    rng = np.random.default_rng(3)
    for kk in (1, 0):
        cb = C.Box(np.floor_divide(Fb.lo, 2), np.floor_divide(Fb.hi + 1, 2))
        pad = C.Box(2 * cb.lo, 2 * cb.lo + 2 * np.array(cb.shape))
        arr = pad.zeros()
        o = Fb.lo - pad.lo
        arr[o[0]:o[0] + Fb.shape[0], o[1]:o[1] + Fb.shape[1], o[2]:o[2] + Fb.shape[2]] = F_fine
        cc = cb.cells()
        F_c = C.coarsen_mean8(pad, arr, cc)
        cells_k = C.block_cells(blocks[kk], nb)
        covered = {tuple(b) for b in blocks[kk + 1].tolist()}
        cand = np.arange(0, len(cells_k), 97)
        keep = np.array([tuple(int(v) for v in np.floor_divide(2 * c, nb)) not in covered for c in cells_k[cand]])
        tgt_idx = rng.choice(cand[keep], min(400, int(keep.sum())), replace=False)
        nz = F_c != 0
        ref = direct.direct_sum(cc[nz], F_c[nz], cells_k[tgt_idx], dx[kk])
        scale = -direct.direct_sum(cc[nz], np.abs(F_c[nz]), cells_k[tgt_idx], dx[kk])
        assert np.abs(got[kk][0][tgt_idx] - ref).max() < tol * scale.max(), kk
        Fb, F_fine = cb, F_c.reshape(cb.shape)


@pytest.fixture(scope="module")
def full_rings():
    """The full-size colliding rings (992 / 2137 / 4776 blocks of 16^3),
    omega_x and omega_z, with the stored oracle samples."""
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "colliding_rings_full_samples.npz"))
    comps = tuple(int(c) for c in gold["components"])
    print("building the full-size colliding rings (components %s)" % (comps,), flush=True)
    p = inputs.colliding_rings(components=comps)
    assert [len(lv.blocks) for lv in p.levels] == list(gold["n_blocks"])
    return p, gold


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_refine", 1e-10)])
def test_full_size_colliding_rings_ring_source_against_stored_oracle(gpu_ctx, full_rings, precision, tol):
    """The two-ring vorticity on all three levels (R/32, R/64, R/128),
    through the whole Sec. 3.4 recursion, against 2000 oracle samples per
    level and component (written by tests/golden/make_colliding_rings_full.py:
    the oracle's psi fields by its FFT box convolution, the samples by
    direct sums)."""
    p, gold = full_rings
    nc = p.n_components
    fields = [lv.values.reshape(nc, -1) for lv in p.levels]
    print("solving the full-size colliding rings, %s" % precision, flush=True)
    got = _solve(gpu_ctx, p, precision, fields)
    for c in range(nc):
        for k in range(3):
            idx = gold["sample%d" % k]
            e = rel_l2(got[k][c][idx], gold["phi%d_c%d" % (k, c)])
            print("level %d component %d: rel L2 %.3e" % (k, c, e), flush=True)
            assert e < tol, (c, k)
