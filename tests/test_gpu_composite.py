"""GPU parity of the composite-grid (multi-level) LGF solve vs the oracle.

The oracle (oracle/composite.py) follows the FLGF-AMR recursion of the
paper's Sec. 3.4 step by step with direct sums; the GPU runs the same steps
with blockwise FFT convolutions.  Tolerance: relative L2 <= 1e-12 per level
on the float64 path.
"""
import numpy as np
import pytest

from oracle import composite as C, direct
from paper_2010_13213_amd import inputs
from helpers import rel_l2

pytestmark = pytest.mark.gpu
TOL64 = 1e-12


def _cube(n, lo=(0, 0, 0)):
    return np.array([(lo[0] + x, lo[1] + y, lo[2] + z) for z in range(n) for y in range(n)
                     for x in range(n)])


def _gpu(ctx, nb, dx0, blocks, fields, ne=0):
    """fields: list (per level) of (n_comp, n_cells) arrays; returns same shape."""
    import torch
    from paper_2010_13213_amd import lgf
    nc = fields[0].shape[0]
    plan = lgf.Plan(ctx, blocks, nb, dx0, nc, "fp64", ne)
    flat = np.concatenate([np.concatenate([fl[c] for fl in fields]) for c in range(nc)])
    u = plan.solve(torch.from_numpy(flat).cuda()).cpu().numpy().reshape(nc, -1)
    plan.close()
    out, base = [], 0
    for fl in fields:
        n = fl.shape[1]
        out.append(u[:, base:base + n])
        base += n
    return out


def _gauss(cells, dx, ctr, w):
    p = (cells + 0.5) * dx
    return np.exp(-((p - ctr) ** 2).sum(axis=1) / (2 * w * w))


def test_two_level_full_parity(gpu_ctx):
    nb = 8
    blocks = [_cube(4), _cube(4, lo=(2, 2, 2))]
    orc = C.CompositeOracle(nb, 1.0, blocks)
    ctr = np.array([15.0, 17.0, 16.0])
    f = [_gauss(orc.cells[k], orc.dx[k], ctr, 4.0) for k in range(2)]
    ref = orc.solve(f)
    got = _gpu(gpu_ctx, nb, 1.0, blocks, [fk[None] for fk in f])
    for k in range(2):
        m = orc.mask[k]
        assert rel_l2(got[k][0][m], ref[k][m]) < TOL64, k
        assert np.all(got[k][0][~m] == 0.0)


def test_three_level_vector_full_parity(gpu_ctx):
    nb = 8
    blocks = [_cube(3, lo=(-1, -1, -1)), _cube(2, lo=(-1, -1, -1)), _cube(2, lo=(-1, -2, -1))]
    orc = C.CompositeOracle(nb, 0.8, blocks)
    rng = np.random.default_rng(2)
    f = [np.stack([_gauss(orc.cells[k], orc.dx[k], np.array([-0.5, -0.3, 0.2]) + 0.3 * c, 2.5)
                   + 0.01 * rng.standard_normal(len(orc.cells[k])) for c in range(3)])
         for k in range(3)]
    got = _gpu(gpu_ctx, nb, 0.8, blocks, f)
    for c in range(3):
        ref = orc.solve([f[k][c] for k in range(3)])
        for k in range(3):
            m = orc.mask[k]
            assert rel_l2(got[k][c][m], ref[k][m]) < TOL64, (c, k)


def _bump(cells, ctr, R):
    t2 = (((cells + 0.5) - ctr) ** 2).sum(axis=1) / (R * R)
    out = np.zeros(len(cells))
    m = t2 < 1
    out[m] = np.exp(-10.0 / (1.0 - t2[m])) * 1e3
    return out


def test_two_level_compact_potential_is_exact_with_wide_extension(gpu_ctx):
    """f^_0 = L_0 Psi, compact Psi: phi_0 = Psi and phi_1 = L_1^-1 P f^_0."""
    nb = 8
    blocks = [_cube(4), _cube(2, lo=(2, 2, 2))]
    orc = C.CompositeOracle(nb, 1.0, blocks, ext_layers=3)
    ctr, rad = np.array([22.0, 22.0, 22.0]), 4.5
    box = C.Box(np.array([-2, -2, -2]), np.array([34, 34, 34]))
    psi = _bump(box.cells(), ctr, rad).reshape(box.shape)
    lap = C.laplacian7(psi, 1.0)
    i, j, k = box.idx(orc.cells[0])
    f0 = lap[i, j, k]
    f1 = np.zeros(len(orc.cells[1]))
    got = _gpu(gpu_ctx, nb, 1.0, blocks, [f0[None], f1[None]], ne=3)
    m0 = orc.mask[0]
    ref0 = _bump(orc.cells[0][m0], ctr, rad)
    assert np.abs(got[0][0][m0] - ref0).max() < 1e-13 * np.abs(ref0).max()
    ref = orc.solve([f0, f1])
    scale = np.abs(ref0).max()
    assert np.abs(got[1][0] - ref[1]).max() < 1e-14 * scale


def test_half_resolution_two_level_ring_parity(gpu_ctx):
    """The two-level perturbed-ring geometry at half resolution (8^3 blocks,
    coarse R/16 within 8 sigma, fine R/32 within 3 sigma of the perturbed
    core), oracle on sampled targets of both levels."""
    p = inputs.two_level_ring(nb=8, dx0=1.0 / 16, components=(0,))
    blocks = [lv.blocks for lv in p.levels]
    orc = C.CompositeOracle(8, p.dx0, blocks)
    f = [lv.values[0].reshape(-1) for lv in p.levels]
    rng = np.random.default_rng(9)
    sample = [rng.choice(np.nonzero(orc.mask[k])[0], 1500, replace=False) for k in range(2)]
    ref = orc.solve(f, sample=sample)
    got = _gpu(gpu_ctx, 8, p.dx0, blocks, [fk[None] for fk in f])
    for k in range(2):
        assert rel_l2(got[k][0][sample[k]], ref[k][sample[k]]) < TOL64, k


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_refine", 1e-10)])
def test_full_size_two_level_ring_against_stored_oracle(gpu_ctx, precision, tol):
    """Coarse R/32 ring support (208 blocks of 16^3) plus R/64 blocks within
    3 sigma of the perturbed core (320 blocks); omega_x and omega_y.  The
    expected values on 600 sampled cells per level were written by
    tests/golden/make_two_level_ring.py, which calls only the oracle."""
    import os
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "two_level_ring_samples.npz"))
    p = inputs.two_level_ring(components=(0, 1))
    assert len(p.levels[0].blocks) == int(gold["n_blocks0"])
    assert len(p.levels[1].blocks) == int(gold["n_blocks1"])
    fields = [lv.values.reshape(2, -1) for lv in p.levels]
    got = _gpu(gpu_ctx, p.nb, p.dx0, [lv.blocks for lv in p.levels], fields) if precision == "fp64" \
        else _gpu_prec(gpu_ctx, p, precision)
    for c in range(2):
        for k in range(2):
            idx = gold["sample%d" % k]
            assert rel_l2(got[k][c][idx], gold["phi%d_c%d" % (k, c)]) < tol, (c, k)


def _gpu_prec(ctx, p, precision):
    import torch
    from paper_2010_13213_amd import lgf
    plan = lgf.Plan.for_problem(ctx, p, precision)
    u = plan.solve(torch.from_numpy(p.flat_source()).cuda()).cpu().numpy().reshape(p.n_components, -1)
    plan.close()
    n0 = len(p.levels[0].blocks) * p.nb ** 3
    return [u[:, :n0], u[:, n0:]]
