"""GPU parity of the FP32 + FP64-refinement path (LGF_FP32_REFINE).

Bar: relative L2 <= 1e-10 against the CPU FP64 oracle, for every result.
Spectra, FFTs and products run in float32; the residual, the convolution of
the two-cell cut and the final accumulation in float64 (see
csrc/lgf_refine.hip).
"""
import numpy as np
import pytest

from oracle import composite as C, direct
from paper_2010_13213_amd import inputs
from helpers import gpu_solve, level_cells, rel_l2

pytestmark = pytest.mark.gpu
TOL_MIXED = 1e-10


def _cube(n, lo=(0, 0, 0)):
    return np.array([(lo[0] + x, lo[1] + y, lo[2] + z) for z in range(n) for y in range(n)
                     for x in range(n)])


def test_gaussian_box_32_mixed_full_parity(gpu_ctx):
    p = inputs.gaussian_box()
    (u, rep) = gpu_solve(gpu_ctx, p, "fp32_refine", report=True)
    # float32 solve, float64 cut (one convolution, or two when rows along y
    # for the x faces save work), float32 correction
    assert rep.passes in (3, 4)
    c = level_cells(p)
    ref = direct.direct_sum(c, p.flat_source(), c, p.dx0)
    assert rel_l2(u[0], ref) < TOL_MIXED


def test_dense_64_box_noise_mixed_sampled(gpu_ctx):
    nb = 8
    blocks = _cube(8, lo=(-3, 1, 0))
    rng = np.random.default_rng(12)
    c = inputs.cell_coords(blocks, nb)
    f = rng.standard_normal(len(c)) + np.exp(-(((c - c.mean(0)) / 9.0) ** 2).sum(1))
    p = inputs.Problem(nb=nb, dx0=0.3, levels=[inputs.Level(blocks=blocks.astype(np.int32),
                                                            values=f.reshape(1, len(blocks), nb, nb, nb))])
    u = gpu_solve(gpu_ctx, p, "fp32_refine")[0]
    idx = rng.choice(len(c), 2000, replace=False)
    ref = direct.direct_sum(c, f, c[idx], 0.3)
    assert rel_l2(u[idx], ref) < TOL_MIXED


def test_vortex_ring_vector_mixed_sampled(gpu_ctx):
    p = inputs.single_ring(components=(0, 1))
    u = gpu_solve(gpu_ctx, p, "fp32_refine")
    rng = np.random.default_rng(13)
    c = level_cells(p)
    idx = rng.choice(len(c), 1000, replace=False)
    for comp in range(2):
        f = p.levels[0].values[comp].reshape(-1)
        ref = direct.direct_sum(c, f, c[idx], p.dx0)
        assert rel_l2(u[comp][idx], ref) < TOL_MIXED


def test_dense_256_box_mixed_sampled(gpu_ctx):
    p = inputs.mstar()
    u = gpu_solve(gpu_ctx, p, "fp32_refine")[0]
    rng = np.random.default_rng(14)
    c = level_cells(p)
    idx = rng.choice(len(c), 200, replace=False)
    f = p.levels[0].values[0].reshape(-1)
    ref = direct.direct_sum(c, f, c[idx], p.dx0)
    assert rel_l2(u[idx], ref) < TOL_MIXED


def test_two_level_mixed_full_parity(gpu_ctx):
    import torch
    from paper_2010_13213_amd import lgf
    nb = 8
    blocks = [_cube(5), _cube(4, lo=(3, 3, 3))]
    orc = C.CompositeOracle(nb, 1.0, blocks)
    ctr = np.array([20.0, 19.0, 21.0])
    f = [np.exp(-(((orc.cells[k] + 0.5) * orc.dx[k] - ctr) ** 2).sum(1) / 18.0) for k in range(2)]
    ref = orc.solve(f)
    plan = lgf.Plan(gpu_ctx, blocks, nb, 1.0, 1, "fp32_refine")
    u = plan.solve(torch.from_numpy(np.concatenate(f)).cuda()).cpu().numpy()
    plan.close()
    n0 = len(orc.cells[0])
    for k, part in enumerate([u[:n0], u[n0:]]):
        m = orc.mask[k]
        assert rel_l2(part[m], ref[k][m]) < TOL_MIXED, k


def _fft_oracle(p, comp):
    from oracle import box
    c = level_cells(p)
    return box.convolve_cells(c, p.levels[0].values[comp].reshape(-1), c, p.dx0)


def test_dense_256_box_mixed_full_parity(gpu_ctx):
    """Every cell of the 256^3 box: the refinement acts next to the box
    surface, so a uniform sample sees it rarely; the whole field does."""
    p = inputs.mstar()
    u = gpu_solve(gpu_ctx, p, "fp32_refine")[0]
    ref = _fft_oracle(p, 0)
    assert rel_l2(u, ref) < TOL_MIXED
    c = level_cells(p)
    depth = np.minimum(c.min(axis=1) - c.min(), (c.max() - c).min(axis=1))
    shell = depth <= 2                                   # within two cells of the box surface
    assert rel_l2(u[shell], ref[shell]) < TOL_MIXED


def test_vortex_ring_mixed_full_parity(gpu_ctx):
    """Config 2 under the mixed path: all cells of both nonzero components."""
    p = inputs.single_ring(components=(0, 1))
    u = gpu_solve(gpu_ctx, p, "fp32_refine")
    for comp in range(2):
        assert rel_l2(u[comp], _fft_oracle(p, comp)) < TOL_MIXED, comp
