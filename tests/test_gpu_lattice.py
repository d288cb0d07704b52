"""The spectral MAC as an FFT over the block lattice.

At each block frequency the level convolution is a linear convolution over
the block lattice; zero-padded to a DFT length L >= 2E - 1 per axis it is
computed exactly (up to rounding) by lattice DFTs and a product with real
lattice spectra.  These tests force that method (LGF_MAC_LATTICE) and check
it against the oracle's direct sum (FP64 1e-12, mixed 1e-10) on boxes of
every compiled length, ragged and sparse supports, one-block-thick boxes,
vector and composite solves; against the block-pair method on the dense
256^3 box and on boxes that need the wide lengths (64 along x or y, 128
along z); and the bit-for-bit identities of the product path (vector =
scalar components, batch = alone, graph replay = eager) under it.  A box
longer than 32 blocks along x or y, or 64 along z, falls back to block
pairs.
"""
import numpy as np
import pytest

from oracle import direct
from paper_2010_13213_amd import inputs
from helpers import gpu_solve, level_cells, rel_l2

pytestmark = pytest.mark.gpu

TOL64, TOLMIX = 1e-12, 1e-10


@pytest.fixture(scope="module")
def lat_ctx():
    import torch
    from paper_2010_13213_amd import lgf
    ctx = lgf.Context(0)
    ctx.set_mac_method("lattice")
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


@pytest.fixture(scope="module")
def pairs_ctx():
    import torch
    from paper_2010_13213_amd import lgf
    ctx = lgf.Context(0)
    ctx.set_mac_method("pairs")
    yield ctx
    torch.cuda.synchronize()
    ctx.close()


def _problem(blocks, nb, f, dx=1.0, n_comp=1):
    blocks = np.asarray(blocks, dtype=np.int32)
    vals = np.asarray(f, dtype=np.float64).reshape(n_comp, len(blocks), nb, nb, nb)
    return inputs.Problem(nb=nb, dx0=dx, levels=[inputs.Level(blocks=blocks, values=vals)], name="test")


def _box(ex, ey, ez, lo=(0, 0, 0)):
    return np.array([(lo[0] + x, lo[1] + y, lo[2] + z) for z in range(ez) for y in range(ey) for x in range(ex)],
                    dtype=np.int32)


@pytest.mark.parametrize("ext,nb,dx", [((1, 1, 1), 8, 1.0), ((2, 3, 1), 8, 0.5), ((4, 4, 4), 8, 1.0),
                                       ((5, 7, 3), 8, 0.3), ((16, 2, 2), 8, 1.0), ((3, 2, 9), 16, 0.25)])
def test_lattice_boxes_full_parity(lat_ctx, ext, nb, dx):
    """Every DFT length up to 32 (4, 8, 16, 32) along every axis, ragged
    extents, single blocks and one-block-thick boxes."""
    rng = np.random.default_rng(sum(ext) * 7 + nb)
    blocks = _box(*ext, lo=(-3, 5, 2))
    c = inputs.cell_coords(blocks, nb)
    f = rng.standard_normal(len(c))
    u = gpu_solve(lat_ctx, _problem(blocks, nb, f, dx))[0]
    if len(c) <= 40000:
        ref = direct.direct_sum(c, f, c, dx)
        assert rel_l2(u, ref) < TOL64
    else:
        idx = rng.choice(len(c), 3000, replace=False)
        ref = direct.direct_sum(c, f, c[idx], dx)
        assert rel_l2(u[idx], ref) < TOL64


@pytest.mark.parametrize("ext,nb,precision,tol", [((2, 2, 20), 8, "fp64", TOL64), ((3, 3, 18), 16, "fp64", TOL64),
                                                   ((2, 3, 32), 8, "fp32_refine", TOLMIX),
                                                   ((5, 6, 24), 8, "fp64", TOL64), ((9, 9, 17), 8, "fp64", TOL64)])
def test_lattice_long_z_boxes_sampled(lat_ctx, ext, nb, precision, tol):
    """z extents 17..32 take the z DFT length 64 (x and y stay <= 32), with
    y lengths 4, 8, 16 and 32."""
    rng = np.random.default_rng(sum(ext) * 11 + nb)
    blocks = _box(*ext, lo=(4, -2, -7))
    c = inputs.cell_coords(blocks, nb)
    f = rng.standard_normal(len(c))
    lat_ctx.set_timing(True)
    lat_ctx.stage_times()
    try:
        u = gpu_solve(lat_ctx, _problem(blocks, nb, f, 0.6), precision)[0]
        st = lat_ctx.stage_times()
    finally:
        lat_ctx.set_timing(False)
    # every convolution ran on the lattice, none on block pairs
    assert st["lat_yz"][1] > 0 and st["smac"][1] == 0, st
    idx = np.concatenate([rng.choice(len(c), 1500, replace=False), [0, len(c) - 1]])
    assert rel_l2(u[idx], direct.direct_sum(c, f, c[idx], 0.6)) < tol


def _lattice_stages(ctx, prob, precision="fp64"):
    ctx.set_timing(True)
    ctx.stage_times()
    try:
        u = gpu_solve(ctx, prob, precision)
        st = ctx.stage_times()
    finally:
        ctx.set_timing(False)
    return u, st


@pytest.mark.parametrize("ext,nb,precision,tol", [((17, 3, 2), 8, "fp64", TOL64), ((2, 20, 3), 8, "fp64", TOL64),
                                                   ((2, 2, 40), 8, "fp64", TOL64), ((3, 18, 35), 8, "fp64", TOL64),
                                                   ((3, 17, 3), 16, "fp64", TOL64),
                                                   ((2, 3, 33), 16, "fp32_refine", TOLMIX),
                                                   ((18, 17, 33), 8, "fp32_refine", TOLMIX)])
def test_lattice_wide_boxes_sampled(lat_ctx, ext, nb, precision, tol):
    """x or y extents 17..32 take the DFT length 64 and z extents 33..64 the
    length 128 (the z line split over four waves); ragged extents, both
    block sizes, both precisions."""
    rng = np.random.default_rng(sum(ext) * 13 + nb)
    blocks = _box(*ext, lo=(-5, 3, -9))
    c = inputs.cell_coords(blocks, nb)
    f = rng.standard_normal(len(c))
    u, st = _lattice_stages(lat_ctx, _problem(blocks, nb, f, 0.4), precision)
    assert st["lat_yz"][1] > 0 and st["smac"][1] == 0, st
    n = 400 if len(c) > 1_000_000 else 1200
    idx = np.concatenate([rng.choice(len(c), n, replace=False), [0, len(c) - 1]])
    assert rel_l2(u[0][idx], direct.direct_sum(c, f, c[idx], 0.4)) < tol


@pytest.mark.parametrize("ext", [(17, 5, 34), (4, 26, 3)])
def test_wide_lattice_matches_pairs_full_field(lat_ctx, pairs_ctx, ext):
    """On every cell: the wide lattice lengths against the block pairs."""
    rng = np.random.default_rng(sum(ext))
    nb = 8
    blocks = _box(*ext, lo=(1, -2, 0))
    blocks = blocks[rng.uniform(size=len(blocks)) < 0.6]
    c = inputs.cell_coords(blocks, nb)
    f = rng.standard_normal(len(c))
    a = gpu_solve(lat_ctx, _problem(blocks, nb, f, 0.5))[0]
    b = gpu_solve(pairs_ctx, _problem(blocks, nb, f, 0.5))[0]
    assert rel_l2(a, b) < 1e-13


def test_lattice_y_extent_33_takes_block_pairs(lat_ctx):
    """Past 32 blocks along y there is no compiled lattice length (levels
    reach 64 blocks per axis): the lattice-only setting falls back to block
    pairs, still exact."""
    rng = np.random.default_rng(77)
    nb = 8
    blocks = _box(2, 33, 2, lo=(0, -16, 0))
    c = inputs.cell_coords(blocks, nb)
    f = rng.standard_normal(len(c))
    lat_ctx.set_timing(True)
    lat_ctx.stage_times()
    try:
        u = gpu_solve(lat_ctx, _problem(blocks, nb, f, 0.6))[0]
        st = lat_ctx.stage_times()
    finally:
        lat_ctx.set_timing(False)
    assert st["lat_yz"][1] == 0 and st["smac"][1] > 0, st
    idx = rng.choice(len(c), 1500, replace=False)
    assert rel_l2(u[idx], direct.direct_sum(c, f, c[idx], 0.6)) < TOL64


@pytest.mark.parametrize("seed", [0, 1])
def test_lattice_sparse_support_full_parity(lat_ctx, seed):
    rng = np.random.default_rng(40 + seed)
    nb = 8
    box = _box(6, 5, 7)
    blocks = box[rng.uniform(size=len(box)) < 0.35] + np.array([2, -4, 1])
    c = inputs.cell_coords(blocks, nb)
    f = rng.standard_normal(len(c))
    u = gpu_solve(lat_ctx, _problem(blocks, nb, f, 0.7))[0]
    assert rel_l2(u, direct.direct_sum(c, f, c, 0.7)) < TOL64


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32_refine", TOLMIX)])
def test_lattice_gaussian_box_and_mixed(lat_ctx, precision, tol):
    p = inputs.gaussian_box()
    u = gpu_solve(lat_ctx, p, precision)[0]
    c = level_cells(p)
    f = p.levels[0].values[0].reshape(-1)
    assert rel_l2(u, direct.direct_sum(c, f, c, p.dx0)) < tol


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32_refine", TOLMIX)])
def test_lattice_vortex_ring_vector_sampled(lat_ctx, precision, tol):
    p = inputs.single_ring()                    # 208 blocks of 16^3, 3 components
    u = gpu_solve(lat_ctx, p, precision)
    c = level_cells(p)
    rng = np.random.default_rng(9)
    idx = rng.choice(len(c), 1000, replace=False)
    for comp in range(2):
        f = p.levels[0].values[comp].reshape(-1)
        nz = f != 0
        assert rel_l2(u[comp][idx], direct.direct_sum(c[nz], f[nz], c[idx], p.dx0)) < tol
    assert np.all(u[2] == 0.0)


def test_lattice_vector_equals_scalar_bitwise(lat_ctx):
    p = inputs.single_ring(nb=8, dx=1.0 / 16, components=(0, 1))
    vec = gpu_solve(lat_ctx, p)
    for comp in range(2):
        one = inputs.Problem(nb=p.nb, dx0=p.dx0, name="one",
                             levels=[inputs.Level(blocks=p.levels[0].blocks,
                                                  values=p.levels[0].values[comp:comp + 1])])
        assert np.array_equal(gpu_solve(lat_ctx, one)[0], vec[comp]), comp


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("fp32_refine", TOLMIX)])
def test_lattice_two_level_ring_against_stored_oracle(lat_ctx, precision, tol):
    """The stored oracle samples of the two-level ring (written by
    tests/golden/make_two_level_ring.py from the oracle only)."""
    import os
    gold = np.load(os.path.join(os.path.dirname(__file__), "golden", "two_level_ring_samples.npz"))
    p = inputs.two_level_ring(components=(0, 1))
    assert len(p.levels[1].blocks) == int(gold["n_blocks1"])
    u = gpu_solve(lat_ctx, p, precision)
    n0 = len(p.levels[0].blocks) * p.nb ** 3
    for k in range(2):
        part = u[:, :n0] if k == 0 else u[:, n0:]
        idx = gold["sample%d" % k]
        for comp in range(2):
            assert rel_l2(part[comp][idx], gold["phi%d_c%d" % (k, comp)]) < tol, (k, comp)


def test_lattice_matches_pairs_on_dense_256_box(lat_ctx, pairs_ctx):
    p = inputs.mstar()
    a = gpu_solve(lat_ctx, p)[0]
    b = gpu_solve(pairs_ctx, p)[0]
    assert rel_l2(a, b) < 1e-13
    c = level_cells(p)
    rng = np.random.default_rng(8)
    idx = rng.choice(len(c), 200, replace=False)
    f = p.levels[0].values[0].reshape(-1)
    assert rel_l2(a[idx], direct.direct_sum(c, f, c[idx], p.dx0)) < TOL64


def test_lattice_batch_equals_alone_bitwise(lat_ctx):
    import torch
    from paper_2010_13213_amd import lgf
    reqs = inputs.served_stream(8, seed=23, sizes=[16, 40, 64, 128])
    alone = []
    for r in reqs:
        plan = lgf.Plan.for_problem(lat_ctx, r.problem, r.precision)
        alone.append(plan.solve(torch.from_numpy(r.problem.flat_source()).cuda()).cpu().numpy())
        plan.close()
    plans = [lgf.Plan.for_problem(lat_ctx, r.problem, r.precision) for r in reqs]
    fs = [torch.from_numpy(r.problem.flat_source()).cuda() for r in reqs]
    us = [torch.empty_like(f) for f in fs]
    lgf.solve_batch(lat_ctx, plans, fs, us)
    torch.cuda.synchronize()
    for i, (a, u) in enumerate(zip(alone, us)):
        assert np.array_equal(a, u.cpu().numpy()), i
    for pl in plans:
        pl.close()


def test_lattice_graph_replays_equal_eager(lat_ctx):
    import torch
    from paper_2010_13213_amd import lgf
    p = inputs.gaussian_box(n_blk=6, nb=8)
    plan = lgf.Plan.for_problem(lat_ctx, p, "fp64")
    f0 = torch.from_numpy(p.flat_source()).cuda()
    f1 = (torch.flip(f0, dims=[0]) * 0.25).contiguous()
    ref0, ref1 = plan.solve(f0), plan.solve(f1)
    torch.cuda.synchronize()
    f = f0.clone()
    u = torch.empty_like(f0)
    g = lgf.Graph(plan, f, u)
    for rep, (src, ref) in enumerate([(f0, ref0), (f1, ref1), (f0, ref0)]):
        f.copy_(src)
        u.fill_(float("nan"))
        g.launch()
        torch.cuda.synchronize()
        assert torch.equal(u, ref), rep
        assert torch.equal(plan.solve(f1), ref1)      # eager work between replays
    g.close()
    plan.close()


def test_box_longer_than_32_blocks_along_x_uses_pairs(lat_ctx):
    nb = 8
    blocks = _box(33, 2, 1)
    rng = np.random.default_rng(12)
    c = inputs.cell_coords(blocks, nb)
    f = rng.standard_normal(len(c))
    lat_ctx.set_timing(True)
    lat_ctx.stage_times()
    try:
        u = gpu_solve(lat_ctx, _problem(blocks, nb, f))[0]
        st = lat_ctx.stage_times()
    finally:
        lat_ctx.set_timing(False)
    assert st["lat_yz"][1] == 0 and st["smac"][1] > 0, st
    idx = rng.choice(len(c), 2000, replace=False)
    assert rel_l2(u[idx], direct.direct_sum(c, f, c[idx], 1.0)) < TOL64


def test_batch_mixing_pair_and_lattice_plans_equals_alone_bitwise():
    # one lgf_solve_batch call over plans whose convolutions use different
    # spectral layouts (block pairs: frequency-major; lattice: block-major):
    # the batched block FFTs take the layout per job
    import torch
    from paper_2010_13213_amd import lgf
    ctx = lgf.Context(0)
    try:
        probs = [inputs.gaussian_box(n_blk=4, nb=8), inputs.gaussian_box(n_blk=6, nb=8),
                 inputs.gaussian_box(n_blk=3, nb=8), inputs.gaussian_box(n_blk=5, nb=8)]
        setup = [("pairs", "fp64"), ("lattice", "fp64"), ("pairs", "fp32_refine"), ("lattice", "fp32_refine")]
        plans = []
        for p, (method, precision) in zip(probs, setup):
            ctx.set_mac_method(method)
            plans.append(lgf.Plan.for_problem(ctx, p, precision))
        fs = [torch.from_numpy(p.flat_source()).cuda() for p in probs]
        alone = [pl.solve(f).cpu().numpy() for pl, f in zip(plans, fs)]
        us = [torch.empty_like(f) for f in fs]
        lgf.solve_batch(ctx, plans, fs, us)
        torch.cuda.synchronize()
        for i, (a, u) in enumerate(zip(alone, us)):
            assert np.array_equal(a, u.cpu().numpy()), setup[i]
        for pl in plans:
            pl.close()
    finally:
        ctx.close()
