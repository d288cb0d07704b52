"""Pins of the composite-grid oracle (paper Sec. 3.2-3.4).

* one level reduces to the plain direct sum;
* trilinear P reproduces polynomials of degree <= 1 exactly and the mean-8
  coarsening conserves sum(f) dx^3;
* the correction source S = (P L_c - L_f P) G of a coarse point source
  decays like |n|^-4 with the magnitudes the paper prints (about 1e-4 at
  14 cells, Sec. 3.4 manufactured test; about 3e-5 at 20 cells, Sec. 3.3
  footnote);
* a coarse-only source f^_0 = L_0 Psi with compact Psi (the paper's
  manufactured-solution idea, Sec. 3.4) through the full two-level
  recursion: phi_0 = Psi exactly on Omega_0, and phi_1 equals the formal
  composite answer L_1^-1 P f^_0 (eq. comm_p / p_bar) to rounding once the
  extended region covers the support of the correction source;
* three levels: the cumulative source F_k conserves the mass of f^ on
  levels >= k and reproduces linear fields exactly (mean of 8 children =
  value at the parent's centre); a smooth coarse source that is linear under
  the refined levels reaches the finest level as L_2^-1 P P f^_0 through
  psi_1 = P psi_0 + L_1^-1 S_1; compact middle- and fine-level sources give
  phi_2 = Psi_2 + L_2^-1 P f^_1 and phi_1 = Psi_1 + L_1^-1 (mean-8 of f^_2).
"""
import numpy as np
import pytest

from oracle import composite as C, direct, lgf_table as T


def _cube_blocks(lo, n):
    return np.array([(x, y, z) for z in range(lo, lo + n) for y in range(lo, lo + n)
                     for x in range(lo, lo + n)])


def _gauss(cells, dx, ctr, w):
    p = (cells + 0.5) * dx
    return np.exp(-((p - ctr) ** 2).sum(axis=1) / (2 * w * w))


def test_single_level_reduces_to_direct_sum():
    nb = 8
    blocks = _cube_blocks(0, 2)
    orc = C.CompositeOracle(nb, 0.5, [blocks])
    cells = orc.cells[0]
    f = _gauss(cells, 0.5, 4.0, 1.5)
    phi = orc.solve([f])[0]
    ref = direct.direct_sum(cells, f, cells, 0.5)
    assert np.array_equal(phi, ref)


def test_trilinear_reproduces_linear_functions():
    box = C.Box(np.array([-3, -3, -3]), np.array([9, 9, 9]))
    cc = box.cells()
    a, b = np.array([0.3, -1.1, 2.0]), 0.7
    coarse = ((cc + 0.5) @ a + b).reshape(box.shape)       # at coarse centres
    fine = np.array([[x, y, z] for x in range(0, 12) for y in range(0, 12)
                     for z in range(0, 12)])
    got = C.interp_trilinear(box, coarse, fine)
    want = ((fine + 0.5) / 2.0) @ a + b                      # fine centres, coarse units
    assert np.max(np.abs(got - want)) < 1e-13


def test_mean8_coarsening_conserves_integral():
    rng = np.random.default_rng(0)
    fb = C.Box(np.array([0, 0, 0]), np.array([8, 8, 8]))
    fine = rng.standard_normal(fb.shape)
    cc = np.array([[x, y, z] for x in range(4) for y in range(4) for z in range(4)])
    coarse = C.coarsen_mean8(fb, fine, cc)
    dxf = 0.5
    assert abs(coarse.sum() * (2 * dxf) ** 3 - fine.sum() * dxf ** 3) < 1e-12
    ones = C.coarsen_mean8(fb, np.ones(fb.shape), cc)
    assert np.all(ones == 1.0)


def _correction_of_point_source(dist):
    """|S| / max|S| at fine cells (2m, 0, 0)-ish along the x axis."""
    R = 30
    cb = C.Box(np.array([-R, -R, -R]), np.array([R + 1] * 3))
    psi = T.G(cb.cells()).reshape(cb.shape)             # coarse dx = 1: L_c psi = delta
    Lpsi = C.laplacian7(psi, 1.0)
    pts = np.array([[m, 0, 0] for m in range(0, 2 * (R - 4))])
    nbrs = [np.array(o) for o in [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0),
                                  (0, 0, 1), (0, 0, -1)]]
    Pp = [C.interp_trilinear(cb, psi, pts + o) for o in nbrs]
    dxf = 0.5
    LP = (sum(Pp[1:]) - 6 * Pp[0]) / dxf ** 2
    S = C.interp_trilinear(cb, Lpsi, pts) - LP
    S = np.abs(S) / np.abs(S).max()
    return {d: S[d] for d in dist}


def test_correction_source_decay_matches_paper_magnitudes():
    s = _correction_of_point_source([14, 20, 40])
    # the paper's figures are order-of-magnitude ("about"): accept a factor 5
    assert 2e-5 < s[14] < 5e-4           # "about 1e-4" at N_E = 14
    assert 6e-6 < s[20] < 1.5e-4         # "about 3e-5 at 20 cells"
    assert 10 < s[20] / s[40] < 24       # |n|^-4 decay: 2^4 = 16


def _bump(cells, ctr, R):
    t2 = (((cells + 0.5) - ctr) ** 2).sum(axis=1) / (R * R)
    out = np.zeros(len(cells))
    m = t2 < 1
    out[m] = np.exp(-10.0 / (1.0 - t2[m])) * 1e3
    return out


def _lap_on_cells(box_lo, box_hi, fn, cells, dx):
    box = C.Box(np.array(box_lo), np.array(box_hi))
    a = fn(box.cells()).reshape(box.shape)
    L = C.laplacian7(a, dx)
    i, j, k = box.idx(cells)
    return L[i, j, k]


# Each composite pin runs with every convolution a direct sum (None) and with
# every convolution a zero-padded FFT over the bounding box (1 target).
FFT_MODES = pytest.mark.parametrize("fft", [None, 1], ids=["direct", "fft"])


def _two_level(ext_layers, fft=None):
    nb = 8
    coarse = _cube_blocks(0, 4)                   # coarse cells [0, 32)^3, dx0 = 1
    fine = _cube_blocks(2, 2)                     # refines coarse cells [8, 16)^3
    orc = C.CompositeOracle(nb, 1.0, [coarse, fine], ext_layers=ext_layers, fft_min_targets=fft)
    ctr, rad = np.array([22.0, 22.0, 22.0]), 4.5  # compact Psi in the coarse-only zone
    psi = lambda c: _bump(c, ctr, rad)
    f0 = _lap_on_cells((-2, -2, -2), (34, 34, 34), psi, orc.cells[0], 1.0)
    f1 = np.zeros(len(orc.cells[1]))
    return orc, psi, f0, f1


@FFT_MODES
def test_two_level_exact_when_extension_covers_correction_support(fft):
    """f^_0 = L_0 Psi with compact Psi: phi_0 = Psi on Omega_0 and
    phi_1 = L_1^-1 P f^_0 exactly once Omega_1^E covers supp S."""
    orc, psi, f0, f1 = _two_level(ext_layers=3, fft=fft)
    assert np.all(orc.mask[0][f0 != 0])           # the source lives on Omega_0
    phi = orc.solve([f0, f1])
    m0 = orc.mask[0]
    ref0 = psi(orc.cells[0][m0])
    assert np.abs(phi[0][m0] - ref0).max() < 1e-12 * np.abs(ref0).max()
    # formal level-1 answer: interpolate f^_0 to the fine lattice and convolve
    cb = C.Box(np.array([-2, -2, -2]), np.array([34, 34, 34]))
    arr = cb.zeros()
    i, j, k = cb.idx(orc.cells[0])
    arr[i, j, k] = f0
    fcells = C.Box(np.array([24, 24, 24]), np.array([62, 62, 62])).cells()
    Pf = C.interp_trilinear(cb, arr, fcells)
    keep = Pf != 0
    ref1 = direct.direct_sum(fcells[keep], Pf[keep], orc.cells[1], 0.5)
    # phi_1 is the small commutator response (|ref1| ~ 1e-5 |Psi|), so check
    # it both against the problem's scale and relative to itself
    scale = np.abs(ref0).max()
    assert np.abs(phi[1] - ref1).max() < 1e-14 * scale
    assert np.linalg.norm(phi[1] - ref1) / np.linalg.norm(ref1) < 1e-9


# ---------------------------------------------------------------- K = 3 --
#
# Pins of the fine -> coarse cumulative source and of the psi_k recursion at
# three levels (Sec. 3.4: F_k = f^_k + P_{k+1->k} F_{k+1}; psi_1 =
# P psi_0 + L_1^-1 (S_1 + f^_1); phi_k = P psi_{k-1} + L_k^-1 (S_k + F_k)).

def _box_blocks(lo, hi):
    """Blocks with lo <= b < hi per axis, z slowest."""
    return np.array([(x, y, z) for z in range(lo[2], hi[2]) for y in range(lo[1], hi[1])
                     for x in range(lo[0], hi[0])])


def _three_level_nested():
    """An irregular three-level mesh of 4^3 blocks (dx0 = 1)."""
    nb = 4
    lv0 = _box_blocks((0, 0, 0), (4, 4, 4))                   # coarse cells [0, 16)^3
    lv1 = np.array([b for b in _box_blocks((2, 2, 2), (6, 6, 6)).tolist()
                    if not (b[0] == 5 and b[1] == 5)])        # refines coarse [4, 12)^3, one column cut
    lv2 = np.array([b for b in _box_blocks((6, 6, 6), (10, 10, 10)).tolist()
                    if not (b[2] == 9 and b[0] == 6)])        # refines level-1 [12, 20)^3, one column cut
    return C.CompositeOracle(nb, 1.0, [lv0, lv1, lv2])


def test_cumulative_source_conserves_mass_at_every_level():
    """sum F_k dx_k^3 over level k = the mass of f^ on levels k..K-1: a dropped
    coarsening, a wrong weight or a lost child changes it."""
    orc = _three_level_nested()
    rng = np.random.default_rng(5)
    fhat = [np.where(orc.mask[k], rng.standard_normal(len(orc.cells[k])), 0.0) for k in range(3)]
    F = orc.cumulative_sources(fhat)
    mass = [float(fhat[k].sum()) * orc.dx[k] ** 3 for k in range(3)]
    for k in range(3):
        want = sum(mass[k:])
        got = float(F[k].sum()) * orc.dx[k] ** 3
        assert abs(got - want) < 1e-12 * sum(abs(m) for m in mass), (k, got, want)
        assert np.array_equal(F[k][orc.mask[k]], fhat[k][orc.mask[k]])   # Omega_k keeps f^_k


def test_cumulative_source_reproduces_linear_fields():
    """f = a.x + b at cell centres on every level: the mean of the 8 children
    of a cell is the value at its centre, so F_k = a.x + b on every level-k
    cell.  A child map shifted by a cell or a block fails this."""
    orc = _three_level_nested()
    a, b = np.array([0.7, -1.3, 2.1]), 0.4
    lin = [((orc.cells[k] + 0.5) * orc.dx[k]) @ a + b for k in range(3)]
    fhat = [np.where(orc.mask[k], lin[k], 0.0) for k in range(3)]
    F = orc.cumulative_sources(fhat)
    for k in range(3):
        assert np.abs(F[k] - lin[k]).max() < 1e-13 * np.abs(lin[k]).max(), k
        assert not orc.mask[k].all() or k == 2        # levels 0 and 1 have covered cells


def _k3_geometry():
    """Three levels of 8^3 blocks: level 1 a 4x2x2-block slab, level 2 a
    2x2x2-block cube flush with level 1's low-x face (so coarse sources
    just outside level 1 sit close to level 2)."""
    nb = 8
    lv0 = _box_blocks((0, 0, 0), (4, 4, 4))                   # coarse cells [0, 32)^3
    lv1 = _box_blocks((2, 3, 3), (6, 5, 5))                   # level-1 cells [16,48) x [24,40)^2
    lv2 = _box_blocks((4, 7, 7), (6, 9, 9))                   # level-2 cells [32,48) x [56,72)^2
    return nb, [lv0, lv1, lv2]


def _lap_box(box, fn, dx):
    return C.laplacian7(fn(box.cells()).reshape(box.shape), dx)


def _pick(box, arr, cells):
    i, j, k = box.idx(cells)
    return arr[i, j, k]


def _sample(orc, k, n, seed):
    idx = np.nonzero(orc.mask[k])[0]
    return np.sort(np.random.default_rng(seed).choice(idx, min(n, len(idx)), replace=False))


def _smooth_step(t):
    """1 for t <= 0, 0 for t >= 1, C-infinity in between."""
    t = np.clip(t, 0.0, 1.0)
    out = (t <= 0).astype(np.float64)
    m = (t > 0) & (t < 1)
    a = np.exp(-1.0 / t[m])
    b = np.exp(-1.0 / (1.0 - t[m]))
    out[m] = b / (a + b)
    return out


@FFT_MODES
def test_three_level_coarse_source_reaches_finest_level_through_psi_recursion(fft):
    """f^_0 = L_0 Psi_0 on Omega_0, nothing finer.  Psi_0 is linear (so
    discrete-harmonic: L_0 Psi_0 = 0) on a coarse box around the refined
    region and falls smoothly to 0 outside it, so f^_0 is compact, lives on
    Omega_0, and psi_0 = Psi_0 carries an O(1) value under levels 1 and 2.
    With the extended regions covering the correction sources, P-bar = P +
    L^-1 S (eqs. comm_p, p_bar) gives phi_0 = Psi_0 and phi_1 = L_1^-1 P f^_0
    exactly, and phi_2 = L_2^-1 P P f^_0 up to the part of S_2 beyond
    Omega_2^E (psi_1 = L_1^-1 P f^_0 is not compact; 7.8e-5 measured here).
    phi_2 runs through psi_1 = P psi_0 + L_1^-1 S_1: dropping either term,
    a wrong sign or a wrong level spacing in it is an O(1) error."""
    nb, lo, hi, w = 4, 7.0, 11.0, 4.0
    lv0 = _box_blocks((0, 0, 0), (5, 5, 5))                   # coarse cells [0, 20)^3
    orc = C.CompositeOracle(nb, 1.0, [lv0, np.array([[4, 4, 4]]), np.array([[8, 8, 8]])], ext_layers=7,
                            fft_min_targets=fft)
    a, b = np.array([0.3, -0.5, 0.8]), 2.0

    def psi0(c):                # linear on centres in [lo, hi)^3, 0 beyond distance w
        p = c + 0.5
        d = np.maximum(np.maximum(lo - p, p - hi), 0.0) / w
        return (p @ a + b) * _smooth_step(d[:, 0]) * _smooth_step(d[:, 1]) * _smooth_step(d[:, 2])

    box0 = C.Box(np.array([-2] * 3), np.array([22] * 3))
    f0 = _pick(box0, _lap_box(box0, psi0, 1.0), orc.cells[0])
    harmonic = np.all((orc.cells[0] >= lo + 1) & (orc.cells[0] < hi - 1), axis=1)
    assert np.abs(f0[harmonic]).max() < 1e-13 * np.abs(f0).max()
    f0[harmonic] = 0.0                 # exactly 0 there; only rounding was left
    assert np.all(orc.mask[0][f0 != 0]) and not orc.mask[0].all()
    zero = [np.zeros(len(orc.cells[k])) for k in (1, 2)]
    samp = [_sample(orc, k, 100, 10 + k) for k in range(3)]
    phi = orc.solve([f0] + zero, sample=samp)
    ref0 = psi0(orc.cells[0][samp[0]])
    assert np.linalg.norm(phi[0][samp[0]] - ref0) / np.linalg.norm(ref0) < 1e-12
    # P f^_0 on level 1 and P P f^_0 on level 2, over boxes holding their support
    arr0 = box0.zeros()
    i, j, k = box0.idx(orc.cells[0])
    arr0[i, j, k] = f0
    box1 = C.Box(np.array([0] * 3), np.array([36] * 3))
    Pf = C.interp_trilinear(box0, arr0, box1.cells())
    box2 = C.Box(2 * box1.lo + 2, 2 * box1.hi - 2)
    PPf = C.interp_trilinear(box1, Pf.reshape(box1.shape), box2.cells())
    for arr, bx in ((Pf, box1), (PPf, box2)):
        e = np.abs(arr.reshape(bx.shape))
        assert max(e[[0, -1]].max(), e[:, [0, -1]].max(), e[:, :, [0, -1]].max()) == 0.0
    c1, c2 = box1.cells(), box2.cells()
    ref1 = direct.direct_sum(c1[Pf != 0], Pf[Pf != 0], orc.cells[1][samp[1]], 0.5)
    ref2 = direct.direct_sum(c2[PPf != 0], PPf[PPf != 0], orc.cells[2][samp[2]], 0.25)
    assert np.linalg.norm(phi[1][samp[1]] - ref1) / np.linalg.norm(ref1) < 1e-12
    e2 = np.linalg.norm(phi[2][samp[2]] - ref2) / np.linalg.norm(ref2)
    assert e2 < 1e-3, e2


@FFT_MODES
def test_three_level_middle_and_fine_sources(fft):
    """f^_1 = L_1 Psi_1 on Omega_1 and f^_2 = L_2 Psi_2 on Omega_2 (compact),
    f^_0 = 0.  Then psi_0 = 0, psi_1 = Psi_1 (the recursion takes f^_1, not
    the cumulative F_1), S_2 = (P L_1 - L_2 P) Psi_1 is compact and covered,
    so exactly phi_2 = Psi_2 + L_2^-1 P f^_1 and phi_1 = Psi_1 + L_1^-1 F
    with F the mean of the 8 children of f^_2 (eq. combine_S)."""
    nb, blocks = _k3_geometry()
    orc = C.CompositeOracle(nb, 1.0, blocks, ext_layers=2, fft_min_targets=fft)
    psi1 = lambda c: _bump(c, np.array([27.0, 32.0, 32.0]), 2.2)   # level-1 x in (24.8, 29.2): Omega_1
    psi2 = lambda c: _bump(c, np.array([40.0, 64.0, 64.0]), 5.5)   # level-2 cells inside Omega_2
    box1 = C.Box(np.array([14, 22, 22]), np.array([50, 42, 42]))
    box2 = C.Box(np.array([30, 54, 54]), np.array([50, 74, 74]))
    f1 = _pick(box1, _lap_box(box1, psi1, 0.5), orc.cells[1])
    lap2 = _lap_box(box2, psi2, 0.25)
    f2 = _pick(box2, lap2, orc.cells[2])
    assert np.all(orc.mask[1][f1 != 0])
    f0 = np.zeros(len(orc.cells[0]))
    samp = [_sample(orc, k, 150, 20 + k) for k in range(3)]
    phi = orc.solve([f0, f1, f2], sample=samp)
    # level 2
    arr1 = box1.zeros()
    i, j, k = box1.idx(orc.cells[1])
    arr1[i, j, k] = f1
    fine = C.Box(np.array([44, 54, 54]), np.array([62, 74, 74]))
    Pf1 = C.interp_trilinear(box1, arr1, fine.cells())
    a = np.abs(Pf1.reshape(fine.shape))
    assert max(a[[0, -1]].max(), a[:, [0, -1]].max(), a[:, :, [0, -1]].max()) == 0.0
    t2 = orc.cells[2][samp[2]]
    ref2 = psi2(t2) + direct.direct_sum(fine.cells()[Pf1 != 0], Pf1[Pf1 != 0], t2, 0.25)
    assert np.linalg.norm(phi[2][samp[2]] - ref2) / np.linalg.norm(ref2) < 1e-11
    # level 1: the 8-children mean of f^_2 by reshaping, independent of the oracle's helper
    assert np.all(box2.lo % 2 == 0) and np.all(np.array(box2.shape) % 2 == 0)
    n = [s // 2 for s in box2.shape]
    F = lap2.reshape(n[0], 2, n[1], 2, n[2], 2).mean(axis=(1, 3, 5)).ravel()
    cc = C.Box(box2.lo // 2, box2.lo // 2 + np.array(n)).cells()
    t1 = orc.cells[1][samp[1]]
    ref1 = psi1(t1) + direct.direct_sum(cc[F != 0], F[F != 0], t1, 0.5)
    assert np.linalg.norm(phi[1][samp[1]] - ref1) / np.linalg.norm(ref1) < 1e-11


def test_cell_masks_state_the_partition():
    """Reading c8 (Sec. 3.1, eq. partition): a cell mask equal to the cover
    reproduces the unmasked recursion bit for bit; dropping uncovered cells
    equals zeroing their sources and discarding their targets; a kept
    covered cell is refused."""
    orc = _three_level_nested()
    blocks = orc.blocks
    rng = np.random.default_rng(11)
    f = [rng.standard_normal(len(orc.cells[k])) for k in range(3)]
    base = orc.solve(f, sample=[np.arange(0, len(orc.cells[k]), 37) for k in range(3)])
    same = C.CompositeOracle(orc.nb, 1.0, blocks, cell_masks=[m.astype(np.uint8) for m in orc.mask])
    got = same.solve(f, sample=[np.arange(0, len(orc.cells[k]), 37) for k in range(3)])
    for a, b in zip(base, got):
        assert np.array_equal(a, b)
    drop = [m.copy() for m in orc.mask]
    drop[0][:700] = False                             # uncovered coarse cells leave Omega_0
    masked = C.CompositeOracle(orc.nb, 1.0, blocks, cell_masks=drop)
    f2 = [np.where(drop[k], f[k], 0.0) for k in range(3)]
    samp = [np.arange(0, len(orc.cells[k]), 23) for k in range(3)]
    ref = orc.solve(f2, sample=samp)
    out = masked.solve(f, sample=samp)
    for k in range(3):
        keep = samp[k][drop[k][samp[k]]]
        assert np.array_equal(out[k][keep], ref[k][keep])
        gone = samp[k][~drop[k][samp[k]]]
        assert np.all(out[k][gone] == 0.0)
    bad = [m.copy() for m in orc.mask]
    bad[1][np.nonzero(~orc.mask[1])[0][0]] = True
    with pytest.raises(ValueError):
        C.CompositeOracle(orc.nb, 1.0, blocks, cell_masks=bad)
