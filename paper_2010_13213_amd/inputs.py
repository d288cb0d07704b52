"""Seeded synthetic inputs: block supports and source fields.

This module holds no arithmetic of the LGF method; it only builds problem
descriptions (occupied N_b^3 blocks per level, source values per cell) that
both the HIP path and the CPU oracle consume.  Layout convention used
everywhere: a level's field is stored block after block, each block as
[z][y][x] with x fastest; cell (x, y, z) of block b sits at lattice point
b * nb + (x, y, z).  Cell (i, j, k) of a level with spacing dx has its centre
at origin + (i + 1/2, j + 1/2, k + 1/2) * dx.

Workloads (shapes follow the paper's vortex-ring experiments, Sec. 6-7):

* ``gaussian_box``    -- scalar Gaussian on a dense cube of 8^3 blocks.
* ``ring_level``      -- thin vortex ring (radius R, Gaussian core sigma),
                         support = blocks with any cell centre within
                         ``k_sigma * sigma`` of the (optionally perturbed) core.
* ``two_level_ring``  -- coarse ring support plus a finer level around the
                         perturbed core.
* ``mstar``           -- dense 256^3 box at dx = R/64 over [-2R, 2R]^3,
                         16^3 blocks, x-vorticity of the ring.
* ``colliding_rings`` -- three levels around two tilted, perturbed rings.
* ``served_stream``   -- independent dense-cube requests with Gaussian blobs.
"""
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


@dataclass
class Level:
    blocks: np.ndarray            # (n, 3) int32 block coordinates
    values: np.ndarray            # (n_comp, n, nb, nb, nb) float64, [b][z][y][x]
    cell_mask: Optional[np.ndarray] = None   # (n, nb, nb, nb) 0/1: the cells of Omega_k (None: not covered)


@dataclass
class Problem:
    nb: int
    dx0: float
    levels: List[Level]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_components(self):
        return self.levels[0].values.shape[0]

    def flat_source(self):
        """f as one float64 array in [comp][level][block][z][y][x] order."""
        nc = self.n_components
        parts = [np.concatenate([lv.values[c].reshape(-1) for lv in self.levels])
                 for c in range(nc)]
        return np.ascontiguousarray(np.concatenate(parts))

    def n_cells(self):
        return sum(len(lv.blocks) for lv in self.levels) * self.nb ** 3


def cell_coords(blocks, nb):
    """(n*nb^3, 3) int32 lattice coordinates in [block][z][y][x] order."""
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    r = np.arange(nb)
    zz, yy, xx = np.meshgrid(r, r, r, indexing="ij")
    local = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    return (blocks[:, None, :] * nb + local[None, :, :]).reshape(-1, 3).astype(np.int32)


def cell_centres(blocks, nb, dx, origin):
    """Physical centres (n, nb, nb, nb, 3) of every cell, [b][z][y][x]."""
    c = cell_coords(blocks, nb).astype(np.float64)
    return (np.asarray(origin) + (c + 0.5) * dx).reshape(len(blocks), nb, nb, nb, 3)


# --------------------------------------------------------------------------
# Ring geometry
# --------------------------------------------------------------------------

def ring_radius_perturbation(seed, R=1.0, n_modes=32, rel_amp=0.01):
    """Return dR(phi): sum_m cos(m phi + theta_m) scaled to max|dR| = rel_amp*R."""
    if seed is None:
        return lambda phi: np.zeros_like(phi)
    rng = np.random.Generator(np.random.PCG64(seed))
    theta = rng.uniform(0.0, 2.0 * np.pi, n_modes)
    m = np.arange(1, n_modes + 1)
    grid = np.linspace(0.0, 2.0 * np.pi, 20000, endpoint=False)
    raw = np.cos(m[None, :] * grid[:, None] + theta[None, :]).sum(axis=1)
    a = rel_amp * R / np.abs(raw).max()

    def dR(phi):
        phi = np.asarray(phi)
        return a * np.cos(m * phi[..., None] + theta).sum(axis=-1)
    return dR


def ring_core_distance(p, R=1.0, dR=None):
    """Distance s from points p (..., 3) to the ring core (axis z, centre 0)."""
    x, y, z = p[..., 0], p[..., 1], p[..., 2]
    rho = np.sqrt(x * x + y * y)
    Rloc = R if dR is None else R + dR(np.arctan2(y, x))
    return np.sqrt(z * z + (rho - Rloc) ** 2), rho


def ring_vorticity(p, R=1.0, sigma=0.1, dR=None):
    """Gaussian-core azimuthal vorticity (omega_x, omega_y, omega_z) at p."""
    s, rho = ring_core_distance(p, R, dR)
    wt = np.exp(-s * s / (2.0 * sigma * sigma)) / (2.0 * np.pi * sigma * sigma)
    rho_safe = np.where(rho > 0, rho, 1.0)
    wx = -wt * p[..., 1] / rho_safe
    wy = wt * p[..., 0] / rho_safe
    return np.stack([wx, wy, np.zeros_like(wx)], axis=0)


def blocks_near_core(nb, dx, box_lo, box_cells, dist_fn, cutoff):
    """Blocks of a box (box_cells per axis) with any cell centre at dist <= cutoff."""
    nblk = box_cells // nb
    origin = np.asarray(box_lo, dtype=np.float64)
    out = []
    r = (np.arange(nb) + 0.5) * dx
    for bz in range(nblk):
        for by in range(nblk):
            for bx in range(nblk):
                X, Y, Z = np.meshgrid(origin[0] + bx * nb * dx + r,
                                      origin[1] + by * nb * dx + r,
                                      origin[2] + bz * nb * dx + r, indexing="ij")
                d = dist_fn(np.stack([X, Y, Z], axis=-1))
                if d.min() <= cutoff:
                    out.append((bx, by, bz))
    return np.asarray(out, dtype=np.int32).reshape(-1, 3)


def _level_from_fn(blocks, nb, dx, origin, fn, n_comp):
    p = cell_centres(blocks, nb, dx, origin)
    vals = fn(p)
    return Level(blocks=np.asarray(blocks, dtype=np.int32),
                 values=np.ascontiguousarray(vals.reshape(n_comp, len(blocks), nb, nb, nb)))


# --------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------

def gaussian_box(n_blk=4, nb=8, width=4.0, noise=1e-3, seed=1):
    """Scalar Gaussian exp(-|x-c|^2 / (2 w^2)) on a dense cube plus U(-noise, noise)."""
    L = n_blk * nb
    b = np.array([(x, y, z) for z in range(n_blk) for y in range(n_blk)
                  for x in range(n_blk)], dtype=np.int32)
    c = cell_coords(b, nb).astype(np.float64)
    mid = (L - 1) / 2.0
    r2 = ((c - mid) ** 2).sum(axis=1)
    f = np.exp(-r2 / (2.0 * width * width))
    rng = np.random.Generator(np.random.PCG64(seed))
    f = f + rng.uniform(-noise, noise, size=f.shape)
    return Problem(nb=nb, dx0=1.0, name="gaussian_box_%d" % L,
                   levels=[Level(blocks=b, values=f.reshape(1, len(b), nb, nb, nb))])


def ring_level(dx, nb, k_sigma, R=1.0, sigma=0.1, dR=None, half_width=2.0,
               components=(0, 1, 2)):
    """One level of the ring: blocks within k_sigma*sigma of the core."""
    box_cells = int(round(2 * half_width * R / dx))
    lo = (-half_width * R,) * 3
    blocks = blocks_near_core(nb, dx, lo, box_cells,
                              lambda p: ring_core_distance(p, R, dR)[0],
                              k_sigma * sigma)
    comps = list(components)
    lv = _level_from_fn(blocks, nb, dx, lo,
                        lambda p: ring_vorticity(p, R, sigma, dR)[comps], len(comps))
    return lv, lo


def single_ring(dx=1.0 / 32, nb=16, k_sigma=8.0, components=(0, 1, 2)):
    """Vector Poisson source of a thin ring on one level (R=1, sigma=0.1R)."""
    lv, lo = ring_level(dx, nb, k_sigma, components=components)
    return Problem(nb=nb, dx0=dx, levels=[lv], name="ring_R/%d" % round(1 / dx),
                   meta={"origin": lo})


def two_level_ring(nb=16, dx0=1.0 / 32, k_coarse=8.0, k_fine=3.0, seed=3,
                   components=(0, 1, 2)):
    """Coarse ring support at dx0, fine level at dx0/2 near the perturbed core."""
    dR = ring_radius_perturbation(seed)
    comps = list(components)
    lo = (-2.0,) * 3
    coarse_blocks = blocks_near_core(nb, dx0, lo, int(round(4 / dx0)),
                                     lambda p: ring_core_distance(p)[0], k_coarse * 0.1)
    dx1 = dx0 / 2
    fine_blocks = blocks_near_core(nb, dx1, lo, int(round(4 / dx1)),
                                   lambda p: ring_core_distance(p, 1.0, dR)[0], k_fine * 0.1)
    fn = lambda p: ring_vorticity(p, 1.0, 0.1, dR)[comps]
    lv0 = _level_from_fn(coarse_blocks, nb, dx0, lo, fn, len(comps))
    lv1 = _level_from_fn(fine_blocks, nb, dx1, lo, fn, len(comps))
    return Problem(nb=nb, dx0=dx0, levels=[lv0, lv1], name="two_level_ring",
                   meta={"origin": lo})


def _rot_y(deg):
    a = np.deg2rad(deg)
    c, s = np.cos(a), np.sin(a)
    return np.array([[c, 0.0, s], [0.0, 1.0, 0.0], [-s, 0.0, c]])


def _ring_frames(sep=3.0, tilt=15.0):
    """Two coaxial rings at z = -+sep/2, each tilted about y toward the other."""
    return [(np.array([0.0, 0.0, -sep / 2]), _rot_y(-tilt)), (np.array([0.0, 0.0, sep / 2]), _rot_y(tilt))]


def two_ring_distance(p, dRs, R=1.0):
    """Distance to the nearer of the two (perturbed, tilted) ring cores."""
    d = None
    for (ctr, Q), dR in zip(_ring_frames(), dRs):
        loc = (p - ctr) @ Q            # into the ring's own frame (axis z)
        s, _ = ring_core_distance(loc, R, dR)
        d = s if d is None else np.minimum(d, s)
    return d


def two_ring_vorticity(p, dRs, R=1.0, sigma=0.1):
    """Sum of the two rings' azimuthal Gaussian-core vorticity (world frame)."""
    w = 0.0
    for (ctr, Q), dR in zip(_ring_frames(), dRs):
        loc = (p - ctr) @ Q
        wl = ring_vorticity(loc, R, sigma, dR)            # (3, ...) in the ring frame
        w = w + np.einsum("ij,j...->i...", Q, wl)
    return w


def _blocks_within(nb, dx, lo, hi, dist_fn, cutoff, bound_fn=None, slack=0.0):
    """Blocks of the box [lo, hi) with any cell centre within `cutoff`.

    A block can only qualify if its centre is within cutoff plus the
    centre-to-corner-cell distance, so candidates are prefiltered at block
    centres.  If `bound_fn` differs from `dist_fn` by at most `slack`
    everywhere, blocks it decides clearly are settled without `dist_fn`.
    """
    lo_b = np.floor(np.asarray(lo) / (nb * dx)).astype(int)
    hi_b = np.ceil(np.asarray(hi) / (nb * dx)).astype(int)
    axes = [np.arange(lo_b[a], hi_b[a]) for a in range(3)]
    BZ, BY, BX = np.meshgrid(axes[2], axes[1], axes[0], indexing="ij")
    cand = np.stack([BX.ravel(), BY.ravel(), BZ.ravel()], axis=1)
    ctr = (cand + 0.5) * nb * dx
    reach = cutoff + slack + np.sqrt(3.0) * 0.5 * (nb - 1) * dx + 1e-12
    cand = cand[(bound_fn or dist_fn)(ctr) <= reach]
    r = (np.arange(nb) + 0.5) * dx
    out = []
    for b in cand:
        X, Y, Z = np.meshgrid(b[0] * nb * dx + r, b[1] * nb * dx + r, b[2] * nb * dx + r, indexing="ij")
        pts = np.stack([X, Y, Z], axis=-1)
        if bound_fn is not None:
            m = bound_fn(pts).min()
            if m > cutoff + slack:
                continue
            if m <= cutoff - slack:
                out.append((int(b[0]), int(b[1]), int(b[2])))
                continue
        if dist_fn(pts).min() <= cutoff:
            out.append((int(b[0]), int(b[1]), int(b[2])))
    return out


def colliding_rings(nb=16, dx0=1.0 / 32, k_fine=4.0, k_coarse=8.0, seeds=(5, 6), components=(0, 1, 2),
                    with_values=True):
    """Three levels around two colliding rings (R = 1, sigma = 0.1 R).

    Finest level (dx0/4): blocks within k_fine sigma of either perturbed core.
    Level 1 (dx0/2): parents of the finest blocks dilated by one block.
    Level 0 (dx0): blocks within k_coarse sigma, plus the parents of level 1
    dilated by one block.  Block coordinates are on the lattice with origin 0.
    """
    dRs = [ring_radius_perturbation(sd) for sd in seeds]
    dist = lambda p: two_ring_distance(p, dRs)
    # the unperturbed distance differs from the perturbed one by at most
    # max|dR| = 0.01 R (the core moves by dR within its plane)
    bound = lambda p: two_ring_distance(p, [None, None])
    ext = (np.array([-2.4, -2.4, -3.0]), np.array([2.4, 2.4, 3.0]))
    fine = _blocks_within(nb, dx0 / 4, ext[0], ext[1], dist, k_fine * 0.1, bound, 0.0100001)

    def parents_dilated(blocks):
        par = {(b[0] // 2, b[1] // 2, b[2] // 2) for b in blocks}
        out = set(par)
        for b in par:
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dxb in (-1, 0, 1):
                        out.add((b[0] + dxb, b[1] + dy, b[2] + dz))
        return out
    mid = sorted(parents_dilated(fine), key=lambda t: (t[2], t[1], t[0]))
    coarse = set(_blocks_within(nb, dx0, ext[0], ext[1], dist, k_coarse * 0.1, bound, 0.0100001)) | \
        parents_dilated(mid)
    coarse = sorted(coarse, key=lambda t: (t[2], t[1], t[0]))
    comps = list(components)
    fn = lambda q: two_ring_vorticity(q, dRs)[comps]
    levels = []
    for k, blocks in enumerate([coarse, mid, fine]):
        b = np.asarray(blocks, dtype=np.int32).reshape(-1, 3)
        if with_values:
            levels.append(_level_from_fn(b, nb, dx0 / 2 ** k, (0.0, 0.0, 0.0), fn, len(comps)))
        else:
            levels.append(Level(blocks=b, values=np.zeros((0, len(b), nb, nb, nb))))
    return Problem(nb=nb, dx0=dx0, levels=levels, name="colliding_rings",
                   meta={"origin": (0.0, 0.0, 0.0)})


def mstar(components=(0,)):
    """Dense 256^3 box, dx = R/64 over [-2R, 2R]^3, 16^3 blocks (4096 blocks)."""
    nb, n_blk, dx = 16, 16, 1.0 / 64
    b = np.array([(x, y, z) for z in range(n_blk) for y in range(n_blk)
                  for x in range(n_blk)], dtype=np.int32)
    comps = list(components)
    lo = (-2.0,) * 3
    lv = _level_from_fn(b, nb, dx, lo, lambda p: ring_vorticity(p)[comps], len(comps))
    return Problem(nb=nb, dx0=dx, levels=[lv], name="dense_256^3_ring_x",
                   meta={"origin": lo})


def blob_cube(L, nb, rng, n_blobs=None):
    """Dense cube of side L cells with 1-4 Gaussian blobs (sigma 2-6 cells)."""
    n_blk = L // nb
    b = np.array([(x, y, z) for z in range(n_blk) for y in range(n_blk)
                  for x in range(n_blk)], dtype=np.int32)
    c = cell_coords(b, nb).astype(np.float64) + 0.5
    k = int(rng.integers(1, 5)) if n_blobs is None else n_blobs
    f = np.zeros(len(c))
    for _ in range(k):
        ctr = rng.uniform(0.0, L, 3)
        sg = rng.uniform(2.0, 6.0)
        amp = rng.normal()
        f += amp * np.exp(-((c - ctr) ** 2).sum(axis=1) / (2.0 * sg * sg))
    return Problem(nb=nb, dx0=1.0, name="blobs_%d" % L,
                   levels=[Level(blocks=b, values=f.reshape(1, len(b), nb, nb, nb))])


@dataclass
class Request:
    rid: int
    problem: Problem
    precision: str            # "fp64" or "fp32_refine"
    arrival: float            # seconds, relative to stream start


def served_stream(n_requests=512, seed=4, rate=None, sizes=None, nb=8):
    """Independent dense-cube solves, side L uniform in {16, 24, ..., 128}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = list(range(16, 129, 8)) if sizes is None else list(sizes)
    out = []
    t = 0.0
    for i in range(n_requests):
        L = int(sizes[int(rng.integers(0, len(sizes)))])
        prob = blob_cube(L, nb, rng)
        prec = "fp64" if rng.uniform() < 0.5 else "fp32_refine"
        gap = rng.exponential(1.0)
        t += gap / rate if rate else 0.0
        out.append(Request(rid=i, problem=prob, precision=prec, arrival=t))
    return out
