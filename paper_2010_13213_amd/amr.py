"""Adaptive refinement on block-structured levels (paper Sec. 3.4 test and
Sec. 4.2).

* ``refine_by_field``: the level hierarchy of the manufactured-solution test
  (Sec. 3.4): a region on level k is refined where |w| exceeds
  alpha^(L_R - k) * max|w| (L_R = number of refinements, alpha = 1/6 there).
  A level-(k+1) block is created for every octant of a level-k block that
  holds such a cell, so level k+1 is properly nested in level k.
* ``indicator_flags``: the criterion of eqs. refine1 / maximumS / refine2 on
  per-block statistics of the combined source S_k (lgf_solve_indicator):
  refine a block when max |S_k| over it exceeds alpha^(N_l - k) S_max,
  coarsen it when that maximum is below beta alpha^(N_l - k) S_max, where
  S_max is the largest block RMS of S_k seen so far (the caller keeps the
  running maximum over time).
* ``manufactured_ring``: the streamfunction Psi = f(d / R) e_theta of the
  Sec. 3.4 test, f(t) = c1 exp(-c2 / (1 - t^2)) for |t| < 1, d the distance
  to the ring core, and its vector Laplacian omega = (Lap psi - psi / rho^2)
  e_theta in closed form.

Only geometry and bookkeeping here; every solve runs through the library.
"""
import numpy as np

from . import inputs


def manufactured_ring(p, R=0.125, c1=1e3, c2=10.0):
    """(Psi, omega) at points p (..., 3): 3-vectors (x, y, z) each, shape (3, ...)."""
    x, y, z = p[..., 0], p[..., 1], p[..., 2]
    rho = np.sqrt(x * x + y * y)
    d = np.sqrt((rho - R) ** 2 + z * z)
    t = d / R
    inside = t < 1.0
    ts = np.where(inside, t, 0.0)
    q = 1.0 - ts * ts
    f = np.where(inside, c1 * np.exp(-c2 / q), 0.0)
    g1 = -2.0 * c2 * ts / (q * q)                           # (log f)'
    g2 = -2.0 * c2 * (1.0 + 3.0 * ts * ts) / q ** 3          # (log f)''
    f1 = f * g1                                            # df/dt
    f2 = f * (g1 * g1 + g2)                                # d2f/dt2
    rho_s = np.where(rho > 0, rho, 1.0)
    d_s = np.where(d > 0, d, 1.0)
    # Lap(psi) in the meridional plane about the core, plus the 1/rho d/drho
    # term of the cylindrical Laplacian and the -psi/rho^2 of the vector one
    lap = f2 / R ** 2 + f1 / (R * d_s) + f1 * (rho - R) / (R * d_s * rho_s) - f / rho_s ** 2
    lap = np.where(inside, lap, 0.0)
    ex, ey = -y / rho_s, x / rho_s                         # e_theta
    psi = np.stack([f * ex, f * ey, np.zeros_like(f)])
    om = np.stack([lap * ex, lap * ey, np.zeros_like(f)])
    return psi, om


def _cells_centres(blocks, nb, dx, origin):
    return inputs.cell_centres(blocks, nb, dx, origin).reshape(-1, 3)


def refine_by_field(field_fn, nb, dx0, base_blocks, n_refine, alpha, origin=(0.0, 0.0, 0.0)):
    """Level block lists (coarsest first) from |field_fn| thresholds.

    field_fn(points (n, 3)) -> (n,) magnitudes; base_blocks: level-0 blocks.
    max|w| is taken over the cells of every level as they are built."""
    levels = [np.asarray(base_blocks, dtype=np.int32).reshape(-1, 3)]
    vals = [field_fn(_cells_centres(levels[0], nb, dx0, origin))]
    for k in range(n_refine):
        wmax = max(float(np.max(v)) for v in vals)
        thr = alpha ** (n_refine - k) * wmax
        b = levels[k]
        v = vals[k].reshape(len(b), nb, nb, nb)               # [block][z][y][x]
        h = nb // 2
        new = set()
        for oz in range(2):
            for oy in range(2):
                for ox in range(2):
                    hot = (v[:, oz * h:(oz + 1) * h, oy * h:(oy + 1) * h, ox * h:(ox + 1) * h] > thr).any(axis=(1, 2, 3))
                    for bb in b[hot]:
                        new.add((2 * int(bb[0]) + ox, 2 * int(bb[1]) + oy, 2 * int(bb[2]) + oz))
        if not new:
            break
        fine = np.array(sorted(new, key=lambda t: (t[2], t[1], t[0])), dtype=np.int32)
        levels.append(fine)
        vals.append(field_fn(_cells_centres(fine, nb, dx0 / 2 ** (k + 1), origin)))
    return levels


def indicator_flags(block_max, k, n_levels, s_max, alpha, beta):
    """+1 refine / -1 coarsen / 0 keep per block of level k (eqs. refine1, refine2).

    block_max: max |S_k| over each block; s_max: the running maximum of the
    block RMS of S_k (eq. maximumS); n_levels: the prescribed maximum level
    N_l."""
    thr = alpha ** (n_levels - k) * s_max
    m = np.asarray(block_max, dtype=np.float64)
    return np.where(m > thr, 1, np.where(m < beta * thr, -1, 0)).astype(np.int8)
