"""Oracle of the velocity refresh u = -C^dagger L_E^-1 omega on one level
(paper Sec. 4.1, eq. vel_update) -- test infrastructure.

Staggering (paper Sec. 2.1: cells and vertices hold scalars, the positive
faces and edges of each cell hold vectors).  Reading: cell n = (i, j, k)
owns the x-face at n + e_x/2 and the x-edge at n + (e_y + e_z)/2 (likewise
for y and z), so every component is a field on its own copy of the cell
lattice, and array index [i, j, k] of a component is the face / edge that
cell owns.

* C (faces -> edges) is the curl with forward differences:
  (C u)_x[n] = (u_z[n + e_y] - u_z[n] - u_y[n + e_z] + u_y[n]) / dx, and
  cyclically.
* C^dagger (edges -> faces), its adjoint (eq. mimetic), is the curl with
  backward differences:
  (C^dagger p)_x[n] = (p_z[n] - p_z[n - e_y] - p_y[n] + p_y[n - e_z]) / dx.
* L_E is the 7-point Laplacian on each edge component's lattice, so
  L_E^-1 omega is the LGF convolution dx^2 G * omega_c of every component.
"""
import numpy as np

from . import direct

_AX = {"x": 0, "y": 1, "z": 2}


def curl_forward(u, dx):
    """C u on the interior of a (3, nx, ny, nz) box array (forward differences;
    the last plane along each differenced axis is left 0)."""
    ux, uy, uz = u
    w = np.zeros_like(u)
    w[0, :, :-1, :-1] = (uz[:, 1:, :-1] - uz[:, :-1, :-1]) - (uy[:, :-1, 1:] - uy[:, :-1, :-1])
    w[1, :-1, :, :-1] = (ux[:-1, :, 1:] - ux[:-1, :, :-1]) - (uz[1:, :, :-1] - uz[:-1, :, :-1])
    w[2, :-1, :-1, :] = (uy[1:, :-1, :] - uy[:-1, :-1, :]) - (ux[:-1, 1:, :] - ux[:-1, :-1, :])
    return w / dx


def curl_backward(p, dx):
    """C^dagger p on the interior of a (3, nx, ny, nz) box array (backward
    differences; the first plane along each differenced axis is left 0)."""
    px, py, pz = p
    u = np.zeros_like(p)
    u[0, :, 1:, 1:] = (pz[:, 1:, 1:] - pz[:, :-1, 1:]) - (py[:, 1:, 1:] - py[:, 1:, :-1])
    u[1, 1:, :, 1:] = (px[1:, :, 1:] - px[1:, :, :-1]) - (pz[1:, :, 1:] - pz[:-1, :, 1:])
    u[2, 1:, 1:, :] = (py[1:, 1:, :] - py[:-1, 1:, :]) - (px[1:, 1:, :] - px[1:, :-1, :])
    return u / dx


def velocity_refresh(src_cells, omega, tgt_cells, dx):
    """u = -C^dagger L_E^-1 omega at target cells (3, n_tgt).

    omega: (3, n_src) edge vorticity at src_cells; the streamfunction
    psi_c = dx^2 G * omega_c is evaluated by direct sums at every target
    and at its three backward neighbours."""
    src = np.asarray(src_cells, dtype=np.int64).reshape(-1, 3)
    tgt = np.asarray(tgt_cells, dtype=np.int64).reshape(-1, 3)
    e = np.eye(3, dtype=np.int64)
    pts = np.concatenate([tgt, tgt - e[0], tgt - e[1], tgt - e[2]])
    psi = np.stack([direct.direct_sum(src, omega[c], pts, dx) for c in range(3)])
    n = len(tgt)
    at = lambda c, s: psi[c, s * n:(s + 1) * n]          # s = 0: n, 1: n - e_x, 2: n - e_y, 3: n - e_z
    px, py, pz = 0, 1, 2
    cx = (at(pz, 0) - at(pz, 2)) - (at(py, 0) - at(py, 3))
    cy = (at(px, 0) - at(px, 3)) - (at(pz, 0) - at(pz, 1))
    cz = (at(py, 0) - at(py, 1)) - (at(px, 0) - at(px, 2))
    return -np.stack([cx, cy, cz]) / dx
