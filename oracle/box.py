"""Whole-box LGF convolution by a zero-padded FFT (test infrastructure).

The definition u(n) = dx^2 * sum_m G(n - m) f(m) (paper Sec. 2.2, eq.
lgf_convolution) over a box of n_0 x n_1 x n_2 cells is a linear
convolution; embedding the source in a grid of 2 n_i cells per axis and
G(d), |d_i| <= n_i - 1, circularly in the same grid makes the circular
convolution of a library FFT equal to it (up to rounding).  The composite
oracle uses this for full fields (the psi_k of Sec. 3.4) where a direct sum
over millions of targets is out of reach; G comes from ``lgf_table`` (the
same near table and far series as the direct sum).  Pinned against the
direct sum and through the composite oracle's closed-form pins.
"""
import numpy as np
import scipy.fft as sfft

from . import lgf_table

_KERNELS = {}


def _workers():
    import os
    return max(1, min(16, os.cpu_count() or 1))


def _octant(shape):
    """G(a, b, c) for 0 <= a < n_0, 0 <= b < n_1, 0 <= c < n_2."""
    n0, n1, n2 = shape
    out = np.empty(shape)
    C = lgf_table.near_cube()
    R = lgf_table.R_NEAR
    b = np.arange(n1)[:, None]
    c = np.arange(n2)[None, :]
    B, Cc = np.broadcast_arrays(b, c)
    for a in range(n0):                       # one plane at a time bounds the memory
        pts = np.stack([np.full(B.shape, a), B, Cc], axis=-1)
        inside = pts.max(axis=-1) <= R
        plane = np.empty(B.shape)
        q = pts[inside]
        plane[inside] = C[q[:, 0], q[:, 1], q[:, 2]]
        plane[~inside] = lgf_table.far_field(pts[~inside])
        out[a] = plane
    return out


def kernel_spectrum(shape):
    """rfftn of G laid circularly on the (2 n_0, 2 n_1, 2 n_2) grid."""
    key = tuple(int(v) for v in shape)
    if key in _KERNELS:
        return _KERNELS[key]
    g = _octant(key)
    # grid index i holds offset i (i < n) or i - 2n (i > n); index n is an
    # offset that never occurs between two cells of the box
    wrap = [np.concatenate([np.arange(n), [0], np.arange(n - 1, 0, -1)]) for n in key]
    kern = g[np.ix_(*wrap)]
    kern[key[0]] = 0.0
    kern[:, key[1]] = 0.0
    kern[:, :, key[2]] = 0.0
    del g
    spec = sfft.rfftn(kern, workers=_workers())
    del kern
    if len(_KERNELS) >= 2:
        _KERNELS.pop(next(iter(_KERNELS)))
    _KERNELS[key] = spec
    return spec


def convolve_box(f, dx=1.0):
    """u = dx^2 * G * f on the box of the dense array f (any shape n_0 x n_1 x n_2)."""
    f = np.asarray(f, dtype=np.float64)
    shape = f.shape
    grid = tuple(2 * n for n in shape)
    spec = kernel_spectrum(shape)
    u = sfft.irfftn(sfft.rfftn(f, grid, workers=_workers()) * spec, grid, workers=_workers())
    return dx * dx * u[:shape[0], :shape[1], :shape[2]]


def convolve_cells(src_cells, src_vals, tgt_cells, dx=1.0):
    """u at tgt_cells of dx^2 G * (sources at src_cells), over their bounding box."""
    src = np.asarray(src_cells, dtype=np.int64).reshape(-1, 3)
    tgt = np.asarray(tgt_cells, dtype=np.int64).reshape(-1, 3)
    lo = np.minimum(src.min(axis=0), tgt.min(axis=0))
    hi = np.maximum(src.max(axis=0), tgt.max(axis=0)) + 1
    f = np.zeros(tuple((hi - lo).tolist()))
    s = src - lo
    np.add.at(f, (s[:, 0], s[:, 1], s[:, 2]), np.asarray(src_vals, dtype=np.float64))
    u = convolve_box(f, dx)
    t = tgt - lo
    return u[t[:, 0], t[:, 1], t[:, 2]]
