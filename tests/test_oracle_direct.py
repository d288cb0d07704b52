"""Pins of the oracle direct sum against exact identities.

* point source reproduces dx^2 G(n - m);
* a compactly supported grid function Psi is recovered from its own 7-point
  Laplacian (G * L Psi = Psi because L G = delta and both decay) -- this is
  the manufactured-solution idea of the paper's Sec. 3.4 test, on one level;
* a library FFT convolution of the same table gives the same sum;
* translation invariance.
"""
import numpy as np
import scipy.fft as sfft

import pytest

from oracle import box, direct, lgf_table as T


def _grid(n0, n1, lo=(0, 0, 0)):
    ax = [np.arange(lo[i], lo[i] + (n1 if i else n0)) for i in range(3)]
    g = np.meshgrid(*ax, indexing="ij")
    return np.stack([a.ravel() for a in g], axis=1)


def test_point_source_gives_scaled_green_function():
    src = np.array([[3, -2, 5]])
    tgt = np.array([[3, -2, 5], [4, -2, 5], [10, 7, -3], [200, -100, 50], [3, -2, 140]])
    dx = 0.37
    u = direct.direct_sum(src, np.array([1.0]), tgt, dx)
    ref = dx * dx * T.G(tgt - src)
    assert np.max(np.abs(u - ref)) == 0.0


def _bump(c, R):
    """Compact bump exp(-10/(1-t^2)) (t = |x|/R < 1), the paper's f(t) shape."""
    t2 = (c ** 2).sum(axis=1) / (R * R)
    out = np.zeros(len(c))
    m = t2 < 1
    out[m] = 1e3 * np.exp(-10.0 / (1.0 - t2[m]))
    return out


def test_compact_function_recovered_from_its_laplacian():
    R = 9.0
    box = _grid(25, 25, lo=(-12, -12, -12))
    psi = _bump(box.astype(float), R)
    P = psi.reshape(25, 25, 25)
    lap = np.zeros_like(P)
    lap[1:-1, 1:-1, 1:-1] = (P[2:, 1:-1, 1:-1] + P[:-2, 1:-1, 1:-1] + P[1:-1, 2:, 1:-1]
                             + P[1:-1, :-2, 1:-1] + P[1:-1, 1:-1, 2:] + P[1:-1, 1:-1, :-2]
                             - 6 * P[1:-1, 1:-1, 1:-1])
    dx = 0.5
    omega = lap.ravel() / dx**2
    keep = omega != 0
    tgt = box[::7]
    u = direct.direct_sum(box[keep], omega[keep], tgt, dx)
    err = np.abs(u - psi[::7]).max() / np.abs(psi).max()
    assert err < 1e-13


def test_direct_sum_equals_fft_convolution():
    rng = np.random.default_rng(5)
    n = 12
    cells = _grid(n, n)
    f = rng.standard_normal(len(cells))
    u = direct.direct_sum(cells, f, cells, 1.0)
    Gc = T.G_cube(n - 1)                       # offsets -(n-1)..(n-1)
    F = f.reshape(n, n, n)
    M = 2 * n - 1
    full = sfft.irfftn(sfft.rfftn(F, (M + n - 1,) * 3) * sfft.rfftn(Gc, (M + n - 1,) * 3),
                       (M + n - 1,) * 3)
    ref = full[n - 1:2 * n - 1, n - 1:2 * n - 1, n - 1:2 * n - 1].ravel()
    assert np.max(np.abs(u - ref)) / np.abs(ref).max() < 1e-13


def test_translation_invariance():
    rng = np.random.default_rng(2)
    src = rng.integers(-20, 20, size=(50, 3))
    f = rng.standard_normal(50)
    tgt = rng.integers(-60, 60, size=(40, 3))
    sh = np.array([17, -33, 91])
    a = direct.direct_sum(src, f, tgt, 1.0)
    b = direct.direct_sum(src + sh, f, tgt + sh, 1.0)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("shape", [(5, 7, 9), (140, 3, 4), (3, 131, 2)])
def test_fft_box_convolution_equals_direct_sum(shape):
    """The oracle's zero-padded FFT over a box (used for full psi fields of
    large composite meshes) against the direct sum, across the near/far
    switch of the table (extents past 129 cells)."""
    rng = np.random.default_rng(sum(shape))
    f = rng.standard_normal(shape)
    ax = [np.arange(n) for n in shape]
    cells = np.stack([a.ravel() for a in np.meshgrid(*ax, indexing="ij")], axis=1)
    u = box.convolve_box(f, 0.3)
    ref = direct.direct_sum(cells, f.ravel(), cells, 0.3)
    assert np.max(np.abs(u.ravel() - ref)) / np.abs(ref).max() < 1e-13
    sub = rng.choice(len(cells), 40, replace=False)
    got = box.convolve_cells(cells[sub] + 11, f.ravel()[sub], cells - 7, 0.3)
    ref2 = direct.direct_sum(cells[sub] + 11, f.ravel()[sub], cells - 7, 0.3)
    assert np.max(np.abs(got - ref2)) / np.abs(ref2).max() < 1e-13
