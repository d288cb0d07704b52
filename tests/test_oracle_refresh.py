"""Pins of the velocity-refresh oracle (paper Sec. 4.1, eq. vel_update).

* C^dagger is the adjoint of C (eq. mimetic): <C u, p> = <u, C^dagger p>
  for compact fields;
* D C^dagger = 0 and C G = 0 (a curl has no divergence, a gradient no curl);
* a compact edge field A gives a compact divergence-free velocity
  u = C^dagger A and vorticity omega = C u; since C C^dagger = G D - L_E on
  edges and C^dagger G = 0, -C^dagger L_E^-1 omega returns u exactly.  A sign
  error, a forward difference in place of a backward one, or an index
  shift in either curl fails this.
"""
import numpy as np

from oracle import refresh


def _bump3(shape, ctr, R, seed):
    ax = [np.arange(n) + 0.5 for n in shape]
    X, Y, Z = np.meshgrid(*ax, indexing="ij")
    out = []
    rng = np.random.default_rng(seed)
    for c in range(3):
        cc = np.asarray(ctr) + rng.uniform(-1.5, 1.5, 3)
        t2 = ((X - cc[0]) ** 2 + (Y - cc[1]) ** 2 + (Z - cc[2]) ** 2) / R ** 2
        f = np.zeros(shape)
        m = t2 < 1
        f[m] = rng.uniform(0.5, 2.0) * np.exp(-4.0 / (1.0 - t2[m]))
        out.append(f)
    return np.stack(out)


def test_backward_curl_is_adjoint_of_forward_curl():
    rng = np.random.default_rng(0)
    shape = (9, 10, 11)
    u = np.zeros((3,) + shape)
    p = np.zeros((3,) + shape)
    u[:, 2:-2, 2:-2, 2:-2] = rng.standard_normal((3, 5, 6, 7))
    p[:, 2:-2, 2:-2, 2:-2] = rng.standard_normal((3, 5, 6, 7))
    lhs = (refresh.curl_forward(u, 0.7) * p).sum()
    rhs = (u * refresh.curl_backward(p, 0.7)).sum()
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_curl_of_gradient_and_divergence_of_curl_vanish():
    rng = np.random.default_rng(1)
    s = rng.standard_normal((12, 12, 12))
    g = np.stack([np.roll(s, -1, 0) - s, np.roll(s, -1, 1) - s, np.roll(s, -1, 2) - s])   # G: cells -> faces
    w = refresh.curl_forward(g, 1.0)[:, 1:-2, 1:-2, 1:-2]
    assert np.abs(w).max() < 1e-12
    p = rng.standard_normal((3, 12, 12, 12))
    u = refresh.curl_backward(p, 1.0)
    div = (u[0] - np.roll(u[0], 1, 0)) + (u[1] - np.roll(u[1], 1, 1)) + (u[2] - np.roll(u[2], 1, 2))   # D: faces -> cells
    assert np.abs(div[2:-1, 2:-1, 2:-1]).max() < 1e-12


def test_refresh_recovers_compact_divergence_free_velocity():
    shape, dx = (26, 26, 26), 0.25
    A = _bump3(shape, (13, 13, 13), 6.0, seed=3)
    u = refresh.curl_backward(A, dx)
    w = refresh.curl_forward(u, dx)
    ax = [np.arange(n) for n in shape]
    cells = np.stack([a.ravel() for a in np.meshgrid(*ax, indexing="ij")], axis=1)
    keep = np.any(w.reshape(3, -1) != 0, axis=0)
    tgt = cells[np.random.default_rng(4).choice(len(cells), 300, replace=False)]
    got = refresh.velocity_refresh(cells[keep], w.reshape(3, -1)[:, keep], tgt, dx)
    want = u[:, tgt[:, 0], tgt[:, 1], tgt[:, 2]]
    assert np.abs(got - want).max() < 1e-12 * np.abs(u).max()
    assert np.abs(want).max() > 0.1 * np.abs(u).max()       # the sample sees the field
