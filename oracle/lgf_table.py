"""Oracle LGF of the 7-point Laplacian (test infrastructure; see package doc).

Conventions (the paper never writes G down -- Sec. 2.2, eq. lgf_convolution
only states phi = G * f with L phi = f and phi -> 0 at infinity):

* L is the unscaled 7-point operator (L g)(n) = sum_{+-e_i} g(n +- e_i) - 6 g(n).
* G solves L G = delta_0 and decays, so G < 0 and G(0) = -0.25273100985866...
* On a lattice of spacing dx the operator is dx^-2 L, so its inverse is
  dx^2 * (G * .).

Near field, |n|_inf <= R_NEAR: the Bessel-integral representation

    G(n) = - \\int_0^inf prod_i e^{-2t} I_{n_i}(2t) dt,

evaluated with the substitution t = e^u and the trapezoid rule in u on a
fine uniform grid (the integrand is analytic in a strip around the real u
axis, so the rule converges geometrically).  e^{-x} I_n(x) is SciPy's
``ive`` (a library primitive) for x <= 1e8; SciPy returns NaN beyond about
2e9, so larger arguments use Hankel's large-argument expansion
e^{-x} I_n(x) ~ (2 pi x)^{-1/2} sum_k (-1)^k a_k(n) / x^k,
a_k(n) = prod_{j<=k} (4 n^2 - (2j-1)^2) / (k! 8^k).

Far field, |n|_inf > R_NEAR: the asymptotic series derived in
``derive_far_field.py`` (Sec. 5 of the paper stores "asymptotic expansions
for far points").
"""
import functools
import math

import numpy as np
from scipy.special import ive

R_NEAR = 128          # exact near field for max|n_i| <= R_NEAR
_U_MIN, _U_MAX, _H = -50.0, 100.0, 0.1   # trapezoid grid in u = log t


_X_HANKEL = 1.0e8


def _ive_hankel(n, x):
    """Hankel expansion of e^{-x} I_n(x), accurate to ~1e-17 for x > 1e8."""
    n = np.asarray(n, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    mu = 4.0 * n * n
    term = np.ones(np.broadcast(n, x).shape)
    acc = term.copy()
    for k in range(1, 30):
        term = -term * (mu - (2 * k - 1) ** 2) / (k * 8.0 * x)
        acc = acc + term
        if np.all(np.abs(term) < 1e-19):
            break
    return acc / np.sqrt(2.0 * math.pi * x)


def ive_any(n, x):
    """e^{-x} I_n(x) for integer n >= 0 and any x >= 0 (broadcasting)."""
    n, x = np.broadcast_arrays(np.asarray(n, dtype=np.float64),
                               np.asarray(x, dtype=np.float64))
    out = np.empty(n.shape)
    small = x <= _X_HANKEL
    out[small] = ive(n[small], x[small])
    out[~small] = _ive_hankel(n[~small], x[~small])
    return out


def _nodes():
    u = np.arange(_U_MIN, _U_MAX + 0.5 * _H, _H)
    t = np.exp(u)
    w = _H * t                     # dt = e^u du
    return t, w


@functools.lru_cache(maxsize=4)
def _bessel_rows(nmax):
    """B[j, n] = e^{-2 t_j} I_n(2 t_j) for n = 0..nmax."""
    t, w = _nodes()
    n = np.arange(nmax + 1)
    B = ive_any(n[None, :], 2.0 * t[:, None])
    return t, w, B


def g_exact(n):
    """G(n) for one lattice point from the Bessel integral (any |n|)."""
    a = [abs(int(v)) for v in n]
    t, w = _nodes()
    prod = w.copy()
    for v in a:
        prod = prod * ive_any(v, 2.0 * t)
    return -float(np.sum(prod))


@functools.lru_cache(maxsize=2)
def near_cube(R=R_NEAR):
    """Dense table C[a, b, c] = G(a, b, c) for 0 <= a, b, c <= R.

    G is even in each coordinate and symmetric under permutations, so the
    cube indexed by |n_1|, |n_2|, |n_3| covers every point with
    max|n_i| <= R.  Each entry is the trapezoid sum
    -sum_j w_j B[j,a] B[j,b] B[j,c], formed as one matrix product per a.
    """
    t, w, B = _bessel_rows(R)
    C = np.empty((R + 1, R + 1, R + 1))
    for a in range(R + 1):
        Y = (w * B[:, a])[:, None] * B          # (nodes, R+1): w_j B_ja B_jb
        C[a] = -(Y.T @ B)                        # sum_j over nodes
    return C


# Coefficients of the far-field numerators (derive_far_field.py).
# Q4  = sum x^4 - 3 sum_{i<j} x_i^2 x_j^2
# Q8  = 23 sum x^8 - 244 sum_{i!=j} x_i^6 x_j^2 + 621 sum_{i<j} x_i^4 x_j^4
#       - 228 sum_i x_i^4 x_j^2 x_k^2
# Q12 = 647 sum x^12 - 16419 sum_{i!=j} x_i^10 x_j^2
#       + 106536 sum_{i!=j} x_i^8 x_j^4 - 15723 sum_i x_i^8 x_j^2 x_k^2
#       - 178221 sum_{i<j} x_i^6 x_j^6 - 74469 sum_{i,j,k distinct} x_i^6 x_j^4 x_k^2
#       + 626835 x^4 y^4 z^4
def _q_polys(x, y, z):
    x2, y2, z2 = x * x, y * y, z * z
    x4, y4, z4 = x2 * x2, y2 * y2, z2 * z2
    q4 = x4 + y4 + z4 - 3.0 * (x2 * y2 + y2 * z2 + z2 * x2)
    x6, y6, z6 = x4 * x2, y4 * y2, z4 * z2
    x8, y8, z8 = x4 * x4, y4 * y4, z4 * z4
    q8 = (23.0 * (x8 + y8 + z8)
          - 244.0 * (x6 * (y2 + z2) + y6 * (x2 + z2) + z6 * (x2 + y2))
          + 621.0 * (x4 * y4 + y4 * z4 + z4 * x4)
          - 228.0 * x2 * y2 * z2 * (x2 + y2 + z2))
    x10, y10, z10 = x8 * x2, y8 * y2, z8 * z2
    x12, y12, z12 = x6 * x6, y6 * y6, z6 * z6
    q12 = (647.0 * (x12 + y12 + z12)
           - 16419.0 * (x10 * (y2 + z2) + y10 * (x2 + z2) + z10 * (x2 + y2))
           + 106536.0 * (x8 * (y4 + z4) + y8 * (x4 + z4) + z8 * (x4 + y4))
           - 15723.0 * x2 * y2 * z2 * (x6 + y6 + z6)
           - 178221.0 * (x6 * y6 + y6 * z6 + z6 * x6)
           - 74469.0 * x2 * y2 * z2 * (x4 * (y2 + z2) + y4 * (x2 + z2) + z4 * (x2 + y2))
           + 626835.0 * x4 * y4 * z4)
    return q4, q8, q12


def far_field(n, n_corrections=3):
    """Asymptotic G(n) with the leading term and up to 3 corrections.

    ``n`` is an (..., 3) array of lattice points (any dtype); returns float64.
    """
    n = np.asarray(n, dtype=np.float64)
    x, y, z = n[..., 0], n[..., 1], n[..., 2]
    r2 = x * x + y * y + z * z
    r = np.sqrt(r2)
    q4, q8, q12 = _q_polys(x, y, z)
    g = 1.0 / (4.0 * math.pi * r)
    if n_corrections >= 1:
        g = g + q4 / (16.0 * math.pi * r ** 7)
    if n_corrections >= 2:
        g = g + q8 / (128.0 * math.pi * r ** 13)
    if n_corrections >= 3:
        g = g + q12 / (512.0 * math.pi * r ** 19)
    return -g


def G(n):
    """G at integer lattice points ``n`` (..., 3): table inside, series outside."""
    n = np.asarray(n, dtype=np.int64)
    a = np.abs(n)
    inside = a.max(axis=-1) <= R_NEAR
    out = np.empty(n.shape[:-1])
    C = near_cube()
    ai = a[inside]
    out[inside] = C[ai[..., 0], ai[..., 1], ai[..., 2]]
    out[~inside] = far_field(n[~inside])
    return out


def G_cube(R):
    """Dense G(n) for n in [-R, R]^3, indexed [n0 + R, n1 + R, n2 + R]."""
    ax = np.arange(-R, R + 1)
    n = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1)
    return G(n)


def watson_G0():
    """G(0) from Watson's closed form for the simple-cubic lattice integral.

    W = (sqrt 6 / (32 pi^3)) Gamma(1/24) Gamma(5/24) Gamma(7/24) Gamma(11/24)
    is (1/pi^3) \\int_{[0,pi]^3} dtheta / (1 - (cos th1 + cos th2 + cos th3)/3);
    with sigma = 2 (3 - sum cos) this gives G(0) = -W / 6.
    """
    import mpmath as mp
    mp.mp.dps = 30
    W = (mp.sqrt(6) / (32 * mp.pi ** 3)) * mp.gamma(mp.mpf(1) / 24) * \
        mp.gamma(mp.mpf(5) / 24) * mp.gamma(mp.mpf(7) / 24) * mp.gamma(mp.mpf(11) / 24)
    return float(-W / 6)
