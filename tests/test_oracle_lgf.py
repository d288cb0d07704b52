"""Pins of the oracle LGF table against closed forms and invariants.

None of these compare the oracle with itself: each checks a value or an
identity fixed by the mathematics (Watson's integral, the lattice equation
L G = delta, the continuum limit, symmetry, an independently derived
asymptotic series, an independent high-precision Bessel evaluation).
"""
import math

import numpy as np
import pytest

from oracle import direct, lgf_table as T


def test_G0_matches_watson_closed_form():
    # G(0) = -W/6 with W = sqrt(6)/(32 pi^3) Gamma(1/24)Gamma(5/24)Gamma(7/24)Gamma(11/24)
    g0 = T.near_cube()[0, 0, 0]
    assert abs(g0 - T.watson_G0()) < 1e-14
    assert abs(g0 - (-0.2527310098586630)) < 1e-14


def test_G100_from_lattice_equation_at_origin():
    # (L G)(0) = 6 G(1,0,0) - 6 G(0) = 1 by symmetry.
    C = T.near_cube()
    assert abs(C[1, 0, 0] - C[0, 0, 0] - 1.0 / 6.0) < 1e-14


def test_lattice_laplacian_of_G_is_delta_across_near_far_switch():
    R = T.R_NEAR + 8
    Gc = T.G_cube(R)
    L = (Gc[2:, 1:-1, 1:-1] + Gc[:-2, 1:-1, 1:-1] + Gc[1:-1, 2:, 1:-1]
         + Gc[1:-1, :-2, 1:-1] + Gc[1:-1, 1:-1, 2:] + Gc[1:-1, 1:-1, :-2]
         - 6.0 * Gc[1:-1, 1:-1, 1:-1])
    L[R - 1, R - 1, R - 1] -= 1.0
    assert np.abs(L).max() < 1e-13


def test_far_field_leading_term_is_continuum_greens_function():
    for n in [(300, 0, 0), (200, 150, 90), (400, 400, 400)]:
        r = math.sqrt(sum(v * v for v in n))
        assert abs(T.G(np.array(n))[()] * 4 * math.pi * r + 1.0) < 1e-4
    # and the exact integral approaches it too
    e = T.g_exact((100, 60, 20))
    r = math.sqrt(100**2 + 60**2 + 20**2)
    assert abs(e * 4 * math.pi * r + 1.0) < 1e-4


@pytest.mark.parametrize("n", [(20, 0, 0), (40, 0, 0), (64, 0, 0), (24, 24, 24),
                               (40, 20, 10)])
def test_far_field_series_orders(n):
    """Truncating after j corrections leaves an error O(|n|^-(2j+2))."""
    n = np.array(n)
    e1 = T.g_exact(n)
    e2 = T.g_exact(2 * n)
    for j, slope in enumerate([2, 4, 6, 8]):
        r1 = abs(T.far_field(n, j) - e1) / abs(e1)
        r2 = abs(T.far_field(2 * n, j) - e2) / abs(e2)
        if r2 < 5e-14:     # near the quadrature accuracy: no order information
            continue
        ratio = r1 / r2
        assert 2 ** slope * 0.6 < ratio < 2 ** slope * 1.7, (j, ratio)


def test_near_far_agree_at_switch_radius():
    R = T.R_NEAR
    pts = np.array([(R, 0, 0), (R, R, 0), (R, R, R), (R, 37, 5), (R, 90, 60)])
    near = np.array([T.g_exact(p) for p in pts])
    far = T.far_field(pts)
    assert np.max(np.abs(near - far) / np.abs(near)) < 5e-14


def test_symmetry_group_of_the_cube():
    rng = np.random.default_rng(0)
    for _ in range(20):
        n = rng.integers(-150, 151, size=3)
        ref = direct.G_points(n[None])[0]
        for perm in [(0, 1, 2), (1, 0, 2), (2, 1, 0), (0, 2, 1), (1, 2, 0), (2, 0, 1)]:
            for sgn in [(1, 1, 1), (-1, 1, 1), (1, -1, -1), (-1, -1, -1)]:
                m = np.array(sgn) * n[list(perm)]
                assert abs(direct.G_points(m[None])[0] - ref) <= 1e-14 * abs(ref)


def test_table_matches_independent_mpmath_quadrature():
    """Two entries recomputed with mpmath Bessel functions at 30 digits."""
    import mpmath as mp
    mp.mp.dps = 30

    def g_mp(n):
        h = mp.mpf("0.25")
        s = mp.mpf(0)
        u = mp.mpf(-40)
        while u <= 70:
            t = mp.e ** u
            x = 2 * t
            p = h * t
            for v in n:
                if x < 1e7:
                    p *= mp.besseli(v, x) * mp.e ** (-x)
                else:
                    mu = 4 * v * v
                    p *= (1 - (mu - 1) / (8 * x) + (mu - 1) * (mu - 9) / (128 * x * x)) \
                        / mp.sqrt(2 * mp.pi * x)
            s += p
            u += h
        s += 2 * (4 * mp.pi) ** mp.mpf(-1.5) / mp.sqrt(mp.e ** (70 + h / 2))
        return -s

    C = T.near_cube()
    for n in [(3, 2, 1), (9, 0, 4)]:
        ref = float(g_mp(n))
        assert abs(C[n] - ref) < 2e-15 * 10, (n, C[n], ref)


@pytest.mark.slow
def test_far_field_coefficients_rederived_symbolically():
    import sympy as sp
    from oracle import derive_far_field as D
    terms = D.derive()
    x, y, z = D.x, D.y, D.z
    r = D.r
    pts = [(3.0, 1.0, 2.0), (5.0, -2.0, 7.0), (1.0, 1.0, 1.0)]
    for p in pts:
        sub = dict(zip((x, y, z), p))
        rr = math.sqrt(sum(v * v for v in p))
        q4, q8, q12 = T._q_polys(*p)
        ours = [1 / (4 * math.pi * rr), q4 / (16 * math.pi * rr**7),
                q8 / (128 * math.pi * rr**13), q12 / (512 * math.pi * rr**19)]
        for t, o in zip(terms, ours):
            v = float(t.subs(sub))
            assert abs(v - o) <= 1e-12 * abs(o) + 1e-300
