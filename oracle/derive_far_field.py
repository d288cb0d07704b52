"""Symbolic derivation of the far-field expansion of the 7-point LGF.

Oracle provenance script (test infrastructure).  The paper tabulates the
LGF near the origin and uses an asymptotic expansion far from it (Sec. 5,
Implementation) but does not print the expansion; this script derives it
from the Fourier symbol of the 7-point operator.

Derivation.  With (L g)(n) = sum_{+-e_i} g(n +- e_i) - 6 g(n) and L G = delta,

    G(n) = -(2 pi)^-3 \\int_{[-pi,pi]^3} e^{i n.theta} / sigma(theta) dtheta,
    sigma(theta) = sum_i 4 sin^2(theta_i / 2)
                 = |theta|^2 - s4/12 + s6/360 - s8/20160 + ...,

with s_{2m} = sum_i theta_i^{2m}.  Expanding 1/sigma = |theta|^-2 sum_k eps^k
and grouping by homogeneity gives terms P(theta)/|theta|^{2k}.  Each is
transformed with the inverse Fourier pairs

    1/|theta|^2 -> 1/(4 pi r),   1/|theta|^4 -> -r/(8 pi),
    1/|theta|^6 -> r^3/(96 pi),  1/|theta|^8 -> -r^5/(2880 pi),

(each follows from the previous one through -Laplacian <-> |theta|^2) and
theta_i^{2m} -> (-1)^m d^{2m}/dx_i^{2m}.  The result is

    G(n) ~ -[ 1/(4 pi r) + Q4/(16 pi r^7) + Q8/(128 pi r^13)
              + Q12/(512 pi r^19) ].

Running this module prints the polynomials Q4, Q8, Q12; the oracle's
``lgf_table.far_field`` and the C direct sum use the printed coefficients,
and ``tests/test_oracle_lgf.py`` re-runs the derivation and compares.
"""
import sympy as sp

x, y, z = sp.symbols("x y z", real=True)
T1, T2, T3, lam = sp.symbols("T1 T2 T3 lam")
r = sp.sqrt(x**2 + y**2 + z**2)

E = {
    1: 1 / (4 * sp.pi * r),
    2: -r / (8 * sp.pi),
    3: r**3 / (96 * sp.pi),
    4: -r**5 / (2880 * sp.pi),
}


def derive(n_terms=4):
    """Return the list [F0, F2, F4, F6] with F^-1[1/sigma] ~ sum F_j."""
    def four_sin2(t):
        return sp.series(4 * sp.sin(t / 2) ** 2, t, 0, 10).removeO()

    sig = sum(four_sin2(lam * T) for T in (T1, T2, T3))
    s2 = lam**2 * (T1**2 + T2**2 + T3**2)
    eps = sp.expand((s2 - sig) / s2)
    geo = sp.expand(sum(eps**k for k in range(n_terms)))
    geo = sp.expand(sp.series(geo, lam, 0, 2 * n_terms - 1).removeO())
    out = []
    for deg in range(0, 2 * n_terms, 2):
        c = geo.coeff(lam, deg)
        m = deg // 2
        num = sp.cancel(sp.expand(c * (T1**2 + T2**2 + T3**2) ** m))
        numP = sp.Poly(sp.expand(num), T1, T2, T3)
        k = m + 1
        acc = 0
        for (a, b, cc), coef in numP.terms():
            p = (a + b + cc) // 2
            d = sp.diff(E[k], x, a, y, b, z, cc) if (a or b or cc) else E[k]
            acc += coef * (-1) ** p * d
        out.append(sp.factor(sp.simplify(acc)))
    return out


def numerator_coefficients(expr, power, denom):
    """Split F = Q(x,y,z) / (denom * pi * r^power); return {monomial: coef}."""
    q = sp.simplify(expr * denom * sp.pi * r**power)
    return {m: int(c) for m, c in sp.Poly(sp.expand(q), x, y, z).terms()}


if __name__ == "__main__":
    terms = derive()
    for t in terms:
        print(t)
