"""Oracle of the integrating factor (test infrastructure).

Paper Sec. 2.3, eqs. heat / IF-single: the solution operator of the
discrete heat equation df/dt = kappa L f on the unbounded lattice is
H(a) = exp(a L) with a = kappa (t - tau) / dx^2 and L the unscaled 7-point
Laplacian.  Along one axis exp(a (S + S^-1 - 2)) = e^{-2a} sum_n I_n(2a) S^n
(the generating function of the modified Bessel functions), so H(a) is the
convolution with E(n) = prod_i e^{-2a} I_{n_i}(2a).  e^{-x} I_n(x) is SciPy's
``ive`` (a library primitive).

Sec. 3.5, eq. FIF-AMR: on the composite mesh phi = Gamma H P f^: on every
level k the composite source (P f^)_k -- the coarsening of finer levels'
sources (the cumulative F_k) plus the interpolation of the coarser levels'
sources (q_0 = f^_0, q_k = P q_{k-1} + f^_k) -- over the level's blocks and
its extended region, convolved with E(a_k), a_k = 4^k a_0, and kept on
Omega_k.  The grid bookkeeping (levels, Omega_k, extended regions, P) is
the LGF composite oracle's.
"""
import numpy as np
from scipy.special import ive

from . import composite as C


def kernel_row(a, nmax):
    """e^{-2a} I_n(2a) for n = 0..nmax."""
    return ive(np.arange(nmax + 1), 2.0 * a)


def apply(src_cells, f, tgt_cells, a, chunk=None):
    """u[t] = sum_s E(t - s) f[s], E the integrating-factor kernel of a (direct sum)."""
    src = np.asarray(src_cells, dtype=np.int64).reshape(-1, 3)
    tgt = np.asarray(tgt_cells, dtype=np.int64).reshape(-1, 3)
    f = np.asarray(f, dtype=np.float64).reshape(-1)
    keep = f != 0.0
    src, f = src[keep], f[keep]
    out = np.zeros(len(tgt))
    if len(src) == 0:
        return out
    span = int(max(np.abs(tgt.max(axis=0)[None] - src.min(axis=0)[None]).max(),
                   np.abs(src.max(axis=0)[None] - tgt.min(axis=0)[None]).max()))
    B = kernel_row(a, span)
    chunk = chunk or max(1, int(4e6 // len(src)))
    for i in range(0, len(tgt), chunk):
        t = tgt[i:i + chunk]
        d = np.abs(t[:, None, :] - src[None, :, :])
        out[i:i + chunk] = (B[d[..., 0]] * B[d[..., 1]] * B[d[..., 2]]) @ f
    return out


def fif_solve(nb, dx0, level_blocks, f_levels, a0, ext_layers=1, sample=None):
    """phi_k on the cells of level-k blocks (0 on covered cells), eq. FIF-AMR."""
    orc = C.CompositeOracle(nb, dx0, level_blocks, ext_layers=ext_layers)
    K = orc.K
    fhat = [np.where(orc.mask[k], f_levels[k], 0.0) for k in range(K)]
    F = orc.cumulative_sources(fhat)
    out = []
    q_cells, q = None, None
    for k in range(K):
        a = a0 * 4.0 ** k
        tsel = np.nonzero(orc.mask[k])[0] if sample is None else np.asarray(sample[k])
        tsel = tsel[orc.mask[k][tsel]]
        tc = orc.cells[k][tsel]
        phi = np.zeros(len(orc.cells[k]))
        if k == 0:
            phi[tsel] = apply(orc.cells[0], F[0], tc, a)
            q_cells, q = orc.cells[0], fhat[0]
        else:
            R = orc.ext_cells[k]
            qb = C.Box.around(np.concatenate([q_cells, np.floor_divide(R, 2)]), 1)
            qa = qb.zeros()
            i, j, kk = qb.idx(q_cells)
            qa[i, j, kk] = q
            Pq = C.interp_trilinear(qb, qa, R)
            rb = C.Box.around(R, 0)
            Fa, fa = rb.zeros(), rb.zeros()
            i2, j2, k2 = rb.idx(orc.cells[k])
            Fa[i2, j2, k2] = F[k]
            fa[i2, j2, k2] = fhat[k]
            i, j, kk = rb.idx(R)
            phi[tsel] = apply(R, Pq + Fa[i, j, kk], tc, a)
            q_cells, q = R, Pq + fa[i, j, kk]
        out.append(phi)
    return out
