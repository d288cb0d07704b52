"""Oracle for the multi-level (composite-grid) LGF solve -- test infrastructure.

Follows the revised FLGF-AMR algorithm of the paper, Sec. 3.4 (eqs.
AMR-LGF-2, partial_LGF, Scorrection, combine_S, FLGF-AMR), in its order:

1. fine -> coarse cumulative source  F_k = f^_k + P_{k+1->k} F_{k+1};
2. coarse -> fine: psi_0 = L_0^-1 f^_0; for k >= 1
       S_k   = (P_{k-1->k} L_{k-1} - L_k P_{k-1->k}) psi_{k-1}   on Omega_k u Omega_k^E
       psi_k = P psi_{k-1} + L_k^-1 (S_k + f^_k)
       phi_k = P psi_{k-1} + L_k^-1 (S_k + F_k)                  on Omega_k
   (phi_0 = L_0^-1 F_0);
3. restriction Gamma: phi_k is kept on Omega_k only.

Every L_k^-1 is the plain direct sum dx_k^2 * G * (.) of ``direct.py``; with
``fft_min_targets`` set, evaluations at that many target cells or more (the
full psi_k fields of large meshes) use the same convolution by a zero-padded
library FFT over the bounding box (``box.py``).

Readings where the paper is silent (each is listed in the design notes):

* levels k = 0..K-1 with dx_k = dx0 / 2^k; a level-(k+1) cell c' is a child
  of level-k cell floor(c'/2);
* Omega_k = cells of level-k blocks not covered by a level-(k+1) block;
* P_{k->k+1}: cell-centred trilinear interpolation; per axis the child at
  offset -1/4 gets 1/4 c[p-1] + 3/4 c[p], the child at +1/4 gets
  3/4 c[p] + 1/4 c[p+1] (Sec. 3.2 leaves the interpolant open);
* P_{k+1->k}: mean of the 8 children (coarsening);
* Omega_k^E: the level-k blocks that are 26-neighbours of level-k blocks
  (one block layer, N_E = N_b), eq. extended_regions with a block-aligned
  distance; S_k is added to the sources only (Sec. 3.4, after Fig. 4).
  ``ext_layers`` widens it (tests use it to cover the whole support of S);
* psi_{k-1} is needed on the coarse parents of Omega_k u Omega_k^E dilated
  by two coarse cells (one for trilinear P, one for L_{k-1});
* L_k = dx_k^-2 * (7-point stencil).
"""
import numpy as np

from . import box as fftbox, direct


# ---------------------------------------------------------------- helpers --

def block_cells(blocks, nb):
    """Set-like (n*nb^3, 3) lattice coordinates of the cells of ``blocks``."""
    blocks = np.asarray(blocks, dtype=np.int64).reshape(-1, 3)
    r = np.arange(nb)
    zz, yy, xx = np.meshgrid(r, r, r, indexing="ij")
    local = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
    return (blocks[:, None, :] * nb + local[None]).reshape(-1, 3)


def dilate_blocks(blocks, layers=1):
    """Blocks within ``layers`` (inf-norm) of any block, as a sorted array."""
    s = {tuple(b) for b in np.asarray(blocks).tolist()}
    out = set(s)
    rng = range(-layers, layers + 1)
    for b in s:
        for dz in rng:
            for dy in rng:
                for dx in rng:
                    out.add((b[0] + dx, b[1] + dy, b[2] + dz))
    return np.array(sorted(out, key=lambda t: (t[2], t[1], t[0])), dtype=np.int64)


class Box:
    """Dense array over an axis-aligned box of lattice cells."""

    def __init__(self, lo, hi):
        self.lo = np.asarray(lo, dtype=np.int64)
        self.hi = np.asarray(hi, dtype=np.int64)      # exclusive
        self.shape = tuple((self.hi - self.lo).tolist())

    @staticmethod
    def around(cells, margin):
        cells = np.asarray(cells)
        return Box(cells.min(axis=0) - margin, cells.max(axis=0) + 1 + margin)

    def idx(self, cells):
        """Array indices of lattice cells; every cell must lie in the box
        (a negative index would otherwise wrap around silently)."""
        c = np.asarray(cells).reshape(-1, 3) - self.lo
        if len(c) and (c.min() < 0 or np.any(c.max(axis=0) >= self.hi - self.lo)):
            raise IndexError("cells outside the box [%s, %s)" % (self.lo.tolist(), self.hi.tolist()))
        return c[:, 0], c[:, 1], c[:, 2]

    def zeros(self):
        return np.zeros(self.shape)

    def cells(self):
        ax = [np.arange(self.lo[i], self.hi[i]) for i in range(3)]
        g = np.meshgrid(*ax, indexing="ij")
        return np.stack([a.ravel() for a in g], axis=1)


def laplacian7(a, dx):
    """dx^-2 (sum of 6 neighbours - 6 a) on the interior of a dense array."""
    out = np.zeros_like(a)
    out[1:-1, 1:-1, 1:-1] = (a[2:, 1:-1, 1:-1] + a[:-2, 1:-1, 1:-1]
                             + a[1:-1, 2:, 1:-1] + a[1:-1, :-2, 1:-1]
                             + a[1:-1, 1:-1, 2:] + a[1:-1, 1:-1, :-2]
                             - 6.0 * a[1:-1, 1:-1, 1:-1]) / (dx * dx)
    return out


def interp_trilinear(coarse_box, coarse, fine_cells):
    """P_{k->k+1}: cell-centred trilinear values at fine cells.

    Per axis a fine cell c' has parent p = floor(c'/2) and side s = c' - 2p;
    weights (1/4, 3/4) on (p-1, p) for s = 0 and (3/4, 1/4) on (p, p+1) for
    s = 1.  The 3-D weights are the products of the per-axis weights.
    """
    fine_cells = np.asarray(fine_cells, dtype=np.int64)
    p = np.floor_divide(fine_cells, 2)
    s = fine_cells - 2 * p
    out = np.zeros(len(fine_cells))
    for ox in (0, 1):
        for oy in (0, 1):
            for oz in (0, 1):
                o = np.array([ox, oy, oz])
                # neighbour index along each axis: s=0 -> (p-1, p); s=1 -> (p, p+1)
                nbr = p + np.where(s == 0, o - 1, o)
                w = np.ones(len(fine_cells))
                for ax in range(3):
                    wa = np.where(s[:, ax] == 0,
                                  np.where(o[ax] == 1, 0.75, 0.25),
                                  np.where(o[ax] == 0, 0.75, 0.25))
                    w = w * wa
                i, j, k = coarse_box.idx(nbr)
                out += w * coarse[i, j, k]
    return out


def coarsen_mean8(fine_box, fine, coarse_cells):
    """P_{k+1->k}: mean of the 8 children 2c + {0,1}^3 of each coarse cell."""
    coarse_cells = np.asarray(coarse_cells, dtype=np.int64)
    out = np.zeros(len(coarse_cells))
    for o in np.ndindex(2, 2, 2):
        i, j, k = fine_box.idx(2 * coarse_cells + np.array(o))
        out += fine[i, j, k]
    return out / 8.0


# ------------------------------------------------------------ the solver --

class CompositeOracle:
    """Composite-grid LGF solve of one scalar component (all steps in FP64)."""

    def __init__(self, nb, dx0, level_blocks, ext_layers=1, fft_min_targets=None, cell_masks=None):
        self.nb = nb
        self.fft_min_targets = fft_min_targets
        self.dx0 = dx0
        self.K = len(level_blocks)
        self.blocks = [np.asarray(b, dtype=np.int64).reshape(-1, 3) for b in level_blocks]
        self.dx = [dx0 / 2 ** k for k in range(self.K)]
        self.cells = [block_cells(b, nb) for b in self.blocks]
        # Omega_k mask over the cells of level-k blocks (True = kept): cells
        # no level-(k+1) block covers, further restricted by the caller's cell
        # mask (the partition of Sec. 3.1 given cell by cell; a kept covered
        # cell would make the levels overlap)
        self.covered, self.mask = [], []
        for k in range(self.K):
            if k + 1 < self.K:
                fine = {tuple(b) for b in self.blocks[k + 1].tolist()}
                child_blk = np.floor_divide(2 * self.cells[k], nb)
                covered = np.array([tuple(c) in fine for c in child_blk.tolist()])
            else:
                covered = np.zeros(len(self.cells[k]), dtype=bool)
            keep = ~covered
            if cell_masks is not None and cell_masks[k] is not None:
                cm = np.asarray(cell_masks[k]).reshape(-1).astype(bool)
                if np.any(cm & covered):
                    raise ValueError("levels overlap after masking (level %d)" % k)
                keep = keep & cm
            self.covered.append(covered)
            self.mask.append(keep)
        # R_k = Omega_k u Omega_k^E as cells of the dilated block set (k >= 1).
        self.ext_blocks = [None] + [dilate_blocks(self.blocks[k], ext_layers)
                                    for k in range(1, self.K)]
        self.ext_cells = [None] + [block_cells(b, nb) for b in self.ext_blocks[1:]]
        # dom(psi_k) for k < K-1: parents of R_{k+1} dilated by 2 coarse cells.
        self.psi_cells = []
        for k in range(self.K - 1):
            par = np.unique(np.floor_divide(self.ext_cells[k + 1], 2), axis=0)
            box = Box.around(par, 2)
            sel = np.zeros(box.shape, dtype=bool)
            i, j, kk = box.idx(par)
            sel[i, j, kk] = True
            d = sel.copy()
            for ax in range(3):       # two passes of +-1 dilation per axis
                for _ in range(2):
                    e = d.copy()
                    sl_lo = [slice(None)] * 3
                    sl_hi = [slice(None)] * 3
                    sl_lo[ax] = slice(1, None)
                    sl_hi[ax] = slice(None, -1)
                    e[tuple(sl_lo)] |= d[tuple(sl_hi)]
                    e[tuple(sl_hi)] |= d[tuple(sl_lo)]
                    d = e
            self.psi_cells.append(box.cells()[d.ravel()])

    # ---- stage: fine -> coarse cumulative source (step 1) ----
    def cumulative_sources(self, fhat):
        """F_k on the cells of level-k blocks, given f^_k (masked sources)."""
        F = [None] * self.K
        F[self.K - 1] = fhat[self.K - 1].copy()
        for k in range(self.K - 2, -1, -1):
            fb = Box.around(self.cells[k + 1], 0)
            arr = fb.zeros()
            i, j, kk = fb.idx(self.cells[k + 1])
            arr[i, j, kk] = F[k + 1]
            Fk = fhat[k].copy()
            cov = self.covered[k]
            Fk[cov] = coarsen_mean8(fb, arr, self.cells[k][cov])
            F[k] = Fk
        return F

    def conv(self, k, src_cells, src_vals, tgt_cells):
        """L_k^-1 applied to a source on cells, evaluated at target cells."""
        keep = src_vals != 0.0
        if self.fft_min_targets is not None and len(tgt_cells) >= self.fft_min_targets and keep.any():
            return fftbox.convolve_cells(src_cells[keep], src_vals[keep], tgt_cells, self.dx[k])
        return direct.direct_sum(src_cells[keep], src_vals[keep], tgt_cells, self.dx[k])

    # ---- stage: correction source S_k on R_k (step 2) ----
    def correction_source(self, k, psi_prev_cells, psi_prev):
        """P psi_{k-1} on R_k and S_k = (P L_{k-1} - L_k P) psi_{k-1} on R_k."""
        cb = Box.around(psi_prev_cells, 0)
        psi_arr = cb.zeros()
        i, j, kk = cb.idx(psi_prev_cells)
        psi_arr[i, j, kk] = psi_prev
        Lpsi = laplacian7(psi_arr, self.dx[k - 1])
        R = self.ext_cells[k]
        fb = Box.around(R, 1)
        halo = fb.cells()
        Ppsi_arr = fb.zeros()
        Ppsi_arr[tuple((halo - fb.lo).T)] = interp_trilinear(cb, psi_arr, halo)
        LPpsi = laplacian7(Ppsi_arr, self.dx[k])
        i, j, kk = fb.idx(R)
        Ppsi_R = Ppsi_arr[i, j, kk]
        S = interp_trilinear(cb, Lpsi, R) - LPpsi[i, j, kk]
        return Ppsi_R, S

    def solve(self, f_levels, sample=None):
        """Return phi_k on the cells of level-k blocks (0 on masked cells).

        ``f_levels[k]`` holds f on the cells of level-k blocks in
        ``block_cells`` order.  ``sample`` (optional list of index arrays)
        restricts the final phi_k evaluation to those cells of each level.
        """
        fhat = [np.where(self.mask[k], f_levels[k], 0.0) for k in range(self.K)]
        F = self.cumulative_sources(fhat)
        # the combined source of each level's phi convolution (eq.
        # combined_source; the refinement indicator of Sec. 4.2): cells, values
        self.combined = [(self.cells[0], F[0].copy())]
        out = []
        psi_cells, psi = None, None
        for k in range(self.K):
            tsel = np.nonzero(self.mask[k])[0] if sample is None else np.asarray(sample[k])
            tsel = tsel[self.mask[k][tsel]]
            phi = np.zeros(len(self.cells[k]))
            if k == 0:
                phi[tsel] = self.conv(0, self.cells[0], F[0], self.cells[0][tsel])
                if self.K > 1:
                    psi_cells = self.psi_cells[0]
                    psi = self.conv(0, self.cells[0], fhat[0], psi_cells)
            else:
                Ppsi_R, S = self.correction_source(k, psi_cells, psi)
                R = self.ext_cells[k]
                # sources on R_k: S + F_k (resp. S + f^_k) on level-k block cells
                rb = Box.around(R, 0)
                srcF = rb.zeros()
                srcf = rb.zeros()
                i, j, kk = rb.idx(R)
                srcF[i, j, kk] = S
                srcf[i, j, kk] = S
                i2, j2, k2 = rb.idx(self.cells[k])
                srcF[i2, j2, k2] += F[k]
                srcf[i2, j2, k2] += fhat[k]
                vF = srcF[i, j, kk]
                vf = srcf[i, j, kk]
                self.combined.append((R, vF.copy()))
                pr = Box.around(R, 0)
                Pp = pr.zeros()
                Pp[i, j, kk] = Ppsi_R
                tc = self.cells[k][tsel]
                ti, tj, tk = pr.idx(tc)
                phi[tsel] = Pp[ti, tj, tk] + self.conv(k, R, vF, tc)
                if k + 1 < self.K:
                    pc = self.psi_cells[k]
                    # P psi_{k-1} at dom(psi_k), which can reach past R_k
                    cb = Box.around(psi_cells, 0)
                    psi_arr = cb.zeros()
                    a, b_, c = cb.idx(psi_cells)
                    psi_arr[a, b_, c] = psi
                    psi = interp_trilinear(cb, psi_arr, pc) + self.conv(k, R, vf, pc)
                    psi_cells = pc
            out.append(phi)
        return out
