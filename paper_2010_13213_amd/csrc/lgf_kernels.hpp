// Host-side launch entry points of the LGF device kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lgf {

// ---- table / spectra (lgf_table.hip) ----
int lgf_table_nodes();
// gcube: (R+1)^3 doubles; B: nodes*(R+1) doubles; w: nodes doubles.
hipError_t build_lgf_table(double *gcube, double *B, double *w, hipStream_t s);
hipError_t eval_lgf_points(const double *gcube, const int *ijk, double *out, int64_t n, hipStream_t s);
// Spectra of every block offset in [0,XH] x [0,YH] x [0,ZH] into
// table[omega][dy][dz][dx] (complex float or double); offsets with negative
// components are served by reflection.
// far: the LGF (cube, then the asymptotic series) or a cube kernel that is 0
// beyond the cube; the kernel is sampled at stride * n; band 1 keeps only
// block offsets with max |d_i| <= D, band 2 only those beyond (0: all).
hipError_t build_spectra(const double *gcube, bool far, int stride, int band, int D, int nb, int XH, int YH, int ZH,
                         bool fp32, void *table, void *scratch, size_t scratch_bytes, hipStream_t s);
// Integrating-factor kernel E(n) = prod_i e^{-2a} I_{n_i}(2a) on the near
// cube layout (row: kTableRadius + 1 doubles of scratch, w: one double).
hipError_t build_if_table(double *cube, double *row, double *w, double a, hipStream_t s);

// ---- block FFTs (lgf_fft.hip) ----
// Spectral workspaces hold spectrum value omega = (kz N + ky) H + kx (of
// n_freq = N^2 H, N = 2 nb, H = nb + 1) of slot sl at omega * n_slots + sl
// (frequency-major: the block-pair MAC) or at sl * n_freq + spec_pos(omega)
// (block-major: the lattice MAC).  Block-major spectra are stored in
// kSpecChunks kx ranges of spec_chunk(N) (the last one shorter), each range
// [kz][ky][kx - k0], the ranges the FFT workgroups of a block work on.
constexpr int kSpecChunks = 3;
__host__ __device__ inline int spec_chunk(int N) { return (N / 2 + 3) / 3; }   // ceil(H / 3)
__host__ __device__ inline int spec_pos(int N, int kx, int ky, int kz) {
    const int kc = spec_chunk(N), k0 = kx / kc * kc;
    const int nk = kc < N / 2 + 1 - k0 ? kc : N / 2 + 1 - k0;
    return N * N * k0 + (kz * N + ky) * nk + (kx - k0);
}
__host__ __device__ inline void spec_freq(int N, int p, int &kx, int &ky, int &kz) {
    const int kc = spec_chunk(N), k0 = p / (N * N * kc) * kc;
    const int nk = kc < N / 2 + 1 - k0 ? kc : N / 2 + 1 - k0;
    const int r = p - N * N * k0;
    kx = k0 + r % nk;
    ky = (r / nk) % N;
    kz = r / (nk * N);
}
// Forward: for each listed block i, read the nb^3 float64 values at
// src + blk_off[i] (elements), multiply by `scale`, zero-pad to (2nb)^3,
// r2c-transform and store the spectrum of slot[i] in Fhat.
hipError_t block_fft_forward(int nb, bool fp32, const double *src, const int64_t *blk_off, const int *slot,
                             int n_blocks, void *Fhat, int64_t n_slots, bool block_major, double scale, hipStream_t s);
// Inverse: for each listed block i, gather the spectrum of slot[i] from Uhat
// (plus Uhat2 when not null: block-major only), c2r-transform, keep the
// [0, nb)^3 corner, multiply by `scale` and write (accumulate = 0) or add
// (accumulate = 1) into dst + blk_off[i].
hipError_t block_fft_inverse(int nb, bool fp32, const void *Uhat, const void *Uhat2, int64_t n_slots, bool block_major, const int *slot,
                             const int64_t *blk_off, int n_blocks, double *dst, double scale, int accumulate,
                             hipStream_t s);

// Batched block FFTs: job i covers blocks [blk_begin, next blk_begin) of the grid.
struct FftJob {
    const double *src;      // forward: source field base;     inverse: unused
    double *dst;            // inverse: destination field base; forward: unused
    const int64_t *blk_off; // per block: element offset in src / dst
    const int *slot;        // per block: slot in the spectral workspace
    void *spec;             // forward: Fhat; inverse: Uhat
    const void *spec2;      // inverse: a second Uhat added to the first (block-major), or null
    int64_t n_slots;
    int block_major;        // spectral layout (see block_fft_forward)
    double scale;
    int accumulate;
    int blk_begin;
};
hipError_t block_fft_forward_batch(int nb, bool fp32, const FftJob *jobs, int n_jobs, int total_blocks, hipStream_t s);
hipError_t block_fft_inverse_batch(int nb, bool fp32, const FftJob *jobs, int n_jobs, int total_blocks, hipStream_t s);

// ---- spectral multiply-accumulate (lgf_smac.hip) ----
// A source row of one convolution: (y, z) in blocks of the padded box and
// the mask of its occupied x positions (bit x set: a source block sits at x).
struct SmacRow {
    int y, z;
    unsigned mask;
    int pad;
};
// A work tile of one convolution: a TY x TZ rectangle of target rows at
// (ty0, tz0) and the lanes that run on it, lanes[lane_off + l] for
// l < n_lanes, each packed as seg | tyl << 8 | tzl << 16 (the lane's A
// targets start at x = seg * A of row (ty0 + tyl, tz0 + tzl)).  Only
// x-segments that hold targets get a lane.
struct SmacTile {
    int ty0, tz0, lane_off, n_lanes;
};
struct SmacGeom {
    int bx;                 // row length template (8 or 16)
    int ty, tz;             // tile shape in rows (one of smac_tiles(bx))
    int ey, ez;             // padded box extent in blocks along y, z (slots)
    int n_freq;
    int64_t n_slots;        // bx * ey * ez
    int XH, YH, ZH, XD, YD, ZD;   // octant spectra table extents (XD = XH + 1, ...)
    int N;                        // FFT edge 2 nb (frequency index remap)
    const int *perm;              // frequency order: reflection partners adjacent
    int n_rows;             // source rows (sy, sz), serpentine order
    int n_tiles;            // work tiles
    const int *lanes;       // packed lane table of the tiles
    int rs;                 // slots per row of the padded box (multiple of bx)
    int tx0, sx0;           // x offsets of this part's target / source segment
    int accum;              // add into Uhat instead of storing
    int64_t fstride;        // elements between the components of Fhat / Uhat
    int axis;               // 0: rows along lattice x; 1: rows along lattice y (x and y swapped)
};
// One convolution of a batched spectral-MAC launch (device-resident table).
struct SmacJob {
    SmacGeom g;
    const void *F;
    void *U;
    const void *K;
    const SmacRow *rows;
    const SmacTile *tiles;
    int64_t wg_begin;       // first workgroup of this job in the batched grid
};
hipError_t smac_batch_launch(int bx, int ty, int tz, bool fp32, bool sparse, const SmacJob *jobs, int n_jobs,
                             int64_t total_wg, hipStream_t s);
int smac_seg_len(int bx);   // A: targets per lane
// Tile shapes (TY, TZ) compiled for row template bx, the default first;
// writes up to max_tiles of them and returns how many exist.
int smac_tiles(int bx, int (*tiles)[2], int max_tiles);
// Uhat[c][omega][t] = sum_s K[omega][t - s] * Fhat[c][omega][s] for the nc
// (1..3) components c, over every source row
// and every target slot of each tile; source positions outside a row's mask
// are skipped when `sparse` (their Fhat must be zero either way).
hipError_t smac_launch(const SmacGeom &g, bool fp32, bool sparse, int nc, const void *Fhat, void *Uhat,
                       const void *Ktab, const SmacRow *rows, const SmacTile *tiles, hipStream_t s);

// ---- spectral MAC by an FFT over the block lattice (lgf_lattice.hip) ----
// Box E = (ex, ey, ez) blocks, lattice DFT lengths (lx, ly, lz), each a
// compiled length (4, 8, 16, 32; lz also 64) with 2 e <= l; N = 2 nb is the block FFT
// edge (n_freq = N^2 (N/2 + 1)).  Fhat / Uhat block-major: [c][slot][omega]
// (slot = (z ey + y) ex + x, n_slots = ex ey ez), components fstride
// (>= n_freq n_slots) elements apart; H:
// [c][omega][kx][z][y] workspace, (omega, kx) slabs of ey ez elements
// hslab (>= ey ez) apart, components hstride (>= n_freq lx hslab) elements
// apart; Khat: real [omega_r][kx][kz][ky] over the stored frequencies
// (ky, kz in [0, N/2]).
struct LatGeom {
    int ex, ey, ez;
    int lx, ly, lz;
    int nc;
    int N;
    int n_freq;
    int64_t n_slots;        // ex * ey * ez
    int64_t fstride, hstride;
    int hslab;
    // source slots that hold a block (1) or not (0), or null when every slot
    // does: the x pass reads empty slots as zero, so Fhat needs no clearing
    const unsigned char *occ;
};
// Octant block-spectra table (offsets 0..XD-1 etc.) of FFT edge N = 2 nb.
struct LatSpecGeom {
    int N;
    int lx, ly, lz;
    int XD, YD, ZD;
};
bool lattice_len_ok(int L);    // compiled x and y lengths: 4, 8, 16, 32, 64
bool lattice_zlen_ok(int L);   // compiled z lengths: also 128
int lattice_len(int extent);   // smallest length L >= max(4, 2 extent - 1)
int lattice_stored_freqs(int N);   // frequencies with stored lattice spectra: (N/2 + 1)^3
// Uhat[c] = the lattice convolution of Fhat[c] with the kernel whose
// spectrum is Khat, for the nc components: lattice_fwd (x DFTs into H),
// lattice_yz (y and z DFTs, product, inverse z and y DFTs in H),
// lattice_inv (inverse x DFTs into Uhat).
hipError_t lattice_fwd(const LatGeom &g, bool fp32, const void *Fhat, void *H, hipStream_t s);
// worder: the n_freq spectrum positions (spec_pos) in the order lattice_yz
// takes them (any permutation; reflection partners adjacent lets them share
// Khat in L2).
hipError_t lattice_yz(const LatGeom &g, bool fp32, void *H, const void *Khat, const int *worder, hipStream_t s);
hipError_t lattice_inv(const LatGeom &g, bool fp32, const void *H, void *Uhat, hipStream_t s);
// The same convolution in one pass per frequency, at lengths 32 x 32 x 32
// only (lattice_fused_ok): the terms of the even and the odd lattice x
// frequencies go to Uhat and Uhat2 (same layout), whose sum is the result
// (block_fft_inverse adds them); no H.
bool lattice_fused_ok(const LatGeom &g);
hipError_t lattice_fused(const LatGeom &g, bool fp32, const void *Fhat, const void *Khat, void *Uhat, void *Uhat2,
                         hipStream_t s);
// Khat for lattice lengths (lx, ly, lz) from the octant table (same
// precision), scaled by 1 / (lx ly lz); scratch holds the complex
// intermediate of a chunk of frequencies.
hipError_t lattice_spectra(const LatSpecGeom &sg, bool fp32, const void *octant, void *Khat, void *scratch,
                           size_t scratch_bytes, hipStream_t s);

// ---- composite-grid kernels (lgf_composite.hip) ----
// dst block b = src block b with the octants flagged in cover[b] (cover may
// be null) zeroed, and the cells whose byte in cmask + b nb^3 is 0 (cmask may
// be null).
hipError_t mask_blocks(int nb, const double *src, double *dst, const int64_t *src_off, const int64_t *dst_off,
                       const unsigned char *cover, int n_blocks, hipStream_t s,
                       const unsigned char *cmask = nullptr);
// coarse octant (octant[i]) of the block at coarse_off[i] = mean of 8 children
// of the fine block at fine_off[i].
hipError_t coarsen_mean8(int nb, const double *fine, double *coarse, const int64_t *fine_off,
                         const int64_t *coarse_off, const unsigned char *octant, int n_pairs, hipStream_t s);
hipError_t copy_blocks(int nb, const double *src, double *dst, const int64_t *src_off, const int64_t *dst_off,
                       int n_blocks, hipStream_t s);
// p[0, bytes) = 0 by a kernel (bytes and p 16-byte aligned); a memset node
// is avoided in code that a caller may capture into a graph.
hipError_t zero_fill(void *p, size_t bytes, hipStream_t s);

// Two-grid fast-LGF far field (lgf_flgf.hip), nb = 16 only: per block, the
// cells at f + off[b] anterpolated to the block's (nb/2)^3 nodes at
// Fc + b (nb/2)^3, and node values Uc interpolated and added to u + off[b].
hipError_t flgf_anterpolate(int nb, const double *f, const int64_t *off, int n_blocks, double *Fc, hipStream_t s);
hipError_t flgf_interpolate_add(int nb, const double *Uc, const int64_t *off, int n_blocks, double *u, hipStream_t s);

// Per block of nb^3 values at v + off[b] (off null: v + b * nb^3): the sum
// of squares into out[2b] and the largest magnitude into out[2b + 1].
hipError_t block_stats(int nb, const double *v, const int64_t *off, int n_blocks, double *out, hipStream_t s);

// Velocity refresh: u = -C^dagger psi (backward-difference curl, 1/dx) on
// the blocks of one level, 3 components comp_len apart; nbr_off[3b + a] is
// the field offset of block b's neighbour one block back along axis a, or -1
// (lgf_refresh.hip).
hipError_t curl_backward_blocks(int nb, const double *psi, double *u, int64_t comp_len, const int64_t *blk_off,
                                const int64_t *nbr_off, int n_blocks, double inv_dx, hipStream_t s);
struct CorrGeom {
    double dxc, dxf;        // cell widths of levels k-1 and k
    int mlo[3], mdim[3];    // dense map of psi_{k-1} blocks: index or -1
    int interp_only;        // 1: no commutator -- the outputs are P psi, P psi + F_k, P psi + f^_k
};
// For each level-k block fblk[b] (x,y,z): P psi_{k-1}, and S + F_k, S + f^_k
// (F_k, f^_k read at own_off[b] when >= 0, else 0) into block b of the
// compact outputs; with interp_only, P psi in place of S.
hipError_t correction_source(int nb, const CorrGeom &g, const double *psi, const int *cmap, const int *fblk,
                             const int64_t *own_off, const double *Fk, const double *fhk, double *Ppsi,
                             double *SrcF, double *Srcf, int n_blocks, hipStream_t s);

// ---- mixed-precision refinement (lgf_refine.hip) ----
struct RefGeom {
    double dx;
    int lo[3], dim[3];      // dense block map of the target set T: T index or -1
};
// depth (L1 distance to the complement of T, capped at 3) of every cell of
// the listed shell blocks
hipError_t refine_depth(int nb, const RefGeom &g, const int *map, const int *shblk, unsigned char *depth, int n_sh,
                        hipStream_t s);
// On every T block: w = u~ where depth >= 2 else 0; dst (+)= w; rho = src -
// L_dx w split into rin (depth >= 3, per T block) and rcut (depth <= 2, per
// shell block).  See lgf_refine.hip.
hipError_t refine_residual(int nb, const RefGeom &g, const int *map, const int *tblk, const int *t2sh,
                           const unsigned char *depth, const double *ut, const double *src, const int64_t *gofs,
                           const int64_t *dofs, double *dst, int accumulate, double *rin, double *rcut, int n_t,
                           hipStream_t s);

}  // namespace lgf
