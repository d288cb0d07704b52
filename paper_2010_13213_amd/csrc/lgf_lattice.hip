// Spectral multiply-accumulate by an FFT over the block lattice (gfx950).
//
// After the forward block FFTs the convolution of a level is, at every
// block frequency omega, a linear convolution over the block lattice
// (paper Sec. 2.2, eq. lgf_convolution, evaluated blockwise):
//
//     Uhat_t(omega) = sum_s K_{t-s}(omega) Fhat_s(omega),   t, s in a box E.
//
// Zero-padding the box to L >= 2E - 1 per axis makes the circular
// convolution of a length-L DFT exact, so the sum becomes
//
//     Uhat = crop_E( IDFT_L( Khat . DFT_L(pad_L(Fhat)) ) ),
//     Khat(omega, k) = sum_d K_d(omega) exp(-2 pi i k.d / L),
//
// with d in (-L/2, L/2) per axis (d = L/2 is never reached and is set to
// zero).  Two symmetries of the block windows of the real kernel, which is
// even along each axis, shape the spectra:
//   * K_{-d}(omega) = conj(K_d(omega)), so Khat is real;
//   * mirroring d along y (z) mirrors omega along y (z), so
//     Khat(omega, k) = Khat(R omega, R k) for R a y and/or z reflection:
//     only frequencies with ky, kz in [0, N/2] are stored (28% at N = 32).
// Khat is stored as real numbers with the 1 / (Lx Ly Lz) of the inverse
// folded in.  The cost per frequency is O(L^3 log L) instead of the O(E^6)
// block pairs.
//
// Layouts (complex R, per component region):
//   Fhat, Uhat [slot][p] (block-major: the block FFTs stream whole
//              spectra; p = spec_pos(omega), chunk-major in kx), slot =
//              (z Ey + y) Ex + x over the box E; the x kernels take p as
//              an opaque index and H is indexed by it;
//   H          [p][kx][z][y]: the box after the x DFT (kx < Lx), slabs
//              hslab apart (padded against power-of-two strides);
//   Khat       [omega_r][kx][kz][ky] (real R), omega_r over the stored
//              frequencies.
// Three kernels, each streaming its data once from HBM:
//   lat_x_fwd  x lines of Fhat -> H (a lane pair per line; a workgroup takes
//              one 128-byte run of frequencies (8 in float64, 16 in float32)
//              x 16 (y, z) rows);
//   lat_yz     one (omega, kx) slab per 2 Ly lanes, in LDS: y DFT, z DFT,
//              product with Khat, inverse z and y DFTs, in place in H (the
//              two halves of a line on lanes of different waves, meeting
//              through LDS);
//   lat_x_inv  inverse x lines of H, cropped, -> Uhat.
// Inputs beyond E are zero (E <= L/2) and outputs beyond E are dropped, so
// every line is split over a lane pair by the radix-2 identities
// (M = L/2, w = exp(-2 pi i / L)):
//   X[2m] = DFT_M(x)[m],  X[2m+1] = DFT_M(w^n x)[m]                (forward)
//   y[n]  = IDFT_M(X[2m])[n] + w^-n IDFT_M(X[2m+1])[n],  n < M      (inverse)
// the inverse with one exchange of half a line between the two lanes.
#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "lgf_device.hpp"
#include "lgf_kernels.hpp"

namespace lgf {

namespace {

constexpr int kLatThreads = 256;

template <typename R> __device__ __forceinline__ cplx<R> czero() { return cmake<R>((R)0, (R)0); }

// c ? a : b per component (a select of whole structs is lowered through
// private memory)
template <typename R> __device__ __forceinline__ cplx<R> csel(bool c, cplx<R> a, cplx<R> b) {
    return cmake<R>(c ? a.x : b.x, c ? a.y : b.y);
}

// Forward half-line DFT of a lane pair: a holds x[n] (n < L/2, zero beyond
// the data); on return a[m] = X[2m + odd].
template <typename R, int L> __device__ __forceinline__ void pair_fwd(cplx<R> (&a)[L / 2], int odd) {
#pragma unroll
    for (int n = 1; n < L / 2; ++n) {
        // select on data, not on the twiddle: the constants stay literal
        const cplx<R> t = cmul(a[n], twiddle<R, L, false>(n));
        a[n] = csel(odd, t, a[n]);
    }
    fft_reg<R, L / 2, false>(a);
}

// Inverse half-line DFT of a lane pair: a holds X[2m + odd] (m < L/2); on
// return out[j] = y[n] with n = j (even lane) or L/4 + j (odd lane),
// j < L/4.  Both lanes of every pair must call it (one exchange).
template <typename R, int L>
__device__ __forceinline__ void pair_inv(cplx<R> (&a)[L / 2], int odd, cplx<R> (&out)[L / 4]) {
    constexpr int M = L / 2;
    fft_reg<R, M, true>(a);
#pragma unroll
    for (int j = 0; j < M / 2; ++j) {
        const int jo = M / 2 + j;   // the odd lane's output index
        const cplx<R> send = csel(odd, a[j], a[jo]);
        cplx<R> recv;
        recv.x = __shfl_xor(send.x, 1);
        recv.y = __shfl_xor(send.y, 1);
        const cplx<R> ye = cmac(a[j], recv, twiddle<R, L, true>(j));     // even lane: n = j
        const cplx<R> yo = cmac(recv, a[jo], twiddle<R, L, true>(jo));   // odd lane: n = jo
        out[j] = csel(odd, yo, ye);
    }
}

// exp(-+2 pi i k / N) for any k in [0, N) known at compile time after
// unrolling (the table holds k < N / 2; the rest are negated)
template <typename R, int N, bool INV> __device__ __forceinline__ cplx<R> twiddle_full(int k) {
    const cplx<R> w = twiddle<R, N, INV>(k % (N / 2));
    return k < N / 2 ? w : cmake<R>(-w.x, -w.y);
}

// Tile of the x kernels: xtw<R> consecutive frequencies (one 128-byte run
// per slot: 8 in float64, 16 in float32) x kTQ consecutive (y, z) rows q of
// one component, a lane pair per line (xthreads<R> threads); row
// rl = wl kTQ + ql.
template <typename R> constexpr int xtw = 128 / (int)sizeof(cplx<R>);
constexpr int kTQ = 16;
template <typename R> constexpr int xthreads = 2 * xtw<R> * kTQ;

struct XTile {
    int c, w0, q0;
};
template <int TW, int TQ = kTQ> __device__ __forceinline__ XTile x_tile(const LatGeom &g, int b) {
    const int per_w = g.ey * g.ez;
    const int wt = (g.n_freq + TW - 1) / TW, qt = (per_w + TQ - 1) / TQ;
    return XTile{b / (wt * qt), (b % wt) * TW, ((b / wt) % qt) * TQ};
}

// Forward x lines at LX = 64 in float64: a lane pair would hold 32 values
// per lane (256 registers, two waves per SIMD), so each line is split over
// four waves instead, one quarter of its frequencies per wave: with x[n]
// the line (n < 32, zero beyond the data) and w = exp(-2 pi i / 64),
//     X[4 m + r] = DFT_16(v)[m],  v[n] = w^(r n) (x[n] + (-i)^r x[n + 16]).
// A tile is kTQ rows of 8 frequencies (128 lines, the pair kernels' tile) on
// 512 threads: wave w takes quarter w mod 4 of lines 64 (w / 4) .. + 63.
// (The inverse split the same way needs more than 128 registers per lane
// for its four-way sum, and in float32 the pair kernels stay faster.)
constexpr int kX4Threads = 512;

// x lines of Fhat -> H.  The tile's lines are staged through LDS: the loads
// read each slot's kTW frequencies as one run, all issued before the first
// is waited on.  MASKED: slots without a source block (g.occ) read as zero.
template <typename R, int LX, bool MASKED>
__global__ void __launch_bounds__(xthreads<R>) lat_x_fwd(LatGeom g, const cplx<R> *__restrict__ F,
                                                         cplx<R> *__restrict__ H) {
    constexpr int M = LX / 2, SP = M + 1, kTW = xtw<R>, kXThreads = xthreads<R>;   // rows padded against bank conflicts
    constexpr int CELLS = kTW * kTQ * M, NI = (CELLS + kXThreads - 1) / kXThreads;
    __shared__ cplx<R> S[kTW * kTQ * SP];
    const int t = threadIdx.x;
    const int ex = g.ex, per_w = g.ey * g.ez;
    const XTile tl = x_tile<kTW>(g, blockIdx.x);
    const cplx<R> *Fc = F + (int64_t)tl.c * g.fstride;
    cplx<R> v[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = t + i * kXThreads;
        const int wl = e % kTW, r = e / kTW, ql = r / M, x = r % M;
        const int q = tl.q0 + ql, w = tl.w0 + wl;
        bool ok = e < CELLS && x < ex && q < per_w && w < g.n_freq;
        if (MASKED) ok = ok && g.occ[q * ex + x] != 0;
        const cplx<R> y = cload_nt(&Fc[ok ? (int64_t)(q * ex + x) * g.n_freq + w : 0]);
        v[i] = csel(ok, y, czero<R>());
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = t + i * kXThreads;
        const int wl = e % kTW, r = e / kTW, ql = r / M, x = r % M;
        if (e < CELLS) S[(wl * kTQ + ql) * SP + x] = v[i];
    }
    __syncthreads();
    const int rl = t >> 1, odd = t & 1;
    const int q = tl.q0 + rl % kTQ, w = tl.w0 + rl / kTQ;
    cplx<R> a[M];
#pragma unroll
    for (int n = 0; n < M; ++n) a[n] = S[rl * SP + n];
    pair_fwd<R, LX>(a, odd);
    if (q < per_w && w < g.n_freq) {
        cplx<R> *out = H + (int64_t)tl.c * g.hstride + (int64_t)w * LX * g.hslab + q;
#pragma unroll
        for (int m = 0; m < M; ++m) out[(2 * m + odd) * g.hslab] = a[m];
    }
}

// One wave's quarter r of the x lines of a tile (LX = 64), from the staged
// line in LDS (row: x[n], n < 32).
template <typename R, int Q4>
__device__ __forceinline__ void x64_fwd_quarter(const cplx<R> *row, cplx<R> *out, int64_t hslab, bool on) {
    cplx<R> v[16];
#pragma unroll
    for (int n = 0; n < 16; ++n) {
        const cplx<R> x0 = row[n], x1 = row[n + 16];
        // (-i)^Q4 x1: 1, -i, -1, i
        const cplx<R> r1 = Q4 == 0 ? x1 : Q4 == 1 ? cmake<R>(x1.y, -x1.x) : Q4 == 2 ? cmake<R>(-x1.x, -x1.y)
                                                                                    : cmake<R>(-x1.y, x1.x);
        v[n] = cadd(x0, r1);
        if (Q4 != 0 && n != 0) v[n] = cmul(v[n], twiddle_full<R, 64, false>(Q4 * n));
    }
    fft_reg<R, 16, false>(v);
    if (on) {
#pragma unroll
        for (int m = 0; m < 16; ++m) out[(4 * m + Q4) * hslab] = v[m];
    }
}

// x lines of Fhat -> H at LX = 64, a line per four waves (x4tq above).
template <typename R, bool MASKED>
__global__ void __launch_bounds__(kX4Threads) lat_x_fwd64(LatGeom g, const cplx<R> *__restrict__ F,
                                                         cplx<R> *__restrict__ H) {
    constexpr int M = 32, SP = M + 1, kTW = xtw<R>, TQ = kTQ;
    static_assert(kTW * TQ * 4 == kX4Threads, "one line per lane of every quarter");
    constexpr int CELLS = kTW * TQ * M, NI = (CELLS + kX4Threads - 1) / kX4Threads;
    __shared__ cplx<R> S[kTW * TQ * SP];
    const int t = threadIdx.x;
    const int ex = g.ex, per_w = g.ey * g.ez;
    const XTile tl = x_tile<kTW, TQ>(g, blockIdx.x);
    const cplx<R> *Fc = F + (int64_t)tl.c * g.fstride;
    cplx<R> v[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = t + i * kX4Threads;
        const int wl = e % kTW, r = e / kTW, ql = r / M, x = r % M;
        const int q = tl.q0 + ql, w = tl.w0 + wl;
        bool ok = e < CELLS && x < ex && q < per_w && w < g.n_freq;
        if (MASKED) ok = ok && g.occ[q * ex + x] != 0;
        const cplx<R> y = cload_nt(&Fc[ok ? (int64_t)(q * ex + x) * g.n_freq + w : 0]);
        v[i] = csel(ok, y, czero<R>());
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = t + i * kX4Threads;
        const int wl = e % kTW, r = e / kTW, ql = r / M, x = r % M;
        if (e < CELLS) S[(wl * TQ + ql) * SP + x] = v[i];
    }
    __syncthreads();
    const int r4 = __builtin_amdgcn_readfirstlane((t >> 6) & 3);   // uniform per wave
    const int rl = (t >> 8) * 64 + (t & 63);
    const int q = tl.q0 + rl % TQ, w = tl.w0 + rl / TQ;
    const bool on = q < per_w && w < g.n_freq;
    cplx<R> *out = H + (int64_t)tl.c * g.hstride + (on ? (int64_t)w * 64 * g.hslab + q : 0);
    const cplx<R> *row = S + rl * SP;
    if (r4 == 0) x64_fwd_quarter<R, 0>(row, out, g.hslab, on);
    else if (r4 == 1) x64_fwd_quarter<R, 1>(row, out, g.hslab, on);
    else if (r4 == 2) x64_fwd_quarter<R, 2>(row, out, g.hslab, on);
    else x64_fwd_quarter<R, 3>(row, out, g.hslab, on);
}

// LDS of lat_yz: the zero-padded slabs P [s][z][y] (rows of MY + 1) and the
// slabs after the y DFT Q [s][ky][z] (lines of MZ + 1; the padding element
// keeps the lines a wave reads at once out of one bank).  When every lane
// has at most one y line (LZ <= 2 LY), P lives at the start of Q: each
// step reads its inputs into registers, and a barrier separates those
// reads from the first write into the shared space.
// Slabs per workgroup: one z line per lane of a half (SL = 128 / LY); at
// LZ = 128 (WIDE) each half-line is split over the two waves of its half,
// so one z line per lane of a wave (SL = 64 / LY).
template <int LY, int LZ, int NT = kLatThreads> struct YzLds {
    static constexpr bool WIDE = LZ > 64;
    static constexpr int SL = WIDE ? NT / (4 * LY) : NT / (2 * LY);
    static constexpr int MY = LY / 2, MZ = LZ / 2, PY = MY + 1, QZ = MZ + 1;
    static constexpr int P_ELEMS = SL * MZ * PY, Q_ELEMS = SL * LY * QZ;
    static constexpr bool ALIAS = SL * MZ <= NT / 2 && P_ELEMS <= Q_ELEMS;
    static constexpr int ELEMS = ALIAS ? Q_ELEMS : P_ELEMS + Q_ELEMS;
};

// Step 2 of lat_yz for the lanes of one half (HF: 0 even, 1 odd): the y
// lines (s, z) of the zero-padded slabs in P, every z < MZ, MY inputs ->
// this half's MY outputs, into Q.  Ends with a barrier.  NT: threads of the
// workgroup, NT / 2 lanes per half.
template <typename R, int LY, int LZ, int HF, int NT = kLatThreads>
__device__ __forceinline__ void yz_ydft(cplx<R> *P, cplx<R> *Q, int lane) {
    using L = YzLds<LY, LZ, NT>;
    constexpr int HL = NT / 2;
    constexpr int SL = L::SL;
    constexpr int MY = LY / 2, MZ = LZ / 2;
    constexpr int PY = MY + 1, QZ = MZ + 1;
    constexpr int YLINES = SL * MZ;
    if (L::ALIAS) {
        const int sl = lane / MZ, z = lane % MZ;
        const bool on = lane < YLINES;
        cplx<R> a[MY];
        if (on) {
            const cplx<R> *prow = P + (sl * MZ + z) * PY;
#pragma unroll
            for (int n = 0; n < MY; ++n) a[n] = prow[n];
            if (HF) {
#pragma unroll
                for (int n = 1; n < MY; ++n) a[n] = cmul(a[n], twiddle<R, LY, false>(n));
            }
            fft_reg<R, MY, false>(a);
        }
        __syncthreads();   // P (inside Q) is read
        if (on) {
#pragma unroll
            for (int m = 0; m < MY; ++m) Q[(sl * LY + 2 * m + HF) * QZ + z] = a[m];
        }
    } else {
        for (int line = lane; line < YLINES; line += HL) {
            const int sl = line / MZ, z = line % MZ;
            const cplx<R> *prow = P + (sl * MZ + z) * PY;
            cplx<R> a[MY];
#pragma unroll
            for (int n = 0; n < MY; ++n) a[n] = prow[n];
            if (HF) {
#pragma unroll
                for (int n = 1; n < MY; ++n) a[n] = cmul(a[n], twiddle<R, LY, false>(n));
            }
            fft_reg<R, MY, false>(a);
#pragma unroll
            for (int m = 0; m < MY; ++m) Q[(sl * LY + 2 * m + HF) * QZ + z] = a[m];
        }
    }
    __syncthreads();
}

// Step 4 of lat_yz for one half: the inverse y lines (s, z), z < ez, this
// half's MY inputs -> MY outputs, combined through the line's slab row in P.
// Ends with a barrier.
template <typename R, int LY, int LZ, int HF, int NT = kLatThreads>
__device__ __forceinline__ void yz_yinv(cplx<R> *P, const cplx<R> *Q, int lane, int ez) {
    using L = YzLds<LY, LZ, NT>;
    constexpr int HL = NT / 2;
    constexpr int SL = L::SL;
    constexpr int MY = LY / 2, MZ = LZ / 2;
    constexpr int PY = MY + 1, QZ = MZ + 1;
    constexpr int YLINES = SL * MZ;
    constexpr int YROUNDS = (YLINES + HL - 1) / HL;
    for (int r = 0; r < YROUNDS; ++r) {
        const int line = lane + r * HL;
        const int sl = line / MZ, z = line % MZ;
        const bool on = line < YLINES && z < ez;
        cplx<R> *prow = P + (sl * MZ + z) * PY;
        cplx<R> b[MY];
        if (on) {
#pragma unroll
            for (int m = 0; m < MY; ++m) b[m] = Q[(sl * LY + 2 * m + HF) * QZ + z];
            fft_reg<R, MY, true>(b);
        }
        if (L::ALIAS) __syncthreads();   // Q is read before P (inside Q) is written
        if (on) {
            if (HF) {
#pragma unroll
                for (int j = 0; j < (MY + 1) / 2; ++j) prow[j] = b[j];
            } else {
#pragma unroll
                for (int j = MY / 2; j < MY; ++j) prow[j] = b[j];
            }
        }
        __syncthreads();
        if (on) {
            if (HF) {
#pragma unroll
                for (int j = MY / 2; j < MY; ++j) prow[j] = cmac(prow[j], b[j], twiddle<R, LY, true>(j));
            } else {
#pragma unroll
                for (int j = 0; j < MY / 2; ++j) prow[j] = cmac(b[j], prow[j], twiddle<R, LY, true>(j));
            }
        }
        __syncthreads();
    }
}

// Steps 2-4 of lat_yz for the lanes of one half (HF: 0 even, 1 odd), on
// the zero-padded slabs in P.  Every index that depends on the half is a
// constant here; both halves pass the same barriers in the same order.
template <typename R, int LY, int LZ, int HF, int NT = kLatThreads>
__device__ __forceinline__ void yz_half(const LatGeom &g, const R *__restrict__ Khat, cplx<R> *P, cplx<R> *Q,
                                        const int (*sinfo)[2], int lane, int ez) {
    constexpr int MZ = LZ / 2;
    constexpr int QZ = MZ + 1;
    const int zsl = lane / LY, ky = lane % LY;
    // the spectra this lane's z line is multiplied by in step 3 (kz = 2m + HF),
    // loaded first so that steps 2 and 3 hide the latency
    R kv[MZ];
    {
        const int wr = sinfo[zsl][0], kf = sinfo[zsl][1];
        const int kx = kf & 255, ry = (kf >> 8) & 1, rz = kf >> 9;
        const int kyk = ry ? (LY - ky) % LY : ky;
        // [kz][ky] plane of the slab; a reflected kz runs backwards from kz = LZ
        const R *kc = Khat + ((int64_t)wr * g.lx + kx) * LZ * LY + kyk;
        const int ks = rz ? -LY : LY;
        const R *kp = (rz ? kc + LZ * LY : kc) + HF * ks;   // kz = HF
#pragma unroll
        for (int m = 0; m < MZ; ++m) {
            kv[m] = (HF == 0 && m == 0) ? kc[0] : *kp;
            kp += 2 * ks;
        }
    }
    __builtin_amdgcn_s_setprio(0);   // loads issued: arithmetic at normal priority
    // 2. y lines (s, z), every z < MZ: MY inputs -> this half's MY outputs
    yz_ydft<R, LY, LZ, HF, NT>(P, Q, lane);
    // 3. z lines (s, ky): X[2m + HF] of the line, product with the spectra,
    // inverse half DFT; then the halves combine through the line
    cplx<R> *qline = Q + (zsl * LY + ky) * QZ;
    cplx<R> a[MZ];
#pragma unroll
    for (int n = 0; n < MZ; ++n) a[n] = qline[n];
    if (HF) {
#pragma unroll
        for (int n = 1; n < MZ; ++n) a[n] = cmul(a[n], twiddle<R, LZ, false>(n));
    }
    fft_reg<R, MZ, false>(a);
#pragma unroll
    for (int m = 0; m < MZ; ++m) a[m] = cmake<R>(a[m].x * kv[m], a[m].y * kv[m]);
    fft_reg<R, MZ, true>(a);   // even half: E[n]; odd half: O[n], n < MZ
    __syncthreads();   // every lane has read its line
    // y[n] = E[n] + w^-n O[n]: the even half keeps n < MZ/2, the odd half the rest
    if (HF) {
#pragma unroll
        for (int j = 0; j < (MZ + 1) / 2; ++j) qline[j] = a[j];                      // O[j] for the even half
    } else {
#pragma unroll
        for (int j = MZ / 2; j < MZ; ++j) qline[j] = a[j];                           // E[j] for the odd half
    }
    __syncthreads();
    if (HF) {
#pragma unroll
        for (int j = MZ / 2; j < MZ; ++j) qline[j] = cmac(qline[j], a[j], twiddle<R, LZ, true>(j));
    } else {
#pragma unroll
        for (int j = 0; j < MZ / 2; ++j) qline[j] = cmac(a[j], qline[j], twiddle<R, LZ, true>(j));
    }
    __syncthreads();
    // 4. inverse y lines (s, z), z < ez: this half's MY inputs -> MY
    // outputs, combined through the line's slab row in P
    yz_yinv<R, LY, LZ, HF, NT>(P, Q, lane, ez);
}

// w[q] = exp(-2 pi i q / 128), q < 128, into LDS (threads t < 64 write)
template <typename R> __device__ __forceinline__ void tw128_fill(cplx<R> *w, int t) {
    if (t < 64) {
#pragma unroll
        for (int q = 0; q < 64; ++q)
            if (t == q) {
                w[q] = cmake<R>((R)kTw128[q][0], (R)kTw128[q][1]);
                w[q + 64] = cmake<R>(-(R)kTw128[q][0], -(R)kTw128[q][1]);
            }
    }
}


// Step 3 of lat_yz at LZ = 128 for one wave: its quarter Q4 = HF + 2 ZP of
// every z line of its slabs.  With x[n] the line (n < 64, zero beyond the
// data) and w = exp(-2 pi i / 128), the frequencies kz = 4 j + Q4 are
//     X[4 j + Q4] = DFT_32(v)[j],  v[n] = w^(Q4 n) (x[n] + (-i)^Q4 x[n + 32]),
// and after the product with the spectra and the inverse DFT_32 of each
// quarter (Y_Q4), the outputs n < 64 are
//     y[n + 32 h] = sum_Q4 i^(Q4 h) T_Q4[n],  T_Q4[n] = w^(-Q4 n) Y_Q4[n],
// summed through the line in LDS (quarters 2 and 3 hand theirs to 0 and 1,
// which leave one partial sum each in the line for the other).  All four
// variants pass the same five barriers.
// kb: the spectra row of this lane at its first kz (kz = Q4), ks: the step
// to the next kz (negative for a reflected kz), k0: the row at kz = 0.
template <typename R, int LY, int HF, int ZP>
__device__ __forceinline__ void yz128_zstep(cplx<R> *qline, const R *kb, const R *k0, int ks) {
    constexpr int Q4 = HF + 2 * ZP;
    cplx<R> v[32];
#pragma unroll
    for (int n = 0; n < 32; ++n) {
        const cplx<R> x0 = qline[n], x1 = qline[n + 32];
        // (-i)^Q4 x1: 1, -i, -1, i
        const cplx<R> r1 = Q4 == 0 ? x1 : Q4 == 1 ? cmake<R>(x1.y, -x1.x) : Q4 == 2 ? cmake<R>(-x1.x, -x1.y)
                                                                                    : cmake<R>(-x1.y, x1.x);
        v[n] = cadd(x0, r1);
        if (Q4 != 0 && n != 0) v[n] = cmul(v[n], twiddle_full<R, 128, false>(Q4 * n));
    }
    // the spectra at kz = 4 j + Q4, loaded here so that the forward DFT
    // hides their latency (earlier they would be live through the y DFT)
    R kv[32];
    kv[0] = Q4 == 0 ? *k0 : *kb;
    const R *kp = kb;
#pragma unroll
    for (int j = 1; j < 32; ++j) {
        kp += 4 * ks;
        kv[j] = *kp;
    }
    fft_reg<R, 32, false>(v);
#pragma unroll
    for (int j = 0; j < 32; ++j) v[j] = cmake<R>(v[j].x * kv[j], v[j].y * kv[j]);
    fft_reg<R, 32, true>(v);
    if (Q4 != 0) {
#pragma unroll
        for (int n = 1; n < 32; ++n) v[n] = cmul(v[n], twiddle_full<R, 128, true>(Q4 * n));
    }
    __syncthreads();   // (1) every lane has read its line
    if (ZP) {
        // quarters 2 and 3 hand over T_2 (at n) and T_3 (at n + 32)
#pragma unroll
        for (int n = 0; n < 32; ++n) qline[n + 32 * HF] = v[n];
        __syncthreads();   // (2)
        __syncthreads();   // (3)
        __syncthreads();   // (4)
        __syncthreads();   // (5)
    } else {
        __syncthreads();   // (2)
        // quarter 0: A = T0 + T2 kept, B = T0 - T2 left at n;
        // quarter 1: D = i (T1 - T3) kept, C = T1 + T3 left at n + 32
#pragma unroll
        for (int n = 0; n < 32; ++n) {
            const cplx<R> o = qline[n + 32 * HF];
            if (HF) {
                qline[n + 32] = cadd(v[n], o);
                const cplx<R> d = csub(v[n], o);
                v[n] = cmake<R>(-d.y, d.x);
            } else {
                qline[n] = csub(v[n], o);
                v[n] = cadd(v[n], o);
            }
        }
        __syncthreads();   // (3)
        // quarter 0: y[n] = A + C; quarter 1: y[n + 32] = D + B
#pragma unroll
        for (int n = 0; n < 32; ++n) v[n] = cadd(v[n], qline[n + 32 * (1 - HF)]);
        __syncthreads();   // (4) C and B are read
#pragma unroll
        for (int n = 0; n < 32; ++n) qline[n + 32 * HF] = v[n];
        __syncthreads();   // (5)
    }
}

// Steps 2-4 of lat_yz at LZ = 128 for the lanes of one half (HF); the two
// waves of the half (zp) take the two quarters of its z frequencies.
template <typename R, int LY, int HF>
__device__ __forceinline__ void yz128_half(const LatGeom &g, const R *__restrict__ Khat, cplx<R> *P, cplx<R> *Q,
                                           const int (*sinfo)[2], int lane, int ez) {
    constexpr int LZ = 128, QZ = LZ / 2 + 1;
    const int zp = __builtin_amdgcn_readfirstlane(lane >> 6);   // uniform per wave
    const int l64 = lane & 63;
    const int zsl = l64 / LY, ky = l64 % LY;
    // spectra rows of this lane's z line, kz = 4 j + 2 zp + HF
    const int wr = sinfo[zsl][0], kf = sinfo[zsl][1];
    const int kx = kf & 255, ry = (kf >> 8) & 1, rz = kf >> 9;
    const int kyk = ry ? (LY - ky) % LY : ky;
    const R *kc = Khat + ((int64_t)wr * g.lx + kx) * LZ * LY + kyk;
    const int ks = rz ? -LY : LY;
    // a reflected kz runs backwards from kz = LZ; kz = 0 is its own reflection
    const R *kb = (rz ? kc + LZ * LY : kc) + (2 * zp + HF) * ks;
    __builtin_amdgcn_s_setprio(0);   // the slab loads are done: arithmetic at normal priority
    yz_ydft<R, LY, LZ, HF>(P, Q, lane);
    cplx<R> *qline = Q + (zsl * LY + ky) * QZ;
    if (zp) yz128_zstep<R, LY, HF, 1>(qline, kb, kc, ks);
    else yz128_zstep<R, LY, HF, 0>(qline, kb, kc, ks);
    yz_yinv<R, LY, LZ, HF>(P, Q, lane, ez);
}

// One (c, omega, kx) slab of H per 2 Ly lanes: y DFT, z DFT, product with
// the spectra, inverse z and y DFTs, in place.  The two halves of every
// line are taken by lanes of different waves (waves 0-1 the even half,
// waves 2-3 the odd half); each half runs its own copy of the line code
// (yz_half), so no index or twiddle depends on the half at run time, and
// the halves meet through LDS.
// Frequencies are taken in the order worder[] (spectrum positions, a
// permutation of the n_freq block frequencies that puts the y/z reflections
// of a frequency next to each other), and workgroups are renumbered so that
// consecutive ones run on one XCD: the reflections share one stored Khat
// plane, which is then read from HBM once and from that XCD's L2 for the
// others.
// Occupancy: 4 workgroups per CU up to LY, LZ = 32; at LZ = 64 the z lines
// of a lane take twice the registers and Q twice the LDS (at LY = 64 the y
// lines), so 2; at LZ = 128 a lane holds a quarter line (as many registers
// as at 64).
template <typename R, int LY, int LZ>
__global__ void __launch_bounds__(kLatThreads) __attribute__((amdgpu_waves_per_eu(LZ <= 32 && LY <= 32 ? 4 : 2))) lat_yz(LatGeom g, cplx<R> *__restrict__ H, const R *__restrict__ Khat,
                                                      const int *__restrict__ worder) {
    constexpr int HL = kLatThreads / 2;                 // lanes per half
    constexpr int SL = YzLds<LY, LZ>::SL;               // slabs per workgroup
    constexpr int MY = LY / 2, MZ = LZ / 2;
    // rows padded by one element: unpadded, the lines a wave reads at once
    // start 256 B apart and fall into one LDS bank
    constexpr int PY = MY + 1;
    constexpr int CELLS = SL * MZ * MY;                 // slab cells zero-padded to MZ x MY
    using L = YzLds<LY, LZ>;
    __shared__ cplx<R> lds[L::ELEMS];
    cplx<R> *Q = lds;                                   // after the y DFT [s][ky][z]
    cplx<R> *P = L::ALIAS ? lds : lds + L::Q_ELEMS;     // slab [s][z][y]
    // per slab: H offset (-1 past the last slab), stored frequency, kx and reflections
    __shared__ int64_t hbase[SL];
    __shared__ int sinfo[SL][2];
    const int t = threadIdx.x;
    // wave priority: a wave issuing its slab and spectra loads (or, at the
    // end, its stores) goes ahead of the waves in their DFT phases, so the
    // memory requests of one workgroup overlap the arithmetic of the others
    // (1.53 -> 1.42 ms at 32 x 32 x 32)
    __builtin_amdgcn_s_setprio(2);
    const int half = __builtin_amdgcn_readfirstlane(t / HL), lane = t % HL;   // half: uniform per wave
    const int ey = g.ey, ez = g.ez;
    // slab counts fit in 32 bits (the launch checks nc * n_freq * lx)
    const int per_c = g.n_freq * g.lx;                  // slabs per component
    const int n_slabs = g.nc * per_c;
    const int s0 = (int)xcd_order(blockIdx.x, gridDim.x) * SL;
    if (t < SL) {
        const int si = s0 + t;
        const bool live = si < n_slabs;
        const int wk = live ? si % per_c : 0;
        // slabs (frequency, kx), kx fastest; at LZ = 128 (one slab per
        // workgroup, 64 KB spectra planes) frequency fastest, so that the
        // reflections sharing a spectra plane run next to each other
        const int p = worder[L::WIDE ? wk % g.n_freq : wk / g.lx], kx = L::WIDE ? wk / g.n_freq : wk % g.lx;
        // spectrum position p -> block frequency (fx, fyv, fzv) -> stored
        // frequency (ky, kz in [0, N/2]) and reflections
        const int N = g.N, Hh = N / 2 + 1;
        int fx, fyv, fzv;
        spec_freq(N, p, fx, fyv, fzv);
        const int ry = fyv > N / 2, rz = fzv > N / 2;
        hbase[t] = live ? (int64_t)(si / per_c) * g.hstride + ((int64_t)p * g.lx + kx) * g.hslab : -1;
        sinfo[t][0] = ((rz ? N - fzv : fzv) * Hh + (ry ? N - fyv : fyv)) * Hh + fx;
        sinfo[t][1] = kx | ry << 8 | rz << 9;
    }
    __syncthreads();
    // 1. load the slabs, zero-padded to MZ x MY (slabs past the end: zero);
    // all loads are issued before the first is waited on (cells outside the
    // data read element 0 and are replaced by zero)
    constexpr int NI = (CELLS + kLatThreads - 1) / kLatThreads;
    cplx<R> v[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = t + i * kLatThreads;
        const int sl = e / (MZ * MY), z = (e / MY) % MZ, y = e % MY;
        const int64_t hb = e < CELLS ? hbase[sl] : -1;
        const bool ok = hb >= 0 && y < ey && z < ez;
        const cplx<R> x = cload_nt(&H[ok ? hb + z * ey + y : 0]);
        v[i] = csel(ok, x, czero<R>());
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = t + i * kLatThreads;
        const int sl = e / (MZ * MY), z = (e / MY) % MZ, y = e % MY;
        if (e < CELLS) P[(sl * MZ + z) * PY + y] = v[i];
    }
    __syncthreads();
    // 2-4, each wave in its half's copy (the same barriers in both)
    if constexpr (L::WIDE) {
        if (half) yz128_half<R, LY, 1>(g, Khat, P, Q, sinfo, lane, ez);
        else yz128_half<R, LY, 0>(g, Khat, P, Q, sinfo, lane, ez);
    } else {
        if (half) yz_half<R, LY, LZ, 1>(g, Khat, P, Q, sinfo, lane, ez);
        else yz_half<R, LY, LZ, 0>(g, Khat, P, Q, sinfo, lane, ez);
    }
    __builtin_amdgcn_s_setprio(2);
    // 5. store the slabs back (streaming stores: lat_x_inv reads them from HBM)
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = t + i * kLatThreads;
        const int sl = e / (MZ * MY), z = (e / MY) % MZ, y = e % MY;
        const int64_t hb = e < CELLS ? hbase[sl] : -1;
        if (hb >= 0 && y < ey && z < ez) cstore_nt(&H[hb + z * ey + y], P[(sl * MZ + z) * PY + y]);
    }
}

// The whole lattice MAC of one frequency at lengths 32 x 32 x 32 (boxes up
// to 16 blocks per axis), in LDS: a workgroup takes (component, frequency,
// kx parity h) and the 16 kx = 2 m + h of that frequency.  With x[n] an x
// line (n < 16, zero beyond the data) and w = exp(-2 pi i / 32),
//     X[2 m + h] = DFT_16(w^(h n) x[n])[m]
// fills 16 slabs [m][z][y]; they go through the y/z steps of lat_yz (16
// slabs per 1024 threads, so the slab cells never leave LDS), and the
// inverse x lines keep n < 16 of
//     y[n] = IDFT_16(Y[2 m])[n] + w^(-n) IDFT_16(Y[2 m + 1])[n]:
// parity 0 writes its term into U0, parity 1 its term into U1, and the
// inverse block FFT adds the two.  Fhat is read and each term written once,
// where the three-pass split writes the box after the x DFT (H) once and
// reads it twice; but a workgroup reads and writes 16 bytes per slot (one
// frequency of the block-major spectra), so the frequencies of one
// 128-byte run go to neighbouring workgroups: the two parities of a
// frequency run next to each other and frequencies in spectrum order, and
// the loads and stores go through L2 (streaming stores of partial lines
// measured 2x slower).  MASKED: slots without a source block (g.occ) read
// as zero.
constexpr int kFuThreads = 1024;

template <typename R, bool MASKED>
__global__ void __launch_bounds__(kFuThreads) lat_fused(LatGeom g, const cplx<R> *__restrict__ F,
                                                       const R *__restrict__ Khat, cplx<R> *__restrict__ U0,
                                                       cplx<R> *__restrict__ U1) {
    constexpr int L = 32, M = 16;
    using Y = YzLds<L, L, kFuThreads>;
    static_assert(Y::SL == M && Y::ALIAS, "one slab per kx of a parity, the slabs inside Q");
    constexpr int PY = M + 1;                             // slab rows [m][z][y] (lat_yz's P)
    constexpr int SX = M + 1;                             // staged x lines [z][y][x]
    static_assert(Y::P_ELEMS + M * M * SX <= Y::ELEMS, "the staged lines fit beside the slabs");
    constexpr int NI = M * M * M / kFuThreads;
    __shared__ cplx<R> lds[Y::ELEMS];
    __shared__ int sinfo[M][2];
    cplx<R> *P = lds, *Q = lds, *S = lds + Y::P_ELEMS;
    const int t = threadIdx.x;
    const int item = (int)xcd_order(blockIdx.x, gridDim.x);
    const int h = item & 1, wc = item >> 1;
    const int c = wc / g.n_freq, p = wc % g.n_freq;
    const int ex = g.ex, ey = g.ey, ez = g.ez;
    if (t < M) {
        const int N = g.N, Hh = N / 2 + 1;
        int fx, fyv, fzv;
        spec_freq(N, p, fx, fyv, fzv);
        const int ry = fyv > N / 2, rz = fzv > N / 2;
        sinfo[t][0] = ((rz ? N - fzv : fzv) * Hh + (ry ? N - fyv : fyv)) * Hh + fx;
        sinfo[t][1] = (2 * t + h) | ry << 8 | rz << 9;
    }
    // 1. the frequency's value in every slot, staged as x lines (all loads
    // issued before the first is waited on; cells outside the data read
    // element 0 and are replaced by zero)
    const cplx<R> *Fc = F + (int64_t)c * g.fstride;
    cplx<R> v[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = t + i * kFuThreads;
        const int x = e % M, y = (e / M) % M, z = e / (M * M);
        const int slot = (z * ey + y) * ex + x;
        bool ok = x < ex && y < ey && z < ez;
        if (MASKED) ok = ok && g.occ[ok ? slot : 0] != 0;
        const cplx<R> f = Fc[ok ? (int64_t)slot * g.n_freq + p : 0];
        v[i] = csel(ok, f, czero<R>());
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = t + i * kFuThreads;
        S[(e / M) * SX + e % M] = v[i];
    }
    __syncthreads();
    // 2. x DFTs of this parity: line (y, z) -> slab row m (zero where the
    // line holds no data, as lat_yz's zero-padded slabs)
    if (t < M * M) {
        const int y = t % M, z = t / M;
        cplx<R> a[M];
#pragma unroll
        for (int n = 0; n < M; ++n) a[n] = S[t * SX + n];
        if (h) {
#pragma unroll
            for (int n = 1; n < M; ++n) a[n] = cmul(a[n], twiddle<R, L, false>(n));
        }
        fft_reg<R, M, false>(a);
#pragma unroll
        for (int m = 0; m < M; ++m) P[(m * M + z) * PY + y] = a[m];
    }
    __syncthreads();
    // 3. y DFTs, z DFTs, product with the spectra, inverse z and y DFTs of
    // the 16 slabs (each wave in its half's copy; ends with a barrier)
    const int half = __builtin_amdgcn_readfirstlane(t / (kFuThreads / 2)), lane = t % (kFuThreads / 2);
    if (half) yz_half<R, L, L, 1, kFuThreads>(g, Khat, P, Q, sinfo, lane, ez);
    else yz_half<R, L, L, 0, kFuThreads>(g, Khat, P, Q, sinfo, lane, ez);
    // 4. inverse x DFTs of this parity over the slabs, this parity's term
    // of the outputs n < ex
    if (t < M * M) {
        const int y = t % M, z = t / M;
        if (y < ey && z < ez) {
            cplx<R> b[M];
#pragma unroll
            for (int m = 0; m < M; ++m) b[m] = P[(m * M + z) * PY + y];
            fft_reg<R, M, true>(b);
            if (h) {
#pragma unroll
                for (int n = 1; n < M; ++n) b[n] = cmul(b[n], twiddle<R, L, true>(n));
            }
            cplx<R> *out = (h ? U1 : U0) + (int64_t)c * g.fstride + (int64_t)((z * ey + y) * ex) * g.n_freq + p;
#pragma unroll
            for (int n = 0; n < M; ++n)
                if (n < ex) out[(int64_t)n * g.n_freq] = b[n];
        }
    }
}

// Inverse x lines of H, cropped to the box, -> Uhat, tile by tile as in
// lat_x_fwd (staged through LDS so that each slot's kTW frequencies are
// stored as one run).  Every lane reaches the exchange.
template <typename R, int LX>
__global__ void __launch_bounds__(xthreads<R>) lat_x_inv(LatGeom g, const cplx<R> *__restrict__ H,
                                                         cplx<R> *__restrict__ U) {
    constexpr int M = LX / 2, SP = M + 1, kTW = xtw<R>, kXThreads = xthreads<R>;   // rows padded against bank conflicts
    constexpr int CELLS = kTW * kTQ * M, NI = (CELLS + kXThreads - 1) / kXThreads;
    __shared__ cplx<R> S[kTW * kTQ * SP];
    const int t = threadIdx.x;
    const int ex = g.ex, per_w = g.ey * g.ez;
    const XTile tl = x_tile<kTW>(g, blockIdx.x);
    const int rl = t >> 1, odd = t & 1;
    const int q = tl.q0 + rl % kTQ, w = tl.w0 + rl / kTQ;
    const bool on = q < per_w && w < g.n_freq;
    // lines outside the data read the tile's first line (their results are dropped)
    const cplx<R> *in = H + (int64_t)tl.c * g.hstride + (on ? (int64_t)w * LX * g.hslab + q : 0);
    cplx<R> a[M];
#pragma unroll
    for (int m = 0; m < M; ++m) a[m] = cload_nt(&in[(2 * m + odd) * g.hslab]);
    cplx<R> out[LX / 4];
    pair_inv<R, LX>(a, odd, out);
#pragma unroll
    for (int j = 0; j < LX / 4; ++j) S[rl * SP + (odd ? M / 2 + j : j)] = out[j];
    __syncthreads();
    cplx<R> *Uc = U + (int64_t)tl.c * g.fstride;
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int e = t + i * kXThreads;
        const int wl = e % kTW, r = e / kTW, ql = r / M, x = r % M;
        const int q2 = tl.q0 + ql, w2 = tl.w0 + wl;
        if (e < CELLS && x < ex && q2 < per_w && w2 < g.n_freq)
            cstore_nt(&Uc[(int64_t)(q2 * ex + x) * g.n_freq + w2], S[(wl * kTQ + ql) * SP + x]);
    }
}

// ---- lattice spectra ----

// K_d(omega) for a lattice offset d from the octant table T[omega][dy][dz][dx]
// (offsets >= 0): a negative dy (dz) takes the row at -ky (-kz); a negative
// dx takes the complex conjugate of the row at (-ky, -kz) (half spectrum in kx).
template <typename R>
__device__ __forceinline__ cplx<R> octant_value(const LatSpecGeom &s, const cplx<R> *__restrict__ T, int w, int dx,
                                                int dy, int dz) {
    const int N = s.N, Hh = N / 2 + 1;
    const int kx = w % Hh, ky = (w / Hh) % N, kz = w / (Hh * N);
    const bool fx = dx < 0;
    const bool fy = (dy < 0) != fx, fz = (dz < 0) != fx;
    const int ky2 = fy ? (N - ky) % N : ky, kz2 = fz ? (N - kz) % N : kz;
    const int64_t row = ((int64_t)kz2 * N + ky2) * Hh + kx;
    const int64_t kper = (int64_t)s.XD * s.YD * s.ZD;
    cplx<R> v = T[row * kper + ((int64_t)abs(dy) * s.ZD + abs(dz)) * s.XD + abs(dx)];
    if (fx) v.y = -v.y;
    return v;
}

// lattice position p in [0, L) -> offset, or a flag for the unused p = L/2
__device__ __forceinline__ int lat_offset(int p, int L, bool &used) {
    used = L == 1 || 2 * p != L;
    return 2 * p < L ? p : p - L;
}

// stored frequency index -> block frequency omega (ky, kz in [0, N/2])
__device__ __forceinline__ int stored_omega(int wr, int N) {
    const int Hh = N / 2 + 1;
    const int kx = wr % Hh, ky = (wr / Hh) % Hh, kz = wr / (Hh * Hh);
    return (kz * N + ky) * Hh + kx;
}

// One (stored omega, pz) plane per workgroup: gather K_d, DFT along x then
// y, into S[wl][pz][ky][kx].
template <typename R, int LX, int LY>
__global__ void __launch_bounds__(kLatThreads) latspec_xy(LatSpecGeom s, const cplx<R> *__restrict__ T,
                                                          cplx<R> *__restrict__ S, int w0, int nw) {
    __shared__ cplx<R> X[LY * LX];
    const int t = threadIdx.x;
    const int wl = blockIdx.x / s.lz, pz = blockIdx.x % s.lz;
    if (wl >= nw) return;
    const int w = stored_omega(w0 + wl, s.N);
    bool uz;
    const int dz = lat_offset(pz, s.lz, uz);
    for (int py = t; py < LY; py += kLatThreads) {
        bool uy;
        const int dy = lat_offset(py, LY, uy);
        cplx<R> a[LX];
#pragma unroll
        for (int px = 0; px < LX; ++px) {
            bool ux;
            const int dx = lat_offset(px, LX, ux);
            a[px] = (ux && uy && uz) ? octant_value<R>(s, T, w, dx, dy, dz) : czero<R>();
        }
        fft_reg<R, LX, false>(a);
#pragma unroll
        for (int kx = 0; kx < LX; ++kx) X[py * LX + kx] = a[kx];
    }
    __syncthreads();
    for (int kx = t; kx < LX; kx += kLatThreads) {
        cplx<R> a[LY];
#pragma unroll
        for (int py = 0; py < LY; ++py) a[py] = X[py * LX + kx];
        fft_reg<R, LY, false>(a);
        cplx<R> *out = S + ((int64_t)wl * s.lz + pz) * (LY * LX) + kx;
#pragma unroll
        for (int ky = 0; ky < LY; ++ky) out[ky * LX] = a[ky];
    }
}

// z DFT of each column of S; the real part, scaled, into
// Khat[wr][kx][kz][ky].
template <typename R, int LZ>
__global__ void __launch_bounds__(kLatThreads) latspec_z(LatSpecGeom s, const cplx<R> *__restrict__ S,
                                                         R *__restrict__ Khat, int w0, int nw, R scale) {
    const int64_t plane = (int64_t)s.lx * s.ly;
    const int64_t col = (int64_t)blockIdx.x * kLatThreads + threadIdx.x;
    if (col >= (int64_t)nw * plane) return;
    const int64_t wl = col / plane, q = col % plane;
    const int ky = (int)(q / s.lx), kx = (int)(q % s.lx);
    cplx<R> a[LZ];
#pragma unroll
    for (int pz = 0; pz < LZ; ++pz) a[pz] = S[(wl * LZ + pz) * plane + q];
    fft_reg<R, LZ, false>(a);
    R *out = Khat + ((int64_t)(w0 + wl) * s.lx + kx) * LZ * s.ly + ky;
#pragma unroll
    for (int kz = 0; kz < LZ; ++kz) out[kz * s.ly] = a[kz].x * scale;
}

// Lattice spectra for lengths beyond the register kernels (x or y of 64, z
// of 128): the same gather and DFTs, each DFT summed directly from a line
// in LDS (once per context; O(L) per output), with the twiddles of
// tw128_fill.

constexpr int kWideXY = 64 * 64;   // largest x-y plane of the wide build

// One (stored omega, pz) plane per workgroup: gather K_d into LDS, DFT along
// x, then along y, into S[wl][pz][ky][kx].
template <typename R>
__global__ void __launch_bounds__(kLatThreads) latspec_wide_xy(LatSpecGeom s, const cplx<R> *__restrict__ T,
                                                               cplx<R> *__restrict__ S, int w0, int nw) {
    __shared__ cplx<R> X[kWideXY];
    __shared__ cplx<R> w[128];
    constexpr int PER = kWideXY / kLatThreads;
    const int t = threadIdx.x;
    const int lx = s.lx, ly = s.ly, n = lx * ly;
    const int wl = blockIdx.x / s.lz, pz = blockIdx.x % s.lz;
    if (wl >= nw) return;
    tw128_fill(w, t);
    const int om = stored_omega(w0 + wl, s.N);
    bool uz;
    const int dz = lat_offset(pz, s.lz, uz);
    for (int e = t; e < n; e += kLatThreads) {
        const int py = e / lx, px = e % lx;
        bool ux, uy;
        const int dx = lat_offset(px, lx, ux), dy = lat_offset(py, ly, uy);
        X[e] = (ux && uy && uz) ? octant_value<R>(s, T, om, dx, dy, dz) : czero<R>();
    }
    __syncthreads();
    const int sx = 128 / lx, sy = 128 / ly;
    cplx<R> acc[PER];
    // x: X[py][kx] = sum_px X[py][px] w^(kx px)
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = t + i * kLatThreads;
        acc[i] = czero<R>();
        if (e < n) {
            const int py = e / lx, kx = e % lx;
            for (int px = 0; px < lx; ++px) acc[i] = cmac(acc[i], X[py * lx + px], w[(kx * px % lx) * sx]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < PER; ++i)
        if (t + i * kLatThreads < n) X[t + i * kLatThreads] = acc[i];
    __syncthreads();
    // y: X[ky][kx] = sum_py X[py][kx] w^(ky py)
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int e = t + i * kLatThreads;
        acc[i] = czero<R>();
        if (e < n) {
            const int ky = e / lx, kx = e % lx;
            for (int py = 0; py < ly; ++py) acc[i] = cmac(acc[i], X[py * lx + kx], w[(ky * py % ly) * sy]);
        }
    }
    cplx<R> *out = S + ((int64_t)wl * s.lz + pz) * n;
#pragma unroll
    for (int i = 0; i < PER; ++i)
        if (t + i * kLatThreads < n) out[t + i * kLatThreads] = acc[i];
}

// z DFT of 16 consecutive columns (ky, kx) of S per workgroup; the real
// part, scaled, into Khat[wr][kx][kz][ky].
constexpr int kWideCols = 16;
template <typename R>
__global__ void __launch_bounds__(kLatThreads) latspec_wide_z(LatSpecGeom s, const cplx<R> *__restrict__ S,
                                                              R *__restrict__ Khat, int w0, int nw, R scale) {
    __shared__ cplx<R> C[128 * kWideCols];
    __shared__ cplx<R> w[128];
    const int t = threadIdx.x;
    const int lz = s.lz;
    const int64_t plane = (int64_t)s.lx * s.ly;
    const int64_t col0 = (int64_t)blockIdx.x * kWideCols;
    const int64_t n_cols = (int64_t)nw * plane;
    tw128_fill(w, t);
    for (int e = t; e < lz * kWideCols; e += kLatThreads) {
        const int pz = e / kWideCols, c = e % kWideCols;
        const int64_t col = col0 + c;
        C[e] = col < n_cols ? S[((col / plane) * lz + pz) * plane + col % plane] : czero<R>();
    }
    __syncthreads();
    const int sz = 128 / lz;
    for (int e = t; e < lz * kWideCols; e += kLatThreads) {
        const int kz = e / kWideCols, c = e % kWideCols;
        const int64_t col = col0 + c;
        if (col >= n_cols) continue;
        cplx<R> acc = czero<R>();
        for (int pz = 0; pz < lz; ++pz) acc = cmac(acc, C[pz * kWideCols + c], w[(kz * pz % lz) * sz]);
        const int64_t wl = col / plane, q = col % plane;
        const int ky = (int)(q / s.lx), kx = (int)(q % s.lx);
        Khat[(((int64_t)(w0 + wl) * s.lx + kx) * lz + kz) * s.ly + ky] = acc.x * scale;
    }
}

// ---- dispatch over the compiled lattice lengths ----

template <typename F> hipError_t with_len(int L, F &&f) {
    switch (L) {
    case 4: return f(std::integral_constant<int, 4>());
    case 8: return f(std::integral_constant<int, 8>());
    case 16: return f(std::integral_constant<int, 16>());
    case 32: return f(std::integral_constant<int, 32>());
    default: return hipErrorInvalidValue;
    }
}

// z lengths of the register spectra build: also 64
template <typename F> hipError_t with_zlen(int L, F &&f) {
    if (L == 64) return f(std::integral_constant<int, 64>());
    return with_len(L, static_cast<F &&>(f));
}

// x and y lengths of the MAC kernels: also 64 (boxes up to 32 blocks)
template <typename F> hipError_t with_xlen(int L, F &&f) {
    if (L == 64) return f(std::integral_constant<int, 64>());
    return with_len(L, static_cast<F &&>(f));
}

// z lengths of lat_yz: also 64 and 128 (boxes up to 64 blocks; at 128 a
// z half-line is split over two waves)
template <typename F> hipError_t with_yz_zlen(int L, F &&f) {
    if (L == 128) return f(std::integral_constant<int, 128>());
    return with_zlen(L, static_cast<F &&>(f));
}

// workgroups of the x kernels: one per (component, frequency tile, row tile)
template <typename R> unsigned x_tiles(const LatGeom &g, int tq) {
    const int per_w = g.ey * g.ez;
    return (unsigned)((int64_t)g.nc * ((g.n_freq + xtw<R> - 1) / xtw<R>) * ((per_w + tq - 1) / tq));
}

template <typename R> hipError_t fwd_impl(const LatGeom &g, const void *F, void *H, hipStream_t s) {
    if constexpr (std::is_same<R, double>::value) {
        if (g.lx == 64) {
            const unsigned blocks = x_tiles<R>(g, kTQ);
            if (g.occ)
                hipLaunchKernelGGL((lat_x_fwd64<R, true>), dim3(blocks), dim3(kX4Threads), 0, s, g,
                                   (const cplx<R> *)F, (cplx<R> *)H);
            else
                hipLaunchKernelGGL((lat_x_fwd64<R, false>), dim3(blocks), dim3(kX4Threads), 0, s, g,
                                   (const cplx<R> *)F, (cplx<R> *)H);
            return hipGetLastError();
        }
    }
    const unsigned blocks = x_tiles<R>(g, kTQ);
    return with_xlen(g.lx, [&](auto lx) {
        constexpr int LX = decltype(lx)::value;
        if (g.occ)
            hipLaunchKernelGGL((lat_x_fwd<R, LX, true>), dim3(blocks), dim3(xthreads<R>), 0, s, g, (const cplx<R> *)F,
                               (cplx<R> *)H);
        else
            hipLaunchKernelGGL((lat_x_fwd<R, LX, false>), dim3(blocks), dim3(xthreads<R>), 0, s, g, (const cplx<R> *)F,
                               (cplx<R> *)H);
        return hipGetLastError();
    });
}

template <typename R>
hipError_t yz_impl(const LatGeom &g, void *H, const void *Khat, const int *worder, hipStream_t s) {
    const int64_t slabs = (int64_t)g.nc * g.n_freq * g.lx;
    if (slabs >= INT32_MAX) return hipErrorInvalidValue;   // the kernel counts slabs in 32 bits
    return with_xlen(g.ly, [&](auto ly) {
        return with_yz_zlen(g.lz, [&](auto lz) {
            constexpr int LY = decltype(ly)::value, LZ = decltype(lz)::value;
            constexpr int SL = YzLds<LY, LZ>::SL;
            hipLaunchKernelGGL((lat_yz<R, LY, LZ>), dim3((unsigned)((slabs + SL - 1) / SL)), dim3(kLatThreads), 0,
                               s, g, (cplx<R> *)H, (const R *)Khat, worder);
            return hipGetLastError();
        });
    });
}

template <typename R>
hipError_t fused_impl(const LatGeom &g, const void *F, const void *Khat, void *U0, void *U1, hipStream_t s) {
    const int64_t items = (int64_t)g.nc * g.n_freq * 2;
    if (items >= INT32_MAX) return hipErrorInvalidValue;   // the kernel counts items in 32 bits
    if (g.occ)
        hipLaunchKernelGGL((lat_fused<R, true>), dim3((unsigned)items), dim3(kFuThreads), 0, s, g,
                           (const cplx<R> *)F, (const R *)Khat, (cplx<R> *)U0, (cplx<R> *)U1);
    else
        hipLaunchKernelGGL((lat_fused<R, false>), dim3((unsigned)items), dim3(kFuThreads), 0, s, g,
                           (const cplx<R> *)F, (const R *)Khat, (cplx<R> *)U0, (cplx<R> *)U1);
    return hipGetLastError();
}

template <typename R> hipError_t inv_impl(const LatGeom &g, const void *H, void *U, hipStream_t s) {
    const unsigned blocks = x_tiles<R>(g, kTQ);
    return with_xlen(g.lx, [&](auto lx) {
        constexpr int LX = decltype(lx)::value;
        hipLaunchKernelGGL((lat_x_inv<R, LX>), dim3(blocks), dim3(xthreads<R>), 0, s, g, (const cplx<R> *)H,
                           (cplx<R> *)U);
        return hipGetLastError();
    });
}

template <typename R> hipError_t spec_impl(const LatSpecGeom &sg, const void *T, void *Khat, void *scratch,
                                           size_t scratch_bytes, hipStream_t s) {
    const int64_t per_w = (int64_t)sg.lx * sg.ly * sg.lz;
    const int64_t chunk = std::max<int64_t>(1, (int64_t)(scratch_bytes / (sizeof(cplx<R>) * per_w)));
    const R scale = (R)(1.0 / (double)per_w);
    const int n_stored = lattice_stored_freqs(sg.N);
    const bool wide = sg.lx > 32 || sg.ly > 32 || sg.lz > 64;
    for (int64_t w0 = 0; w0 < n_stored; w0 += chunk) {
        const int nw = (int)std::min<int64_t>(chunk, n_stored - w0);
        if (wide) {
            hipLaunchKernelGGL((latspec_wide_xy<R>), dim3((unsigned)(nw * sg.lz)), dim3(kLatThreads), 0, s, sg,
                               (const cplx<R> *)T, (cplx<R> *)scratch, (int)w0, nw);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            const int64_t cols = (int64_t)nw * sg.lx * sg.ly;
            hipLaunchKernelGGL((latspec_wide_z<R>), dim3((unsigned)((cols + kWideCols - 1) / kWideCols)),
                               dim3(kLatThreads), 0, s, sg, (const cplx<R> *)scratch, (R *)Khat, (int)w0, nw, scale);
            e = hipGetLastError();
            if (e != hipSuccess) return e;
            continue;
        }
        hipError_t e = with_len(sg.lx, [&](auto lx) {
            return with_len(sg.ly, [&](auto ly) {
                constexpr int LX = decltype(lx)::value, LY = decltype(ly)::value;
                hipLaunchKernelGGL((latspec_xy<R, LX, LY>), dim3((unsigned)(nw * sg.lz)), dim3(kLatThreads), 0, s,
                                   sg, (const cplx<R> *)T, (cplx<R> *)scratch, (int)w0, nw);
                return hipGetLastError();
            });
        });
        if (e != hipSuccess) return e;
        const int64_t cols = (int64_t)nw * sg.lx * sg.ly;
        e = with_zlen(sg.lz, [&](auto lz) {
            constexpr int LZ = decltype(lz)::value;
            hipLaunchKernelGGL((latspec_z<R, LZ>), dim3((unsigned)((cols + kLatThreads - 1) / kLatThreads)),
                               dim3(kLatThreads), 0, s, sg, (const cplx<R> *)scratch, (R *)Khat, (int)w0, nw, scale);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

bool lattice_len_ok(int L) { return L == 4 || L == 8 || L == 16 || L == 32 || L == 64; }

bool lattice_zlen_ok(int L) { return lattice_len_ok(L) || L == 128; }

int lattice_len(int extent) {
    int L = 4;
    while (L < 2 * extent - 1) L *= 2;
    return L;
}

int lattice_stored_freqs(int N) { return (N / 2 + 1) * (N / 2 + 1) * (N / 2 + 1); }

static bool geom_ok(const LatGeom &g) {
    return lattice_len_ok(g.lx) && lattice_len_ok(g.ly) && lattice_zlen_ok(g.lz) && g.nc >= 1 && g.ex >= 1 &&
           g.ey >= 1 && g.ez >= 1 && 2 * g.ex <= g.lx && 2 * g.ey <= g.ly && 2 * g.ez <= g.lz && g.N >= 2 &&
           g.n_freq == g.N * g.N * (g.N / 2 + 1) && g.n_slots == (int64_t)g.ex * g.ey * g.ez &&
           g.fstride >= (int64_t)g.n_freq * g.n_slots &&
           g.hslab >= g.ey * g.ez && g.hstride >= (int64_t)g.n_freq * g.lx * g.hslab;
}

hipError_t lattice_fwd(const LatGeom &g, bool fp32, const void *Fhat, void *H, hipStream_t s) {
    if (!geom_ok(g)) return hipErrorInvalidValue;
    return fp32 ? fwd_impl<float>(g, Fhat, H, s) : fwd_impl<double>(g, Fhat, H, s);
}

hipError_t lattice_yz(const LatGeom &g, bool fp32, void *H, const void *Khat, const int *worder, hipStream_t s) {
    if (!geom_ok(g) || worder == nullptr) return hipErrorInvalidValue;
    return fp32 ? yz_impl<float>(g, H, Khat, worder, s) : yz_impl<double>(g, H, Khat, worder, s);
}

hipError_t lattice_inv(const LatGeom &g, bool fp32, const void *H, void *Uhat, hipStream_t s) {
    if (!geom_ok(g)) return hipErrorInvalidValue;
    return fp32 ? inv_impl<float>(g, H, Uhat, s) : inv_impl<double>(g, H, Uhat, s);
}

bool lattice_fused_ok(const LatGeom &g) { return g.lx == 32 && g.ly == 32 && g.lz == 32; }

hipError_t lattice_fused(const LatGeom &g, bool fp32, const void *Fhat, const void *Khat, void *Uhat, void *Uhat2,
                         hipStream_t s) {
    if (!geom_ok(g) || !lattice_fused_ok(g) || Uhat2 == nullptr) return hipErrorInvalidValue;
    return fp32 ? fused_impl<float>(g, Fhat, Khat, Uhat, Uhat2, s) : fused_impl<double>(g, Fhat, Khat, Uhat, Uhat2, s);
}

hipError_t lattice_spectra(const LatSpecGeom &sg, bool fp32, const void *octant, void *Khat, void *scratch,
                           size_t scratch_bytes, hipStream_t s) {
    if (!lattice_len_ok(sg.lx) || !lattice_len_ok(sg.ly) || !lattice_zlen_ok(sg.lz) || sg.XD < sg.lx / 2 ||
        sg.YD < sg.ly / 2 || sg.ZD < sg.lz / 2)
        return hipErrorInvalidValue;
    return fp32 ? spec_impl<float>(sg, octant, Khat, scratch, scratch_bytes, s)
                : spec_impl<double>(sg, octant, Khat, scratch, scratch_bytes, s);
}

}  // namespace lgf
