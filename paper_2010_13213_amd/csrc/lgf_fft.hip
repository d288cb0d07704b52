// Batched zero-padded (2nb)^3 block FFTs staged in LDS (gfx950).
//
// The LGF convolution of one source block with one target block (paper
// Sec. 2.2, eq. lgf_convolution, evaluated blockwise) is a linear
// convolution of an nb^3 block with a (2nb-1)^3 kernel window; zero-padding
// the block to (2nb)^3 makes the circular convolution of the FFT exact.
//
// Forward (three workgroups per source block, one per third of the kx range):
//   x: nb^2 rows of nb reals, zero-padded to N = 2nb -> N/2+1 complex, the
//      chunk's kx kept                                                 (LDS A)
//   y: nb x (chunk) columns, zero-padded to N                          (LDS B)
//   z: N x (chunk) columns, zero-padded to N -> written to HBM
// (a third of the LDS each: two workgroups fit a CU in float64)
// The zero half of the input is never loaded.  Inverse runs the same stages
// backwards, chunk by chunk in one workgroup per block, and keeps only the
// [0, nb)^3 corner of the result.
//
// Every forward line has nb nonzero inputs out of N = 2nb, so it is split
// in halves by the radix-2 identities (M = nb, w = exp(-2 pi i / N)):
//   X[2m] = DFT_M(x)[m],  X[2m+1] = DFT_M(w^n x)[m].
// The forward workgroup has 2 nb^2 threads: the first nb^2 (whole waves)
// take the even half of every line, the rest the odd half, so the half is
// uniform over a wave (the odd twiddles are a branch).  Half-length lines
// halve the registers of a lane and double the waves of a block.  The
// inverse keeps one thread per whole line.
//
// Spectra are stored block-major (a block's spectrum is one contiguous run;
// the lattice MAC) or frequency-major (one 16-byte entry, 8 in float32, per
// frequency row, so neighbouring slots share HBM lines; the block-pair MAC).
// Workgroups are renumbered so that consecutive ones (the chunks of a block,
// neighbouring slots) run at the same time on one XCD and meet in its L2.
#include "lgf_device.hpp"
#include "lgf_kernels.hpp"

namespace lgf {

namespace {

template <int NB, typename R> struct FftShape {
    static constexpr int N = 2 * NB;
    static constexpr int M = NB;                // half-line length
    static constexpr int H = NB + 1;            // r2c length along x
    static constexpr int HL = NB * NB;          // lanes per half
    static constexpr int NT = 2 * HL;           // threads per block
    // kx in kSpecChunks chunks of KC (= spec_chunk(N)): one forward
    // workgroup each; the inverse walks them in turn
    static constexpr int KC = (H + 2) / 3;
    static_assert(kSpecChunks == 3, "KC is a third of the kx range");
    static constexpr int FA_ELEMS = NB * NB * KC;   // [z][y][kxl]
    static constexpr int FB_ELEMS = NB * N * KC;    // [z][ky][kxl]
};

template <int NB> constexpr int fft_threads = 2 * NB * NB;   // FftShape<NB, R>::NT, usable in a macro


// x[n] * w^n (the odd half's input), n < M, w = exp(-2 pi i / N)
template <typename R, int N, int M> __device__ __forceinline__ void odd_twiddle(cplx<R> (&a)[M]) {
#pragma unroll
    for (int n = 1; n < M; ++n) a[n] = cmul(a[n], twiddle<R, N, false>(n));
}

// Spectrum position p of slot sl at Fhat[p * ws + sl * ss]: frequency-major
// (p = omega, ws = n_slots, ss = 1) or block-major (p = spec_pos(omega),
// ws = 1, ss = n_freq).
template <int NB> constexpr int64_t fft_freqs = 4 * NB * NB * (NB + 1);   // (2nb)^2 (nb + 1)

// Forward transform of block b, kx chunk `chunk` (kx in [chunk KC, ...)):
// the x pass is computed whole and only the chunk's kx are kept, so three
// workgroups share a block and each needs a third of the LDS.
// BM: block-major (chunk-major within a block, spec_pos) or frequency-major
// spectra.  A, B: the workgroup's LDS (FA_ELEMS, FB_ELEMS).
template <int NB, typename R, bool BM>
__device__ __forceinline__ void fwd_body(const double *__restrict__ src, const int64_t *__restrict__ blk_off,
                                         const int *__restrict__ slot, cplx<R> *__restrict__ Fhat, int64_t n_slots,
                                         double scale, int b, int chunk, cplx<R> *A, cplx<R> *B) {
    using S = FftShape<NB, R>;
    constexpr int N = S::N, M = S::M, H = S::H, KC = S::KC, HL = S::HL;
    static_assert(KC * kSpecChunks >= H && KC * (kSpecChunks - 1) < H, "kx chunks");
    const double *in = src + blk_off[b];
    const int64_t ws = BM ? 1 : n_slots;
    cplx<R> *Fb = Fhat + slot[b] * (BM ? fft_freqs<NB> : 1);
    const int t = threadIdx.x;
    const int half = t / HL, lane = t % HL;
    const int k0 = chunk * KC, nk = min(KC, H - k0);

    // x pass: row (y, z) = lane; this half's outputs kx = 2m + half, kept in the chunk
    {
        const int y = lane % NB, z = lane / NB;
        const double *row = in + ((size_t)z * NB + y) * NB;
        cplx<R> a[M];
#pragma unroll
        for (int n = 0; n < M; ++n) a[n] = cmake<R>((R)(row[n] * scale), (R)0);
        if (half) odd_twiddle<R, N, M>(a);
        fft_reg<R, M, false>(a);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const int kxl = 2 * m + half - k0;
            if (kxl >= 0 && kxl < nk) A[(z * NB + y) * KC + kxl] = a[m];
        }
    }
    __syncthreads();
    // y pass: column (z, kxl)
    for (int line = lane; line < NB * nk; line += HL) {
        const int kxl = line % nk, z = line / nk;
        cplx<R> a[M];
#pragma unroll
        for (int y = 0; y < M; ++y) a[y] = A[(z * NB + y) * KC + kxl];
        if (half) odd_twiddle<R, N, M>(a);
        fft_reg<R, M, false>(a);
#pragma unroll
        for (int m = 0; m < M; ++m) B[(z * N + 2 * m + half) * KC + kxl] = a[m];
    }
    __syncthreads();
    // z pass: column (ky, kxl) -> HBM
    for (int line = lane; line < N * nk; line += HL) {
        const int kxl = line % nk, ky = line / nk;
        cplx<R> a[M];
#pragma unroll
        for (int z = 0; z < M; ++z) a[z] = B[(z * N + ky) * KC + kxl];
        if (half) odd_twiddle<R, N, M>(a);
        fft_reg<R, M, false>(a);
        const int kx = k0 + kxl;
        // position of kz = half, and the step between kz and kz + 2:
        // block-major the chunk's run [kz][ky][kxl] (spec_pos), frequency-major omega
        cplx<R> *o = Fb + (BM ? (int64_t)N * N * k0 + (half * N + ky) * nk + kxl : ((int64_t)half * N + ky) * H + kx) * ws;
        const int64_t step = (BM ? 2 * N * nk : 2 * N * H) * ws;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            // block-major spectra go to the lattice x pass, which reads them from HBM;
            // the frequency-major ones are re-read by the pair MAC
            if constexpr (BM) cstore_nt(&o[m * step], a[m]);
            else o[m * step] = a[m];
        }
    }
}

// workgroup -> (block, chunk); the chunks of a block are consecutive and run
// on one XCD (they read the same input block).  One instantiation per
// spectrum layout, so each gets its own register allocation.
template <int NB, typename R, bool BM>
__global__ void __launch_bounds__(fft_threads<NB>) __attribute__((amdgpu_waves_per_eu(4))) fwd_kernel(const double *__restrict__ src, const int64_t *__restrict__ blk_off,
                                                  const int *__restrict__ slot, cplx<R> *__restrict__ Fhat,
                                                  int64_t n_slots, double scale) {
    using S = FftShape<NB, R>;
    __shared__ cplx<R> A[S::FA_ELEMS];
    __shared__ cplx<R> B[S::FB_ELEMS];
    const int wg = (int)xcd_order(blockIdx.x, gridDim.x);
    fwd_body<NB, R, BM>(src, blk_off, slot, Fhat, n_slots, scale, wg / kSpecChunks, wg % kSpecChunks, A, B);
}

__device__ __forceinline__ int find_job(const FftJob *__restrict__ jobs, int n_jobs, int b) {
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (jobs[mid].blk_begin <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <int NB, typename R>
__global__ void __launch_bounds__(fft_threads<NB>) __attribute__((amdgpu_waves_per_eu(4))) fwd_batch_kernel(const FftJob *__restrict__ jobs, int n_jobs) {
    const int wg = (int)xcd_order(blockIdx.x, gridDim.x);
    using S = FftShape<NB, R>;
    __shared__ cplx<R> A[S::FA_ELEMS];
    __shared__ cplx<R> B[S::FB_ELEMS];
    const int b = wg / kSpecChunks;
    const FftJob &j = jobs[find_job(jobs, n_jobs, b)];
    if (j.block_major)
        fwd_body<NB, R, true>(j.src, j.blk_off, j.slot, (cplx<R> *)j.spec, j.n_slots, j.scale, b - j.blk_begin,
                              wg % kSpecChunks, A, B);
    else
        fwd_body<NB, R, false>(j.src, j.blk_off, j.slot, (cplx<R> *)j.spec, j.n_slots, j.scale, b - j.blk_begin,
                               wg % kSpecChunks, A, B);
}

// The inverse keeps one thread per whole line (256 threads) and walks the
// kx chunks of the forward: per chunk an inverse z pass from HBM (one
// contiguous run of a block-major spectrum), an inverse y pass, and the
// chunk's share of the complex-to-real x sums, accumulated in registers by
// the thread that owns the row.  LDS holds one chunk (73.7 KB in float64),
// so two workgroups fit a CU.
constexpr int kInvThreads = 256;

// Re(v exp(+2 pi i j / N)), j a compile-time value after unrolling
template <typename R, int N> __device__ __forceinline__ R re_rot(cplx<R> v, int j) {
    const int q = (j % N) * (64 / N);   // in 64ths of a turn
    const R c = q < 32 ? (R)kTw128[2 * q][0] : -(R)kTw128[2 * (q - 32)][0];
    const R s = q < 32 ? -(R)kTw128[2 * q][1] : (R)kTw128[2 * (q - 32)][1];   // sin(2 pi q / 64)
    return v.x * c - v.y * s;
}

// C: [z][ky][kxl] after the z pass (FB_ELEMS), D: [z][y][kxl] after the y
// pass (FA_ELEMS), the workgroup's LDS.
template <int NB, typename R, bool BM, bool SUM2 = false>
__device__ __forceinline__ void inv_body(const cplx<R> *__restrict__ Uhat, const cplx<R> *__restrict__ Uhat2,
                                         int64_t n_slots,
                                         const int *__restrict__ slot, const int64_t *__restrict__ blk_off,
                                         double *__restrict__ dst, double scale, int accumulate, int b, cplx<R> *C,
                                         cplx<R> *D) {
    using S = FftShape<NB, R>;
    constexpr int N = S::N, H = S::H, KC = S::KC;
    static_assert(NB * NB <= kInvThreads, "one x row per thread");
    const int64_t ws = BM ? 1 : n_slots;
    const cplx<R> *Ub = Uhat + slot[b] * (BM ? fft_freqs<NB> : 1);
    const cplx<R> *Ub2 = SUM2 ? Uhat2 + slot[b] * fft_freqs<NB> : nullptr;
    const int t = threadIdx.x;
    R acc[NB];
#pragma unroll
    for (int x = 0; x < NB; ++x) acc[x] = (R)0;

#pragma unroll
    for (int c = 0; c < kSpecChunks; ++c) {
        const int k0 = c * KC;
        const int nk = KC < H - k0 ? KC : H - k0;
        // inverse z pass: column (ky, kxl) from HBM, keep z < nb
        for (int line = t; line < N * nk; line += kInvThreads) {
            const int kxl = line % nk, ky = line / nk;
            cplx<R> a[N];
#pragma unroll
            for (int kz = 0; kz < N; ++kz) {
                const int64_t pos =
                    BM ? (int64_t)N * N * k0 + (kz * N + ky) * nk + kxl : ((int64_t)kz * N + ky) * H + k0 + kxl;
                if constexpr (BM) a[kz] = cload_nt(&Ub[pos * ws]);
                else a[kz] = Ub[pos * ws];
                if constexpr (SUM2) a[kz] = cadd(a[kz], cload_nt(&Ub2[pos]));
            }
            fft_reg<R, N, true>(a);
#pragma unroll
            for (int z = 0; z < NB; ++z) C[(z * N + ky) * KC + kxl] = a[z];
        }
        __syncthreads();
        // inverse y pass: column (z, kxl), keep y < nb
        for (int line = t; line < NB * nk; line += kInvThreads) {
            const int kxl = line % nk, z = line / nk;
            cplx<R> a[N];
#pragma unroll
            for (int ky = 0; ky < N; ++ky) a[ky] = C[(z * N + ky) * KC + kxl];
            fft_reg<R, N, true>(a);
#pragma unroll
            for (int y = 0; y < NB; ++y) D[(z * NB + y) * KC + kxl] = a[y];
        }
        __syncthreads();
        // x sums of row (y, z) = t: u[x] += c_kx Re(X[kx] exp(2 pi i kx x / N)),
        // c_kx = 1 at kx = 0 and N/2 (real by symmetry), 2 otherwise
        if (t < NB * NB) {
            const cplx<R> *row = D + t * KC;
#pragma unroll
            for (int kxl = 0; kxl < KC; ++kxl) {
                const int kx = c * KC + kxl;
                if (kx < H) {
                    const cplx<R> v = row[kxl];
                    const R w = (kx == 0 || kx == N / 2) ? (R)1 : (R)2;
#pragma unroll
                    for (int x = 0; x < NB; ++x) acc[x] += w * re_rot<R, N>(v, kx * x);
                }
            }
        }
        __syncthreads();   // C and D are rewritten by the next chunk
    }
    if (t < NB * NB) {
        double *o = dst + blk_off[b] + (size_t)t * NB;   // row (y, z) = t: z = t / NB, y = t % NB
#pragma unroll
        for (int x = 0; x < NB; ++x) {
            const double v = (double)acc[x] * scale;
            o[x] = accumulate ? o[x] + v : v;
        }
    }
}

// SUM2: the spectrum is Uhat + Uhat2 (block-major)
template <int NB, typename R, bool SUM2>
__global__ void __launch_bounds__(kInvThreads) inv_kernel(const cplx<R> *__restrict__ Uhat,
                                                  const cplx<R> *__restrict__ Uhat2, int64_t n_slots,
                                                  int block_major, const int *__restrict__ slot,
                                                  const int64_t *__restrict__ blk_off, double *__restrict__ dst,
                                                  double scale, int accumulate) {
    using S = FftShape<NB, R>;
    __shared__ cplx<R> C[S::FB_ELEMS];
    __shared__ cplx<R> D[S::FA_ELEMS];
    const int b = (int)xcd_order(blockIdx.x, gridDim.x);
    if (SUM2) inv_body<NB, R, true, true>(Uhat, Uhat2, n_slots, slot, blk_off, dst, scale, accumulate, b, C, D);
    else if (block_major) inv_body<NB, R, true>(Uhat, nullptr, n_slots, slot, blk_off, dst, scale, accumulate, b, C, D);
    else inv_body<NB, R, false>(Uhat, nullptr, n_slots, slot, blk_off, dst, scale, accumulate, b, C, D);
}

template <int NB, typename R>
__global__ void __launch_bounds__(kInvThreads) inv_batch_kernel(const FftJob *__restrict__ jobs, int n_jobs) {
    using S = FftShape<NB, R>;
    __shared__ cplx<R> C[S::FB_ELEMS];
    __shared__ cplx<R> D[S::FA_ELEMS];
    const int b = (int)xcd_order(blockIdx.x, gridDim.x);
    const FftJob &j = jobs[find_job(jobs, n_jobs, b)];
    if (j.spec2)
        inv_body<NB, R, true, true>((const cplx<R> *)j.spec, (const cplx<R> *)j.spec2, j.n_slots, j.slot, j.blk_off,
                                    j.dst, j.scale, j.accumulate, b - j.blk_begin, C, D);
    else if (j.block_major)
        inv_body<NB, R, true>((const cplx<R> *)j.spec, nullptr, j.n_slots, j.slot, j.blk_off, j.dst, j.scale,
                              j.accumulate, b - j.blk_begin, C, D);
    else
        inv_body<NB, R, false>((const cplx<R> *)j.spec, nullptr, j.n_slots, j.slot, j.blk_off, j.dst, j.scale,
                               j.accumulate, b - j.blk_begin, C, D);
}

template <int NB, typename R>
hipError_t batch_launch(bool inverse, const FftJob *jobs, int n_jobs, int total_blocks, hipStream_t s) {
    if (n_jobs <= 0 || total_blocks <= 0) return hipSuccess;
    if (inverse)
        hipLaunchKernelGGL((inv_batch_kernel<NB, R>), dim3(total_blocks), dim3(kInvThreads), 0, s, jobs, n_jobs);
    else
        hipLaunchKernelGGL((fwd_batch_kernel<NB, R>), dim3(total_blocks * kSpecChunks), dim3(FftShape<NB, R>::NT), 0, s,
                           jobs, n_jobs);
    return hipGetLastError();
}

template <int NB, typename R>
hipError_t fwd_launch(const double *src, const int64_t *blk_off, const int *slot, int n_blocks, void *Fhat,
                      int64_t n_slots, bool block_major, double scale, hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    if (block_major)
        hipLaunchKernelGGL((fwd_kernel<NB, R, true>), dim3(n_blocks * kSpecChunks), dim3(FftShape<NB, R>::NT), 0, s,
                           src, blk_off, slot, (cplx<R> *)Fhat, n_slots, scale);
    else
        hipLaunchKernelGGL((fwd_kernel<NB, R, false>), dim3(n_blocks * kSpecChunks), dim3(FftShape<NB, R>::NT), 0, s,
                           src, blk_off, slot, (cplx<R> *)Fhat, n_slots, scale);
    return hipGetLastError();
}

template <int NB, typename R>
hipError_t inv_launch(const void *Uhat, const void *Uhat2, int64_t n_slots, bool block_major, const int *slot,
                      const int64_t *blk_off, int n_blocks, double *dst, double scale, int accumulate, hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    if (Uhat2 != nullptr && !block_major) return hipErrorInvalidValue;
    if (Uhat2 != nullptr)
        hipLaunchKernelGGL((inv_kernel<NB, R, true>), dim3(n_blocks), dim3(kInvThreads), 0, s, (const cplx<R> *)Uhat,
                           (const cplx<R> *)Uhat2, n_slots, (int)block_major, slot, blk_off, dst, scale, accumulate);
    else
        hipLaunchKernelGGL((inv_kernel<NB, R, false>), dim3(n_blocks), dim3(kInvThreads), 0, s, (const cplx<R> *)Uhat,
                           nullptr, n_slots, (int)block_major, slot, blk_off, dst, scale, accumulate);
    return hipGetLastError();
}

}  // namespace

hipError_t block_fft_forward(int nb, bool fp32, const double *src, const int64_t *blk_off, const int *slot,
                             int n_blocks, void *Fhat, int64_t n_slots, bool block_major, double scale, hipStream_t s) {
    if (nb == 16)
        return fp32 ? fwd_launch<16, float>(src, blk_off, slot, n_blocks, Fhat, n_slots, block_major, scale, s)
                    : fwd_launch<16, double>(src, blk_off, slot, n_blocks, Fhat, n_slots, block_major, scale, s);
    if (nb == 8)
        return fp32 ? fwd_launch<8, float>(src, blk_off, slot, n_blocks, Fhat, n_slots, block_major, scale, s)
                    : fwd_launch<8, double>(src, blk_off, slot, n_blocks, Fhat, n_slots, block_major, scale, s);
    return hipErrorInvalidValue;
}

hipError_t block_fft_forward_batch(int nb, bool fp32, const FftJob *jobs, int n_jobs, int total_blocks,
                                   hipStream_t s) {
    if (nb == 16)
        return fp32 ? batch_launch<16, float>(false, jobs, n_jobs, total_blocks, s)
                    : batch_launch<16, double>(false, jobs, n_jobs, total_blocks, s);
    if (nb == 8)
        return fp32 ? batch_launch<8, float>(false, jobs, n_jobs, total_blocks, s)
                    : batch_launch<8, double>(false, jobs, n_jobs, total_blocks, s);
    return hipErrorInvalidValue;
}

hipError_t block_fft_inverse_batch(int nb, bool fp32, const FftJob *jobs, int n_jobs, int total_blocks,
                                   hipStream_t s) {
    if (nb == 16)
        return fp32 ? batch_launch<16, float>(true, jobs, n_jobs, total_blocks, s)
                    : batch_launch<16, double>(true, jobs, n_jobs, total_blocks, s);
    if (nb == 8)
        return fp32 ? batch_launch<8, float>(true, jobs, n_jobs, total_blocks, s)
                    : batch_launch<8, double>(true, jobs, n_jobs, total_blocks, s);
    return hipErrorInvalidValue;
}

hipError_t block_fft_inverse(int nb, bool fp32, const void *Uhat, const void *Uhat2, int64_t n_slots,
                             bool block_major, const int *slot, const int64_t *blk_off, int n_blocks, double *dst,
                             double scale, int accumulate, hipStream_t s) {
    if (nb == 16)
        return fp32 ? inv_launch<16, float>(Uhat, Uhat2, n_slots, block_major, slot, blk_off, n_blocks, dst, scale,
                                            accumulate, s)
                    : inv_launch<16, double>(Uhat, Uhat2, n_slots, block_major, slot, blk_off, n_blocks, dst, scale,
                                             accumulate, s);
    if (nb == 8)
        return fp32 ? inv_launch<8, float>(Uhat, Uhat2, n_slots, block_major, slot, blk_off, n_blocks, dst, scale,
                                           accumulate, s)
                    : inv_launch<8, double>(Uhat, Uhat2, n_slots, block_major, slot, blk_off, n_blocks, dst, scale,
                                            accumulate, s);
    return hipErrorInvalidValue;
}

}  // namespace lgf
