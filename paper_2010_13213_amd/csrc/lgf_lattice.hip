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
// zero).  K_{-d}(omega) is the complex conjugate of K_d(omega) (the window
// of a real, even kernel mirrored), so Khat is real: it is stored as real
// numbers with the 1 / (Lx Ly Lz) of the inverse folded in.  The cost per
// frequency is O(L^3 log L) instead of the O(E^6) block pairs.
//
// Layouts (complex R, per component region):
//   Fhat, Uhat [omega][slot], slot = (z Ey + y) Ex + x over the box E;
//   H          [omega][z][ky][kx], z < Ez: the box after the x and y DFTs;
//   Khat       [omega][kz][ky][kx] (real R).
// Three kernels: xy forward (one workgroup per PL planes (component, omega,
// z), LDS-staged, register FFTs per line), z (a lane pair per column
// (omega, ky, kx): DFT, product with Khat, inverse DFT, in place), xy
// inverse.  Each streams its data once from HBM.  The spectra Khat are
// built once per (nb, precision, Lx, Ly, Lz) from the octant table of
// block spectra with the same line FFTs.
#include <algorithm>
#include <type_traits>

#include "lgf_device.hpp"
#include "lgf_kernels.hpp"

namespace lgf {

namespace {

constexpr int kLatThreads = 256;

template <typename R> __device__ __forceinline__ cplx<R> czero() { return cmake<R>((R)0, (R)0); }

// Forward DFT of the x and y axes of PL planes (component, omega, z).
template <typename R, int LX, int LY>
__global__ void __launch_bounds__(kLatThreads) lat_fwd_xy(LatGeom g, const cplx<R> *__restrict__ F,
                                                          cplx<R> *__restrict__ H) {
    constexpr int PL = kLatThreads / LX;      // planes per workgroup
    constexpr int YR = LY / 2;                // rows of a plane that can hold data (Ey <= LY/2)
    __shared__ cplx<R> X[PL * YR * LX];
    const int t = threadIdx.x;
    const int ex = g.ex, ey = g.ey, ez = g.ez;
    const int64_t n_items = (int64_t)g.nc * g.n_freq * ez;
    const int64_t item0 = (int64_t)blockIdx.x * PL;
    const int plane = ey * ex;
    // 1. coalesced load of the planes into rows of X (row stride LX)
    for (int e = t; e < PL * plane; e += kLatThreads) {
        const int p = e / plane, r = e % plane;
        const int64_t item = item0 + p;
        if (item >= n_items) break;
        const int64_t cw = item / ez;                  // c * n_freq + omega
        const int z = (int)(item % ez);
        const int64_t c = cw / g.n_freq, w = cw % g.n_freq;
        const cplx<R> v = F[c * g.fstride + w * g.n_slots + (int64_t)z * plane + r];
        X[(p * YR + r / ex) * LX + r % ex] = v;
    }
    __syncthreads();
    // 2. x lines (p, y), y < ey
    for (int e = t; e < PL * ey; e += kLatThreads) {
        const int p = e / ey, y = e % ey;
        cplx<R> a[LX];
        cplx<R> *row = X + (p * YR + y) * LX;
#pragma unroll
        for (int x = 0; x < LX; ++x) a[x] = x < ex ? row[x] : czero<R>();
        fft_reg<R, LX, false>(a);
#pragma unroll
        for (int x = 0; x < LX; ++x) row[x] = a[x];
    }
    __syncthreads();
    // 3. y lines (p, kx) -> H
    {
        const int p = t / LX, kx = t % LX;
        const int64_t item = item0 + p;
        if (item < n_items) {
            cplx<R> a[LY];
#pragma unroll
            for (int y = 0; y < LY; ++y) a[y] = y < ey ? X[(p * YR + y) * LX + kx] : czero<R>();
            fft_reg<R, LY, false>(a);
            const int64_t cw = item / ez;
            const int z = (int)(item % ez);
            const int64_t c = cw / g.n_freq, w = cw % g.n_freq;
            cplx<R> *out = H + c * g.hstride + (w * ez + z) * (int64_t)(LY * LX) + kx;
#pragma unroll
            for (int ky = 0; ky < LY; ++ky) out[ky * LX] = a[ky];
        }
    }
}

// z lines: DFT, product with the real spectrum, inverse DFT, in place.
// The input of a line is zero beyond ez <= LZ/2 and only its first LZ/2
// outputs are kept, so each line is split over a pair of lanes by the
// radix-2 identities (M = LZ/2, w = exp(-2 pi i / LZ)):
//   X[2m]   = DFT_M(x)[m],            X[2m+1] = DFT_M(w^n x)[m],
//   y[n]    = IDFT_M(X[2m] K[2m])[n] + w^-n IDFT_M(X[2m+1] K[2m+1])[n], n < M.
// The even lane does the first half, the odd lane the second; one exchange
// of half a line each way forms y.  Half-length lines halve the registers
// a lane holds.
template <typename R, int LZ>
__global__ void __launch_bounds__(kLatThreads) lat_z(LatGeom g, cplx<R> *__restrict__ H, const R *__restrict__ Khat) {
    constexpr int M = LZ / 2;
    const int64_t plane = (int64_t)g.lx * g.ly;
    const int64_t gid = (int64_t)blockIdx.x * kLatThreads + threadIdx.x;
    const int64_t col = gid >> 1;                          // omega * plane + (ky, kx)
    const int odd = (int)(gid & 1);
    // both lanes of a pair stay to the exchange; a dead pair only skips memory
    const bool live = col < (int64_t)g.n_freq * plane;
    const int64_t w = live ? col / plane : 0, q = live ? col % plane : 0;
    const int ez = g.ez;
    // the spectrum column is read once per component; later components find
    // it in L2
    const R *kc = Khat + (w * LZ + odd) * plane + q;       // kz = 2m + odd
    for (int c = 0; c < g.nc; ++c) {
        cplx<R> *hc = H + c * g.hstride + w * ez * plane + q;
        cplx<R> a[M];
#pragma unroll
        for (int n = 0; n < M; ++n) {
            const cplx<R> x = (live && n < ez) ? hc[n * plane] : czero<R>();
            // select on data, not on the twiddle: constants stay literal
            a[n] = (n > 0 && odd) ? cmul(x, twiddle<R, LZ, false>(n)) : x;
        }
        fft_reg<R, M, false>(a);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const R k = live ? kc[2 * m * plane] : (R)0;
            a[m] = cmake<R>(a[m].x * k, a[m].y * k);
        }
        fft_reg<R, M, true>(a);
        // even lane: y[j] = E[j] + w^-j O[j]; odd lane: y[M/2+j] likewise
#pragma unroll
        for (int j = 0; j < (M + 1) / 2; ++j) {
            const int jo = M / 2 + j;           // the odd lane's output index
            if (jo >= M) break;
            const cplx<R> send = odd ? a[j] : a[jo];
            cplx<R> recv;
            recv.x = __shfl_xor(send.x, 1);
            recv.y = __shfl_xor(send.y, 1);
            const int n = odd ? jo : j;
            const cplx<R> ye = cadd(a[j], cmul(recv, twiddle<R, LZ, true>(j)));    // even lane: n = j
            const cplx<R> yo = cadd(recv, cmul(a[jo], twiddle<R, LZ, true>(jo)));  // odd lane: n = jo
            const cplx<R> y = odd ? yo : ye;
            if (live && n < ez) hc[n * plane] = y;
        }
    }
}

// Inverse DFT of the y and x axes, cropped to the box, into Uhat.
template <typename R, int LX, int LY>
__global__ void __launch_bounds__(kLatThreads) lat_inv_xy(LatGeom g, const cplx<R> *__restrict__ H,
                                                          cplx<R> *__restrict__ U) {
    constexpr int PL = kLatThreads / LX;
    constexpr int YR = LY / 2;
    __shared__ cplx<R> X[PL * YR * LX];
    const int t = threadIdx.x;
    const int ex = g.ex, ey = g.ey, ez = g.ez;
    const int64_t n_items = (int64_t)g.nc * g.n_freq * ez;
    const int64_t item0 = (int64_t)blockIdx.x * PL;
    const int plane = ey * ex;
    // 1. y lines (p, kx) from H, keep y < ey
    {
        const int p = t / LX, kx = t % LX;
        const int64_t item = item0 + p;
        if (item < n_items) {
            const int64_t cw = item / ez;
            const int z = (int)(item % ez);
            const int64_t c = cw / g.n_freq, w = cw % g.n_freq;
            const cplx<R> *in = H + c * g.hstride + (w * ez + z) * (int64_t)(LY * LX) + kx;
            cplx<R> a[LY];
#pragma unroll
            for (int ky = 0; ky < LY; ++ky) a[ky] = in[ky * LX];
            fft_reg<R, LY, true>(a);
#pragma unroll
            for (int y = 0; y < LY; ++y)
                if (y < ey) X[(p * YR + y) * LX + kx] = a[y];
        }
    }
    __syncthreads();
    // 2. x lines (p, y), keep x < ex (in place, row start)
    for (int e = t; e < PL * ey; e += kLatThreads) {
        const int p = e / ey, y = e % ey;
        cplx<R> *row = X + (p * YR + y) * LX;
        cplx<R> a[LX];
#pragma unroll
        for (int x = 0; x < LX; ++x) a[x] = row[x];
        fft_reg<R, LX, true>(a);
#pragma unroll
        for (int x = 0; x < LX; ++x)
            if (x < ex) row[x] = a[x];
    }
    __syncthreads();
    // 3. coalesced store of the cropped planes
    for (int e = t; e < PL * plane; e += kLatThreads) {
        const int p = e / plane, r = e % plane;
        const int64_t item = item0 + p;
        if (item >= n_items) break;
        const int64_t cw = item / ez;
        const int z = (int)(item % ez);
        const int64_t c = cw / g.n_freq, w = cw % g.n_freq;
        U[c * g.fstride + w * g.n_slots + (int64_t)z * plane + r] = X[(p * YR + r / ex) * LX + r % ex];
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

// One (omega, pz) plane per workgroup: gather K_d, DFT along x then y, into S.
template <typename R, int LX, int LY>
__global__ void __launch_bounds__(kLatThreads) latspec_xy(LatSpecGeom s, const cplx<R> *__restrict__ T,
                                                          cplx<R> *__restrict__ S, int w0, int nw) {
    __shared__ cplx<R> X[LY * LX];
    const int t = threadIdx.x;
    const int wl = blockIdx.x / s.lz, pz = blockIdx.x % s.lz;
    if (wl >= nw) return;
    const int w = w0 + wl;
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

// z DFT of each column of S; the real part, scaled, into Khat.
template <typename R, int LZ>
__global__ void __launch_bounds__(kLatThreads) latspec_z(LatSpecGeom s, const cplx<R> *__restrict__ S,
                                                         R *__restrict__ Khat, int w0, int nw, R scale) {
    const int64_t plane = (int64_t)s.lx * s.ly;
    const int64_t col = (int64_t)blockIdx.x * kLatThreads + threadIdx.x;
    if (col >= (int64_t)nw * plane) return;
    const int64_t wl = col / plane, q = col % plane;
    cplx<R> a[LZ];
#pragma unroll
    for (int pz = 0; pz < LZ; ++pz) a[pz] = S[(wl * LZ + pz) * plane + q];
    fft_reg<R, LZ, false>(a);
    R *out = Khat + ((int64_t)(w0 + wl) * LZ) * plane + q;
#pragma unroll
    for (int kz = 0; kz < LZ; ++kz) out[kz * plane] = a[kz].x * scale;
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

template <typename R> hipError_t fwd_impl(const LatGeom &g, const void *F, void *H, hipStream_t s) {
    const int64_t items = (int64_t)g.nc * g.n_freq * g.ez;
    return with_len(g.lx, [&](auto lx) {
        return with_len(g.ly, [&](auto ly) {
            constexpr int LX = decltype(lx)::value, LY = decltype(ly)::value;
            constexpr int PL = kLatThreads / LX;
            hipLaunchKernelGGL((lat_fwd_xy<R, LX, LY>), dim3((unsigned)((items + PL - 1) / PL)), dim3(kLatThreads),
                               0, s, g, (const cplx<R> *)F, (cplx<R> *)H);
            return hipGetLastError();
        });
    });
}

template <typename R> hipError_t z_impl(const LatGeom &g, void *H, const void *Khat, hipStream_t s) {
    const int64_t lanes = 2 * (int64_t)g.n_freq * g.lx * g.ly;   // two lanes per z line
    return with_len(g.lz, [&](auto lz) {
        constexpr int LZ = decltype(lz)::value;
        hipLaunchKernelGGL((lat_z<R, LZ>), dim3((unsigned)((lanes + kLatThreads - 1) / kLatThreads)),
                           dim3(kLatThreads), 0, s, g, (cplx<R> *)H, (const R *)Khat);
        return hipGetLastError();
    });
}

template <typename R> hipError_t inv_impl(const LatGeom &g, const void *H, void *U, hipStream_t s) {
    const int64_t items = (int64_t)g.nc * g.n_freq * g.ez;
    return with_len(g.lx, [&](auto lx) {
        return with_len(g.ly, [&](auto ly) {
            constexpr int LX = decltype(lx)::value, LY = decltype(ly)::value;
            constexpr int PL = kLatThreads / LX;
            hipLaunchKernelGGL((lat_inv_xy<R, LX, LY>), dim3((unsigned)((items + PL - 1) / PL)), dim3(kLatThreads),
                               0, s, g, (const cplx<R> *)H, (cplx<R> *)U);
            return hipGetLastError();
        });
    });
}

template <typename R> hipError_t spec_impl(const LatSpecGeom &sg, const void *T, void *Khat, void *scratch,
                                           size_t scratch_bytes, hipStream_t s) {
    const int64_t per_w = (int64_t)sg.lx * sg.ly * sg.lz;
    const int64_t chunk = std::max<int64_t>(1, (int64_t)(scratch_bytes / (sizeof(cplx<R>) * per_w)));
    const R scale = (R)(1.0 / (double)per_w);
    for (int64_t w0 = 0; w0 < sg.n_freq; w0 += chunk) {
        const int nw = (int)std::min<int64_t>(chunk, sg.n_freq - w0);
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
        e = with_len(sg.lz, [&](auto lz) {
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

bool lattice_len_ok(int L) { return L == 4 || L == 8 || L == 16 || L == 32; }

int lattice_len(int extent) {
    int L = 4;
    while (L < 2 * extent - 1) L *= 2;
    return L;
}

static bool geom_ok(const LatGeom &g) {
    return lattice_len_ok(g.lx) && lattice_len_ok(g.ly) && lattice_len_ok(g.lz) && g.nc >= 1 && g.ex >= 1 &&
           g.ey >= 1 && g.ez >= 1 && 2 * g.ex <= g.lx && 2 * g.ey <= g.ly && 2 * g.ez <= g.lz;
}

hipError_t lattice_fwd(const LatGeom &g, bool fp32, const void *Fhat, void *H, hipStream_t s) {
    if (!geom_ok(g)) return hipErrorInvalidValue;
    return fp32 ? fwd_impl<float>(g, Fhat, H, s) : fwd_impl<double>(g, Fhat, H, s);
}

hipError_t lattice_z(const LatGeom &g, bool fp32, void *H, const void *Khat, hipStream_t s) {
    if (!geom_ok(g)) return hipErrorInvalidValue;
    return fp32 ? z_impl<float>(g, H, Khat, s) : z_impl<double>(g, H, Khat, s);
}

hipError_t lattice_inv(const LatGeom &g, bool fp32, const void *H, void *Uhat, hipStream_t s) {
    if (!geom_ok(g)) return hipErrorInvalidValue;
    return fp32 ? inv_impl<float>(g, H, Uhat, s) : inv_impl<double>(g, H, Uhat, s);
}

hipError_t lattice_conv(const LatGeom &g, bool fp32, const void *Fhat, void *H, const void *Khat, void *Uhat,
                        hipStream_t s) {
    hipError_t e = lattice_fwd(g, fp32, Fhat, H, s);
    if (e == hipSuccess) e = lattice_z(g, fp32, H, Khat, s);
    if (e == hipSuccess) e = lattice_inv(g, fp32, H, Uhat, s);
    return e;
}

hipError_t lattice_spectra(const LatSpecGeom &sg, bool fp32, const void *octant, void *Khat, void *scratch,
                           size_t scratch_bytes, hipStream_t s) {
    if (!lattice_len_ok(sg.lx) || !lattice_len_ok(sg.ly) || !lattice_len_ok(sg.lz) || sg.XD < sg.lx / 2 ||
        sg.YD < sg.ly / 2 || sg.ZD < sg.lz / 2)
        return hipErrorInvalidValue;
    return fp32 ? spec_impl<float>(sg, octant, Khat, scratch, scratch_bytes, s)
                : spec_impl<double>(sg, octant, Khat, scratch, scratch_bytes, s);
}

}  // namespace lgf
