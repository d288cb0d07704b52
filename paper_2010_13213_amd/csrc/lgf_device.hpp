// Device-side building blocks shared by the LGF kernels (gfx950).
//
// * cplx<R>: a 2-vector complex number in float or double.
// * fft_reg<N, INV>: an in-register radix-2 FFT of length N (2 to 64) on a
//   per-thread array; all indices are compile-time so the array lives in
//   VGPRs.  Forward uses exp(-2 pi i k / N), inverse exp(+2 pi i k / N), no
//   scaling.  Twiddles are compile-time constants (cos, -sin)(2 pi k / 128),
//   folded into the unrolled butterflies.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lgf {

template <typename R> struct alignas(2 * sizeof(R)) cplx {
    R x, y;
};

// Streaming store of one complex value (non-temporal: the line is not kept
// in the caches), for outputs far larger than L2 that the next kernel reads
// back from HBM anyway.
template <typename R> __device__ __forceinline__ void cstore_nt(cplx<R> *p, cplx<R> v) {
    typedef R v2 __attribute__((ext_vector_type(2)));
    v2 t;
    t.x = v.x;
    t.y = v.y;
    __builtin_nontemporal_store(t, reinterpret_cast<v2 *>(p));
}

// Streaming load of one complex value, for data that is read exactly once.
template <typename R> __device__ __forceinline__ cplx<R> cload_nt(const cplx<R> *p) {
    typedef R v2 __attribute__((ext_vector_type(2)));
    const v2 t = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(p));
    cplx<R> c;
    c.x = t.x;
    c.y = t.y;
    return c;
}

template <typename R> __device__ __forceinline__ cplx<R> cmake(R a, R b) {
    cplx<R> c;
    c.x = a;
    c.y = b;
    return c;
}
template <typename R> __device__ __forceinline__ cplx<R> cadd(cplx<R> a, cplx<R> b) {
    return cmake(a.x + b.x, a.y + b.y);
}
template <typename R> __device__ __forceinline__ cplx<R> csub(cplx<R> a, cplx<R> b) {
    return cmake(a.x - b.x, a.y - b.y);
}
template <typename R> __device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
    return cmake(fma(a.x, b.x, -a.y * b.y), fma(a.x, b.y, a.y * b.x));
}
// acc + a * b with four fused multiply-adds
template <typename R> __device__ __forceinline__ cplx<R> cmac(cplx<R> acc, cplx<R> a, cplx<R> b) {
    acc.x = fma(a.x, b.x, acc.x);
    acc.x = fma(-a.y, b.y, acc.x);
    acc.y = fma(a.x, b.y, acc.y);
    acc.y = fma(a.y, b.x, acc.y);
    return acc;
}

// exp(-2 pi i k / 128), k = 0..63, as (cos, -sin) pairs, each correctly
// rounded to float64 (every shorter length takes every (128 / N)-th entry).
constexpr double kTw128[64][2] = {
    {1.0, 0.0},
    {0.9987954562051724, -0.049067674327418015},
    {0.9951847266721969, -0.0980171403295606},
    {0.989176509964781, -0.14673047445536175},
    {0.9807852804032304, -0.19509032201612828},
    {0.970031253194544, -0.2429801799032639},
    {0.9569403357322088, -0.2902846772544624},
    {0.9415440651830208, -0.33688985339222005},
    {0.9238795325112867, -0.3826834323650898},
    {0.9039892931234433, -0.4275550934302821},
    {0.881921264348355, -0.47139673682599764},
    {0.8577286100002721, -0.5141027441932218},
    {0.8314696123025452, -0.5555702330196022},
    {0.8032075314806449, -0.5956993044924334},
    {0.773010453362737, -0.6343932841636455},
    {0.7409511253549591, -0.6715589548470184},
    {0.7071067811865476, -0.7071067811865476},
    {0.6715589548470184, -0.7409511253549591},
    {0.6343932841636455, -0.773010453362737},
    {0.5956993044924334, -0.8032075314806449},
    {0.5555702330196022, -0.8314696123025452},
    {0.5141027441932218, -0.8577286100002721},
    {0.47139673682599764, -0.881921264348355},
    {0.4275550934302821, -0.9039892931234433},
    {0.3826834323650898, -0.9238795325112867},
    {0.33688985339222005, -0.9415440651830208},
    {0.2902846772544624, -0.9569403357322088},
    {0.2429801799032639, -0.970031253194544},
    {0.19509032201612828, -0.9807852804032304},
    {0.14673047445536175, -0.989176509964781},
    {0.0980171403295606, -0.9951847266721969},
    {0.049067674327418015, -0.9987954562051724},
    {0.0, -1.0},
    {-0.049067674327418015, -0.9987954562051724},
    {-0.0980171403295606, -0.9951847266721969},
    {-0.14673047445536175, -0.989176509964781},
    {-0.19509032201612828, -0.9807852804032304},
    {-0.2429801799032639, -0.970031253194544},
    {-0.2902846772544624, -0.9569403357322088},
    {-0.33688985339222005, -0.9415440651830208},
    {-0.3826834323650898, -0.9238795325112867},
    {-0.4275550934302821, -0.9039892931234433},
    {-0.47139673682599764, -0.881921264348355},
    {-0.5141027441932218, -0.8577286100002721},
    {-0.5555702330196022, -0.8314696123025452},
    {-0.5956993044924334, -0.8032075314806449},
    {-0.6343932841636455, -0.773010453362737},
    {-0.6715589548470184, -0.7409511253549591},
    {-0.7071067811865476, -0.7071067811865476},
    {-0.7409511253549591, -0.6715589548470184},
    {-0.773010453362737, -0.6343932841636455},
    {-0.8032075314806449, -0.5956993044924334},
    {-0.8314696123025452, -0.5555702330196022},
    {-0.8577286100002721, -0.5141027441932218},
    {-0.881921264348355, -0.47139673682599764},
    {-0.9039892931234433, -0.4275550934302821},
    {-0.9238795325112867, -0.3826834323650898},
    {-0.9415440651830208, -0.33688985339222005},
    {-0.9569403357322088, -0.2902846772544624},
    {-0.970031253194544, -0.2429801799032639},
    {-0.9807852804032304, -0.19509032201612828},
    {-0.989176509964781, -0.14673047445536175},
    {-0.9951847266721969, -0.0980171403295606},
    {-0.9987954562051724, -0.049067674327418015},
};

template <typename R, int N, bool INV> __device__ __forceinline__ cplx<R> twiddle(int k) {
    // exp(-+2 pi i k / N) = table entry k * (128 / N), k < N / 2
    static_assert(N >= 2 && N <= 128 && 128 % N == 0, "twiddle length");
    const int j = k * (128 / N);
    const R c = (R)kTw128[j][0];
    const R s = (R)kTw128[j][1];
    return INV ? cmake(c, -s) : cmake(c, s);
}

template <int N> struct bitrev {
    static constexpr int L = (N == 64) ? 6 : (N == 32) ? 5 : (N == 16) ? 4 : (N == 8) ? 3 : (N == 4) ? 2 : 1;
    static __host__ __device__ constexpr int of(int i) {
        int r = 0;
        for (int b = 0; b < L; ++b)
            if (i & (1 << b)) r |= 1 << (L - 1 - b);
        return r;
    }
};

// In-register radix-2 decimation-in-time FFT.
template <typename R, int N, bool INV> __device__ __forceinline__ void fft_reg(cplx<R> (&a)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const int j = bitrev<N>::of(i);
        if (j > i) {   // per component: a struct copy can be lowered through private memory
            const R tx = a[i].x, ty = a[i].y;
            a[i].x = a[j].x;
            a[i].y = a[j].y;
            a[j].x = tx;
            a[j].y = ty;
        }
    }
#pragma unroll
    for (int len = 2; len <= N; len <<= 1) {
        const int half = len >> 1;
#pragma unroll
        for (int i = 0; i < N; i += len) {
#pragma unroll
            for (int k = 0; k < half; ++k) {
                const cplx<R> u = a[i + k], v = a[i + k + half];
                if (k == 0) {
                    a[i + k] = cadd(u, v);
                    a[i + k + half] = csub(u, v);
                } else {
                    // u + w v with four fused multiply-adds, then u - w v = 2u - (u + w v)
                    const cplx<R> w = twiddle<R, N, INV>(k * (N / len));
                    cplx<R> p;
                    p.x = fma(w.x, v.x, fma(-w.y, v.y, u.x));
                    p.y = fma(w.x, v.y, fma(w.y, v.x, u.y));
                    a[i + k] = p;
                    a[i + k + half] = cmake<R>(fma((R)2, u.x, -p.x), fma((R)2, u.y, -p.y));
                }
            }
        }
    }
}

// ---- LGF lookup (device table + asymptotic series) ----------------------

constexpr int kTableRadius = 128;       // exact near field for max|n_i| <= 128

// Asymptotic LGF of the unscaled 7-point Laplacian for large |n| (three
// corrections beyond -1/(4 pi r)); coefficients from the symbol expansion of
// sum_i 4 sin^2(theta_i / 2).
__device__ __forceinline__ double lgf_far(double x, double y, double z) {
    const double pi = 3.14159265358979323846;
    const double x2 = x * x, y2 = y * y, z2 = z * z;
    const double x4 = x2 * x2, y4 = y2 * y2, z4 = z2 * z2;
    const double x6 = x4 * x2, y6 = y4 * y2, z6 = z4 * z2;
    const double x8 = x4 * x4, y8 = y4 * y4, z8 = z4 * z4;
    const double p2 = x2 * y2 * z2;
    const double r2 = x2 + y2 + z2;
    const double r = sqrt(r2);
    const double s4 = x4 + y4 + z4;
    const double m22 = x2 * y2 + y2 * z2 + z2 * x2;
    const double q4 = s4 - 3.0 * m22;
    const double q8 = 23.0 * (x8 + y8 + z8) - 244.0 * (x6 * (y2 + z2) + y6 * (z2 + x2) + z6 * (x2 + y2)) +
                      621.0 * (x4 * y4 + y4 * z4 + z4 * x4) - 228.0 * p2 * r2;
    const double q12 = 647.0 * (x6 * x6 + y6 * y6 + z6 * z6) -
                       16419.0 * (x8 * x2 * (y2 + z2) + y8 * y2 * (z2 + x2) + z8 * z2 * (x2 + y2)) +
                       106536.0 * (x8 * (y4 + z4) + y8 * (z4 + x4) + z8 * (x4 + y4)) -
                       15723.0 * p2 * (x6 + y6 + z6) - 178221.0 * (x6 * y6 + y6 * z6 + z6 * x6) -
                       74469.0 * p2 * (x4 * (y2 + z2) + y4 * (z2 + x2) + z4 * (x2 + y2)) +
                       626835.0 * x4 * y4 * z4;
    const double ir = 1.0 / r;
    const double ir2 = ir * ir;
    const double ir6 = ir2 * ir2 * ir2;
    const double g = ir * (0.25 / pi) * (1.0 + q4 * ir6 * 0.25 + q8 * ir6 * ir6 * (1.0 / 32.0) +
                                        q12 * ir6 * ir6 * ir6 * (1.0 / 128.0));
    return -g;
}

// G(n) from the dense near cube gc[(a*(R+1) + b)*(R+1) + c], a,b,c = |n_i|.
__device__ __forceinline__ double lgf_G(const double *__restrict__ gc, int nx, int ny, int nz) {
    const int a = abs(nx), b = abs(ny), c = abs(nz);
    if (a <= kTableRadius && b <= kTableRadius && c <= kTableRadius) {
        const int s = kTableRadius + 1;
        return gc[((size_t)a * s + b) * s + c];
    }
    return lgf_far((double)a, (double)b, (double)c);
}

// The kernel of a convolution at lattice offset n: the LGF (far = true: the
// near cube, then the asymptotic series), or a kernel tabulated on the same
// cube that vanishes beyond it (far = false: the integrating factor).
__device__ __forceinline__ double kernel_at(const double *__restrict__ gc, bool far, int nx, int ny, int nz) {
    if (far) return lgf_G(gc, nx, ny, nz);
    const int a = abs(nx), b = abs(ny), c = abs(nz);
    if (a <= kTableRadius && b <= kTableRadius && c <= kTableRadius) {
        const int s = kTableRadius + 1;
        return gc[((size_t)a * s + b) * s + c];
    }
    return 0.0;
}

// Workgroups are dispatched round-robin over the 8 XCDs (hardware id b lands
// on XCD b mod 8); renumber them so that consecutive logical ids run on the
// same XCD and share its L2.  A bijection on [0, n) for any n.
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t n) {
    const int64_t xcd = b % 8, idx = b / 8, per = n / 8, rem = n % 8;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

}  // namespace lgf
