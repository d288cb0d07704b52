// LGF table generation and LGF block spectra (plan time, float64).
//
// Table (paper Sec. 5: G is tabulated exactly close to the origin and
// replaced by its asymptotic series far from it; one table serves every
// level).
// The LGF of the unscaled 7-point Laplacian has the Bessel-integral form
//
//     G(n) = - \int_0^inf prod_i e^{-2t} I_{n_i}(2t) dt.
//
// With t = e^u the integrand is smooth and decays at both ends, so the
// trapezoid rule on a uniform u grid converges geometrically.  For every
// node t_j this file computes the row B_j(n) = e^{-x} I_n(x), x = 2 t_j,
// n = 0..R (R = 128), by
//   * the power series of I_n for x <= 1,
//   * the backward continued-fraction recurrence for rho_k = I_k / I_{k-1}
//     (rho_k = 1 / (2k/x + rho_{k+1})) together with the normalisation
//     e^x = I_0 + 2 sum_{k>=1} I_k, accumulated backward as
//     T_k = rho_k (1 + T_{k+1}) so that e^{-x} I_0 = 1 / (1 + 2 T_1),
//     for 1 < x <= 1e5,
//   * Hankel's expansion e^{-x} I_n(x) ~ (2 pi x)^{-1/2} sum_k (-1)^k a_k(n)/x^k,
//     a_k = prod_{j<=k} (4n^2 - (2j-1)^2) / (k! 8^k), for x > 1e5,
// and then G(a, b, c) = - sum_j w_j B_j(a) B_j(b) B_j(c) for 0 <= a, b, c <= R
// (a rank-n_nodes contraction).  Beyond max|n_i| > R the asymptotic series of
// lgf_device.hpp is used.
//
// Spectra (Sec. 2.2 convolution evaluated blockwise): for a block offset d the
// kernel window K_d(m) = G(d nb + m), m in [-(nb-1), nb-1]^3, is laid on a
// (2nb)^3 grid circularly (index m mod 2nb; the index nb stays 0) and
// transformed with a real-to-complex FFT.  G is even in every coordinate, so
// only offsets with dx, dy, dz >= 0 are stored (frequency-major,
// tab[omega][dy][dz][dx]); a reflection of the offset is a reflection of the
// window, i.e. a sign flip of the matching frequency index (see the loader
// in lgf_smac.hip).
#include <math.h>

#include "lgf_device.hpp"
#include "lgf_kernels.hpp"

namespace lgf {

namespace {

constexpr int kS = kTableRadius + 1;

__global__ void bessel_rows_kernel(double *__restrict__ B, double *__restrict__ w, int n_nodes, double u0,
                                   double h) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_nodes) return;
    const double u = u0 + j * h;
    const double t = exp(u);
    const double x = 2.0 * t;
    w[j] = h * t;
    double *row = B + (size_t)j * kS;
    if (x <= 1.0) {
        const double q = 0.25 * x * x;
        for (int n = 0; n < kS; ++n) {
            // (x/2)^n / n! * e^{-x}, then the series in q
            double term = exp(n * log(0.5 * x) - lgamma((double)n + 1.0) - x);
            double sum = term;
            for (int k = 1; k < 60; ++k) {
                term *= q / ((double)k * (double)(n + k));
                sum += term;
                if (term < 1e-19 * sum) break;
            }
            row[n] = sum;
        }
    } else if (x <= 1.0e5) {
        const int N = kTableRadius + 40 + (int)(10.0 * sqrt(x));
        double rho = 0.0, T = 0.0;
        for (int k = N; k >= 1; --k) {
            rho = 1.0 / (2.0 * k / x + rho);
            T = rho * (1.0 + T);
            if (k <= kTableRadius) row[k] = rho;
        }
        double v = 1.0 / (1.0 + 2.0 * T);
        row[0] = v;
        for (int k = 1; k < kS; ++k) {
            v *= row[k];
            row[k] = v;
        }
    } else {
        const double pre = 1.0 / sqrt(2.0 * 3.14159265358979323846 * x);
        for (int n = 0; n < kS; ++n) {
            const double mu = 4.0 * n * n;
            double term = 1.0, sum = 1.0;
            for (int k = 1; k < 40; ++k) {
                const double o = 2.0 * k - 1.0;
                term = -term * (mu - o * o) / (8.0 * k * x);
                sum += term;
                if (fabs(term) < 1e-19) break;
            }
            row[n] = pre * sum;
        }
    }
}

__global__ void near_cube_kernel(const double *__restrict__ B, const double *__restrict__ w, int n_nodes,
                                 double *__restrict__ gc) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kS * kS * kS) return;
    const int c = idx % kS;
    const int b = (idx / kS) % kS;
    const int a = idx / (kS * kS);
    // sort so that every permutation of (a, b, c) rounds identically
    int hi = max(a, max(b, c)), lo = min(a, min(b, c));
    int mid = a + b + c - hi - lo;
    double acc = 0.0;
    for (int j = 0; j < n_nodes; ++j) {
        const double *r = B + (size_t)j * kS;
        acc = fma(w[j] * r[hi] * r[mid], r[lo], acc);
    }
    gc[idx] = -acc;
}

__global__ void eval_points_kernel(const double *__restrict__ gc, const int *__restrict__ ijk,
                                   double *__restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = lgf_G(gc, ijk[3 * i], ijk[3 * i + 1], ijk[3 * i + 2]);
}

// ---- spectra: three global-memory FFT passes over a chunk of offsets ----

struct SpecGeom {
    int nb, XH, YH, ZH, XD, YD, ZD;
    int o_begin, o_count;   // linear offset range [o_begin, o_begin + o_count)
    int far;                // 1: the LGF (cube + asymptotic series); 0: a cube kernel, 0 beyond it
    int stride;             // the kernel sampled at stride * n
    int band, D;            // 0: every offset; 1: only max|d_i| <= D; 2: only max|d_i| > D
};

__device__ __forceinline__ void offset_of(const SpecGeom &g, int o, int &dx, int &dy, int &dz) {
    // linear offset o -> (dx, dy, dz) >= 0; table order is [dy][dz][dx]
    dx = o % g.XD;
    dz = (o / g.XD) % g.ZD;
    dy = o / (g.XD * g.ZD);
}

template <int N> __device__ __forceinline__ int circ(int i) {
    // grid index -> window displacement m (index N/2 is unused)
    return i < N / 2 ? i : i - N;
}

template <int N>
__global__ void spec_pass_x(const double *__restrict__ gc, SpecGeom g, cplx<double> *__restrict__ S) {
    constexpr int H = N / 2 + 1;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)g.o_count * N * N) return;
    const int y = tid % N, z = (tid / N) % N;
    const int ol = (int)(tid / (N * N));
    int dx, dy, dz;
    offset_of(g, g.o_begin + ol, dx, dy, dz);
    cplx<double> a[N];
    const int dm = max(dx, max(dy, dz));
    const bool zero_row = (y == N / 2) || (z == N / 2) || (g.band == 1 && dm > g.D) || (g.band == 2 && dm <= g.D);
#pragma unroll
    for (int x = 0; x < N; ++x) {
        double v = 0.0;
        if (!zero_row && x != N / 2)
            v = kernel_at(gc, g.far != 0, g.stride * (dx * g.nb + circ<N>(x)), g.stride * (dy * g.nb + circ<N>(y)),
                          g.stride * (dz * g.nb + circ<N>(z)));
        a[x] = cmake(v, 0.0);
    }
    fft_reg<double, N, false>(a);
    cplx<double> *o = S + ((size_t)ol * N * N + (size_t)z * N + y) * H;
#pragma unroll
    for (int k = 0; k < H; ++k) o[k] = a[k];
}

template <int N> __global__ void spec_pass_y(SpecGeom g, cplx<double> *__restrict__ S) {
    constexpr int H = N / 2 + 1;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)g.o_count * N * H) return;
    const int kx = tid % H, z = (tid / H) % N;
    const int ol = (int)(tid / (N * H));
    cplx<double> *base = S + ((size_t)ol * N * N + (size_t)z * N) * H + kx;
    cplx<double> a[N];
#pragma unroll
    for (int y = 0; y < N; ++y) a[y] = base[(size_t)y * H];
    fft_reg<double, N, false>(a);
#pragma unroll
    for (int y = 0; y < N; ++y) base[(size_t)y * H] = a[y];
}

template <int N, typename T>
__global__ void spec_pass_z(SpecGeom g, const cplx<double> *__restrict__ S, cplx<T> *__restrict__ tab) {
    constexpr int H = N / 2 + 1;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)g.o_count * N * H) return;
    const int kx = tid % H, ky = (tid / H) % N;
    const int ol = (int)(tid / (N * H));
    const cplx<double> *base = S + (size_t)ol * N * N * H + (size_t)ky * H + kx;
    cplx<double> a[N];
#pragma unroll
    for (int z = 0; z < N; ++z) a[z] = base[(size_t)z * N * H];
    fft_reg<double, N, false>(a);
    const size_t per = (size_t)g.XD * g.YD * g.ZD;
    const int o = g.o_begin + ol;
#pragma unroll
    for (int kz = 0; kz < N; ++kz) {
        const size_t omega = ((size_t)kz * N + ky) * H + kx;
        cplx<T> v;
        v.x = (T)a[kz].x;
        v.y = (T)a[kz].y;
        tab[omega * per + o] = v;
    }
}

template <int N, typename T>
hipError_t build_spectra_n(const double *gc, bool far, int stride, int band, int D, int nb, int XH, int YH, int ZH,
                           void *table, void *scratch, size_t scratch_bytes, hipStream_t s) {
    constexpr int H = N / 2 + 1;
    SpecGeom g;
    g.far = far ? 1 : 0;
    g.stride = stride;
    g.band = band;
    g.D = D;
    g.nb = nb;
    g.XH = XH;
    g.YH = YH;
    g.ZH = ZH;
    g.XD = XH + 1;
    g.YD = YH + 1;
    g.ZD = ZH + 1;
    const int n_off = g.XD * g.YD * g.ZD;
    const size_t per_off = (size_t)N * N * H * sizeof(cplx<double>);
    const int chunk = (int)std::min<size_t>((size_t)n_off, scratch_bytes / per_off);
    if (chunk < 1) return hipErrorInvalidValue;
    cplx<double> *S = (cplx<double> *)scratch;
    for (int o0 = 0; o0 < n_off; o0 += chunk) {
        g.o_begin = o0;
        g.o_count = std::min(chunk, n_off - o0);
        const int64_t nx = (int64_t)g.o_count * N * N, nyz = (int64_t)g.o_count * N * H;
        hipLaunchKernelGGL(spec_pass_x<N>, dim3((unsigned)((nx + 127) / 128)), dim3(128), 0, s, gc, g, S);
        hipLaunchKernelGGL(spec_pass_y<N>, dim3((unsigned)((nyz + 127) / 128)), dim3(128), 0, s, g, S);
        hipLaunchKernelGGL((spec_pass_z<N, T>), dim3((unsigned)((nyz + 127) / 128)), dim3(128), 0, s, g, S,
                           (cplx<T> *)table);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

// Trapezoid grid in u = log t: [-42, 100] with step 1/8.  The integrand
// behaves like e^u for u -> -inf and like e^{-u/2} (4 pi)^{-3/2} for
// u -> +inf, so both truncations are below 1e-18.
constexpr double kU0 = -42.0, kU1 = 100.0, kH = 0.125;

int lgf_table_nodes() { return (int)((kU1 - kU0) / kH) + 1; }

hipError_t build_lgf_table(double *gcube, double *B, double *w, hipStream_t s) {
    const int n_nodes = lgf_table_nodes();
    hipLaunchKernelGGL(bessel_rows_kernel, dim3((n_nodes + 63) / 64), dim3(64), 0, s, B, w, n_nodes, kU0, kH);
    const int total = kS * kS * kS;
    hipLaunchKernelGGL(near_cube_kernel, dim3((total + 255) / 256), dim3(256), 0, s, B, w, n_nodes, gcube);
    return hipGetLastError();
}

hipError_t eval_lgf_points(const double *gcube, const int *ijk, double *out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(eval_points_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, gcube, ijk, out,
                       n);
    return hipGetLastError();
}

hipError_t build_spectra(const double *gcube, bool far, int stride, int band, int D, int nb, int XH, int YH, int ZH,
                         bool fp32, void *table, void *scratch, size_t scratch_bytes, hipStream_t s) {
    if (nb == 16)
        return fp32 ? build_spectra_n<32, float>(gcube, far, stride, band, D, nb, XH, YH, ZH, table, scratch,
                                                 scratch_bytes, s)
                    : build_spectra_n<32, double>(gcube, far, stride, band, D, nb, XH, YH, ZH, table, scratch,
                                                  scratch_bytes, s);
    if (nb == 8)
        return fp32 ? build_spectra_n<16, float>(gcube, far, stride, band, D, nb, XH, YH, ZH, table, scratch,
                                                 scratch_bytes, s)
                    : build_spectra_n<16, double>(gcube, far, stride, band, D, nb, XH, YH, ZH, table, scratch,
                                                  scratch_bytes, s);
    return hipErrorInvalidValue;
}

// Integrating factor of the discrete heat equation (paper Sec. 2.3, eqs.
// heat, IF-single): H(a) = exp(a L) for the unscaled 7-point L, a =
// kappa (t - tau) / dx^2.  exp(a (S + S^-1 - 2)) along one axis has the
// kernel e^{-2a} I_n(2a) (the generating function of I_n), so the 3-D kernel
// is E(n) = prod_i e^{-2a} I_{n_i}(2a): the integrand of the LGF's Bessel
// form at t = a.  One Bessel row at x = 2a (bessel_rows_kernel with the
// single node t = a), then the cube of its products.
namespace {
__global__ void if_cube_kernel(const double *__restrict__ B, double *__restrict__ cube) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kS * kS * kS) return;
    const int c = idx % kS, b = (idx / kS) % kS, a = idx / (kS * kS);
    const int hi = max(a, max(b, c)), lo = min(a, min(b, c)), mid = a + b + c - hi - lo;
    cube[idx] = B[hi] * B[mid] * B[lo];
}
}  // namespace

hipError_t build_if_table(double *cube, double *row, double *w, double a, hipStream_t s) {
    if (!(a > 0.0)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(bessel_rows_kernel, dim3(1), dim3(64), 0, s, row, w, 1, log(a), 0.0);
    const int total = kS * kS * kS;
    hipLaunchKernelGGL(if_cube_kernel, dim3((total + 255) / 256), dim3(256), 0, s, row, cube);
    return hipGetLastError();
}

}  // namespace lgf
