// Two-grid fast-LGF far field: anterpolation of a block's cells to its own
// node lattice and interpolation back (the far-field approximation of the
// fast LGF summation, paper Sec. 2.2 / Sec. 5, read from first principles).
//
// Every block of NB^3 cells owns (NB/2)^3 nodes, node k at fine position
// 2k + 1 along each axis (so node differences are even lattice vectors).  A
// cell takes the 4 nodes nearest to it along each axis, the window shifted
// to stay inside the block, with cubic Lagrange weights; the 3-D weights are
// products.  Interpolation I: cell value = sum over its 64 nodes of weight *
// node value.  Anterpolation A = I^T: node value = sum over the block's
// cells of the same weights times the cell values.  Both run as three 1-D
// passes through LDS, one workgroup per block.
#include <cstdint>

#include "lgf_kernels.hpp"

namespace lgf {

namespace {

// W[k * NB + i]: weight of node k for cell i along one axis (0 outside the
// cell's window).
template <int NB> __device__ void node_weights(double *W) {
    constexpr int H = NB / 2;
    for (int e = threadIdx.x; e < H * NB; e += blockDim.x) {
        const int k = e / NB, i = e % NB;
        const double x = (i + 0.5) * 0.5;
        int start = (int)floor(x - 0.5) - 1;
        start = start < 0 ? 0 : (start > H - 4 ? H - 4 : start);
        double w = 0.0;
        if (k >= start && k < start + 4) {
            w = 1.0;
            const double pk = k + 0.5;
            for (int j = start; j < start + 4; ++j)
                if (j != k) w *= (x - (j + 0.5)) / (pk - (j + 0.5));
        }
        W[e] = w;
    }
}

template <int NB>
__global__ void __launch_bounds__(256) anterp_kernel(const double *__restrict__ f, const int64_t *__restrict__ off,
                                                     double *__restrict__ Fc) {
    constexpr int H = NB / 2;
    __shared__ double W[H * NB];
    __shared__ double S0[NB * NB * NB];
    __shared__ double S1[NB * NB * H];
    const int b = blockIdx.x;
    node_weights<NB>(W);
    const double *src = f + off[b];
    for (int i = threadIdx.x; i < NB * NB * NB; i += 256) S0[i] = src[i];
    __syncthreads();
    // x: S1[z][y][kx]
    for (int e = threadIdx.x; e < NB * NB * H; e += 256) {
        const int kx = e % H, zy = e / H;
        double a = 0.0;
        for (int i = 0; i < NB; ++i) a = fma(W[kx * NB + i], S0[zy * NB + i], a);
        S1[e] = a;
    }
    __syncthreads();
    // y: S0[z][ky][kx] (reused)
    for (int e = threadIdx.x; e < NB * H * H; e += 256) {
        const int kx = e % H, ky = (e / H) % H, z = e / (H * H);
        double a = 0.0;
        for (int j = 0; j < NB; ++j) a = fma(W[ky * NB + j], S1[(z * NB + j) * H + kx], a);
        S0[e] = a;
    }
    __syncthreads();
    // z: out[kz][ky][kx]
    double *dst = Fc + (int64_t)b * H * H * H;
    for (int e = threadIdx.x; e < H * H * H; e += 256) {
        const int kxy = e % (H * H), kz = e / (H * H);
        double a = 0.0;
        for (int l = 0; l < NB; ++l) a = fma(W[kz * NB + l], S0[l * H * H + kxy], a);
        dst[e] = a;
    }
}

template <int NB>
__global__ void __launch_bounds__(256) interp_kernel(const double *__restrict__ Uc, const int64_t *__restrict__ off,
                                                     double *__restrict__ u) {
    constexpr int H = NB / 2;
    __shared__ double W[H * NB];
    __shared__ double T0[NB * NB * NB];
    __shared__ double T1[NB * NB * H];
    const int b = blockIdx.x;
    node_weights<NB>(W);
    const double *src = Uc + (int64_t)b * H * H * H;
    for (int i = threadIdx.x; i < H * H * H; i += 256) T0[i] = src[i];
    __syncthreads();
    // z: T1[z][ky][kx]
    for (int e = threadIdx.x; e < NB * H * H; e += 256) {
        const int kxy = e % (H * H), z = e / (H * H);
        double a = 0.0;
        for (int k = 0; k < H; ++k) a = fma(W[k * NB + z], T0[k * H * H + kxy], a);
        T1[e] = a;
    }
    __syncthreads();
    // y: T0[z][y][kx]
    for (int e = threadIdx.x; e < NB * NB * H; e += 256) {
        const int kx = e % H, y = (e / H) % NB, z = e / (H * NB);
        double a = 0.0;
        for (int k = 0; k < H; ++k) a = fma(W[k * NB + y], T1[(z * H + k) * H + kx], a);
        T0[e] = a;
    }
    __syncthreads();
    // x: u[z][y][x] +=
    double *dst = u + off[b];
    for (int e = threadIdx.x; e < NB * NB * NB; e += 256) {
        const int x = e % NB, zy = e / NB;
        double a = 0.0;
        for (int k = 0; k < H; ++k) a = fma(W[k * NB + x], T0[zy * H + k], a);
        dst[e] += a;
    }
}

}  // namespace

hipError_t flgf_anterpolate(int nb, const double *f, const int64_t *off, int n_blocks, double *Fc, hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    if (nb != 16) return hipErrorInvalidValue;
    anterp_kernel<16><<<n_blocks, 256, 0, s>>>(f, off, Fc);
    return hipGetLastError();
}

hipError_t flgf_interpolate_add(int nb, const double *Uc, const int64_t *off, int n_blocks, double *u, hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    if (nb != 16) return hipErrorInvalidValue;
    interp_kernel<16><<<n_blocks, 256, 0, s>>>(Uc, off, u);
    return hipGetLastError();
}

}  // namespace lgf
