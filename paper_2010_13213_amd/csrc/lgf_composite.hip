// Composite-grid (multi-level) kernels of the FLGF-AMR solve (gfx950).
//
// Paper Sec. 3.2-3.4.  Level k+1 halves the cell width of level k; a
// level-(k+1) cell c' is a child of level-k cell floor(c'/2).
//  * mask_blocks: restriction to Omega_k -- cells of a level-k block whose
//    octant is covered by a level-(k+1) block, and cells the caller's cell
//    mask drops, are zeroed (f^_k = Gamma_k f_k, and the returned phi_k is 0
//    there).
//  * coarsen_mean8: P_{k+1->k}, the mean of the 8 children, written into the
//    covered octant of the parent block (step 1 of the algorithm,
//    F_k = f^_k + P_{k+1->k} F_{k+1}).
//  * correction: for one level-k block of Omega_k u Omega_k^E, from
//    psi_{k-1} staged in LDS it forms
//        P psi_{k-1}                       (cell-centred trilinear, weights 1/4, 3/4)
//        S = P (L_{k-1} psi_{k-1}) - L_k (P psi_{k-1})    (eq. source_correct)
//    and writes P psi, S + F_k and S + f^_k (the two right-hand sides of
//    eq. combine_S; F_k / f^_k are zero outside the level's own blocks).
//  * copy_blocks: block-list copy (P psi into the targets before the
//    convolution adds L_k^-1 of the sources).
#include <algorithm>
#include <cstdint>

#include "lgf_device.hpp"
#include "lgf_kernels.hpp"

namespace lgf {

namespace {

__device__ __forceinline__ int fdiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

template <int NB>
__global__ void __launch_bounds__(256) mask_kernel(const double *__restrict__ src, double *__restrict__ dst,
                                                   const int64_t *__restrict__ src_off,
                                                   const int64_t *__restrict__ dst_off,
                                                   const unsigned char *__restrict__ cover,
                                                   const unsigned char *__restrict__ cmask) {
    constexpr int H = NB / 2;
    const int b = blockIdx.x;
    const double *s = src + src_off[b];
    double *d = dst + dst_off[b];
    const unsigned m = cover ? cover[b] : 0u;
    const unsigned char *cm = cmask ? cmask + (size_t)b * NB * NB * NB : nullptr;
    for (int i = threadIdx.x; i < NB * NB * NB; i += 256) {
        const int x = i % NB, y = (i / NB) % NB, z = i / (NB * NB);
        const int oct = (x >= H) | ((y >= H) << 1) | ((z >= H) << 2);
        const bool keep = !((m >> oct) & 1u) && (!cm || cm[i]);
        d[i] = keep ? s[i] : 0.0;
    }
}

// pairs[i] = {fine block offset, coarse block offset, octant}: one workgroup
// per fine block, one thread per coarse cell of the octant.
template <int NB>
__global__ void __launch_bounds__(256) coarsen_kernel(const double *__restrict__ fine, double *__restrict__ coarse,
                                                      const int64_t *__restrict__ fine_off,
                                                      const int64_t *__restrict__ coarse_off,
                                                      const unsigned char *__restrict__ octant) {
    constexpr int H = NB / 2;
    const int b = blockIdx.x;
    const double *f = fine + fine_off[b];
    double *c = coarse + coarse_off[b];
    const int o = octant[b];
    const int ox = (o & 1) * H, oy = ((o >> 1) & 1) * H, oz = ((o >> 2) & 1) * H;
    for (int i = threadIdx.x; i < H * H * H; i += 256) {
        const int x = i % H, y = (i / H) % H, z = i / (H * H);
        double acc = 0.0;
#pragma unroll
        for (int dz = 0; dz < 2; ++dz)
#pragma unroll
            for (int dy = 0; dy < 2; ++dy)
#pragma unroll
                for (int dx = 0; dx < 2; ++dx)
                    acc += f[((2 * z + dz) * NB + (2 * y + dy)) * NB + (2 * x + dx)];
        c[((oz + z) * NB + (oy + y)) * NB + (ox + x)] = acc * 0.125;
    }
}

__global__ void copy_kernel(const double *__restrict__ src, double *__restrict__ dst,
                            const int64_t *__restrict__ src_off, const int64_t *__restrict__ dst_off, int nb3) {
    const int b = blockIdx.x;
    const double *s = src + src_off[b];
    double *d = dst + dst_off[b];
    for (int i = threadIdx.x; i < nb3; i += blockDim.x) d[i] = s[i];
}

// Zero n 16-byte words (grid-stride, vector stores).  Used instead of a
// memset node wherever a solve may be captured into a graph.
__global__ void zero_kernel(int4 *__restrict__ p, int64_t n) {
    const int4 z = make_int4(0, 0, 0, 0);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = z;
}

// Trilinear value at fine cell (fx, fy, fz) from a coarse array staged in LDS
// with origin q0 and edge CS.
template <int CS>
__device__ __forceinline__ double trilinear(const double *c, int q0x, int q0y, int q0z, int fx, int fy, int fz) {
    const int px = fdiv(fx, 2), py = fdiv(fy, 2), pz = fdiv(fz, 2);
    const int sx = fx - 2 * px, sy = fy - 2 * py, sz = fz - 2 * pz;
    // per axis: s = 0 -> (p-1: 1/4, p: 3/4), s = 1 -> (p: 3/4, p+1: 1/4)
    const int ax = (sx == 0 ? px - 1 : px) - q0x, ay = (sy == 0 ? py - 1 : py) - q0y,
              az = (sz == 0 ? pz - 1 : pz) - q0z;
    const double wx0 = sx == 0 ? 0.25 : 0.75, wx1 = 1.0 - wx0;
    const double wy0 = sy == 0 ? 0.25 : 0.75, wy1 = 1.0 - wy0;
    const double wz0 = sz == 0 ? 0.25 : 0.75, wz1 = 1.0 - wz0;
    auto at = [&](int i, int j, int k) { return c[(k * CS + j) * CS + i]; };
    const double v0 = wy0 * (wx0 * at(ax, ay, az) + wx1 * at(ax + 1, ay, az)) +
                      wy1 * (wx0 * at(ax, ay + 1, az) + wx1 * at(ax + 1, ay + 1, az));
    const double v1 = wy0 * (wx0 * at(ax, ay, az + 1) + wx1 * at(ax + 1, ay, az + 1)) +
                      wy1 * (wx0 * at(ax, ay + 1, az + 1) + wx1 * at(ax + 1, ay + 1, az + 1));
    return wz0 * v0 + wz1 * v1;
}

template <int NB>
__global__ void __launch_bounds__(256) correction_kernel(CorrGeom g, const double *__restrict__ psi,
                                                         const int *__restrict__ cmap,
                                                         const int *__restrict__ fblk,
                                                         const int64_t *__restrict__ own_off,
                                                         const double *__restrict__ Fk,
                                                         const double *__restrict__ fhk,
                                                         double *__restrict__ Ppsi, double *__restrict__ SrcF,
                                                         double *__restrict__ Srcf) {
    constexpr int H = NB / 2;
    constexpr int CS = H + 4;    // staged coarse psi: [B*H - 2, B*H + H + 2)
    constexpr int CL = H + 2;    // coarse L psi:      [B*H - 1, B*H + H + 1)
    constexpr int FS = NB + 2;   // fine P psi:        [B*NB - 1, B*NB + NB + 1)
    __shared__ double cps[CS * CS * CS];
    __shared__ double clp[CL * CL * CL];
    __shared__ double fpp[FS * FS * FS];
    const int b = blockIdx.x;
    const int Bx = fblk[3 * b], By = fblk[3 * b + 1], Bz = fblk[3 * b + 2];
    const int q0x = Bx * H - 2, q0y = By * H - 2, q0z = Bz * H - 2;
    const double icd2 = 1.0 / (g.dxc * g.dxc), ifd2 = 1.0 / (g.dxf * g.dxf);

    // stage psi_{k-1}
    for (int i = threadIdx.x; i < CS * CS * CS; i += 256) {
        const int qx = q0x + i % CS, qy = q0y + (i / CS) % CS, qz = q0z + i / (CS * CS);
        const int cbx = fdiv(qx, NB), cby = fdiv(qy, NB), cbz = fdiv(qz, NB);
        const int mx = cbx - g.mlo[0], my = cby - g.mlo[1], mz = cbz - g.mlo[2];
        double v = 0.0;
        if (mx >= 0 && my >= 0 && mz >= 0 && mx < g.mdim[0] && my < g.mdim[1] && mz < g.mdim[2]) {
            const int idx = cmap[((size_t)mz * g.mdim[1] + my) * g.mdim[0] + mx];
            if (idx >= 0)
                v = psi[(size_t)idx * NB * NB * NB + (((qz - cbz * NB) * NB + (qy - cby * NB)) * NB + (qx - cbx * NB))];
        }
        cps[i] = v;
    }
    __syncthreads();
    // L_{k-1} psi on the inner coarse cells
    for (int i = threadIdx.x; i < CL * CL * CL; i += 256) {
        const int x = i % CL + 1, y = (i / CL) % CL + 1, z = i / (CL * CL) + 1;
        auto at = [&](int a, int bb, int c) { return cps[(c * CS + bb) * CS + a]; };
        clp[i] = (at(x + 1, y, z) + at(x - 1, y, z) + at(x, y + 1, z) + at(x, y - 1, z) + at(x, y, z + 1) +
                  at(x, y, z - 1) - 6.0 * at(x, y, z)) *
                 icd2;
    }
    // P psi on the fine block plus one halo layer
    for (int i = threadIdx.x; i < FS * FS * FS; i += 256) {
        const int fx = Bx * NB - 1 + i % FS, fy = By * NB - 1 + (i / FS) % FS, fz = Bz * NB - 1 + i / (FS * FS);
        fpp[i] = trilinear<CS>(cps, q0x, q0y, q0z, fx, fy, fz);
    }
    __syncthreads();
    const int64_t oo = own_off[b];
    const size_t base = (size_t)b * NB * NB * NB;
    for (int i = threadIdx.x; i < NB * NB * NB; i += 256) {
        const int x = i % NB, y = (i / NB) % NB, z = i / (NB * NB);
        const int fx = Bx * NB + x, fy = By * NB + y, fz = Bz * NB + z;
        auto at = [&](int a, int bb, int c) { return fpp[((c + 1) * FS + (bb + 1)) * FS + (a + 1)]; };
        const double pp = at(x, y, z);
        const double lpp = (at(x + 1, y, z) + at(x - 1, y, z) + at(x, y + 1, z) + at(x, y - 1, z) +
                            at(x, y, z + 1) + at(x, y, z - 1) - 6.0 * pp) *
                           ifd2;
        const double plp = trilinear<CL>(clp, q0x + 1, q0y + 1, q0z + 1, fx, fy, fz);
        const double S = g.interp_only ? pp : plp - lpp;
        Ppsi[base + i] = pp;
        const double fk = oo >= 0 ? Fk[oo + i] : 0.0;
        const double hk = oo >= 0 ? fhk[oo + i] : 0.0;
        SrcF[base + i] = S + fk;
        Srcf[base + i] = S + hk;
    }
}

}  // namespace

hipError_t mask_blocks(int nb, const double *src, double *dst, const int64_t *src_off, const int64_t *dst_off,
                       const unsigned char *cover, int n_blocks, hipStream_t s, const unsigned char *cmask) {
    if (n_blocks <= 0) return hipSuccess;
    if (nb == 16)
        hipLaunchKernelGGL(mask_kernel<16>, dim3(n_blocks), dim3(256), 0, s, src, dst, src_off, dst_off, cover,
                           cmask);
    else if (nb == 8)
        hipLaunchKernelGGL(mask_kernel<8>, dim3(n_blocks), dim3(256), 0, s, src, dst, src_off, dst_off, cover,
                           cmask);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t coarsen_mean8(int nb, const double *fine, double *coarse, const int64_t *fine_off,
                         const int64_t *coarse_off, const unsigned char *octant, int n_pairs, hipStream_t s) {
    if (n_pairs <= 0) return hipSuccess;
    if (nb == 16)
        hipLaunchKernelGGL(coarsen_kernel<16>, dim3(n_pairs), dim3(256), 0, s, fine, coarse, fine_off, coarse_off,
                           octant);
    else if (nb == 8)
        hipLaunchKernelGGL(coarsen_kernel<8>, dim3(n_pairs), dim3(256), 0, s, fine, coarse, fine_off, coarse_off,
                           octant);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t copy_blocks(int nb, const double *src, double *dst, const int64_t *src_off, const int64_t *dst_off,
                       int n_blocks, hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    hipLaunchKernelGGL(copy_kernel, dim3(n_blocks), dim3(256), 0, s, src, dst, src_off, dst_off, nb * nb * nb);
    return hipGetLastError();
}

hipError_t zero_fill(void *p, size_t bytes, hipStream_t s) {
    if (bytes == 0) return hipSuccess;
    if (bytes % 16 != 0 || ((uintptr_t)p) % 16 != 0) return hipErrorInvalidValue;
    const int64_t n = (int64_t)(bytes / 16);
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (int4 *)p, n);
    return hipGetLastError();
}

hipError_t correction_source(int nb, const CorrGeom &g, const double *psi, const int *cmap, const int *fblk,
                             const int64_t *own_off, const double *Fk, const double *fhk, double *Ppsi,
                             double *SrcF, double *Srcf, int n_blocks, hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    if (nb == 16)
        hipLaunchKernelGGL(correction_kernel<16>, dim3(n_blocks), dim3(256), 0, s, g, psi, cmap, fblk, own_off, Fk,
                           fhk, Ppsi, SrcF, Srcf);
    else if (nb == 8)
        hipLaunchKernelGGL(correction_kernel<8>, dim3(n_blocks), dim3(256), 0, s, g, psi, cmap, fblk, own_off, Fk,
                           fhk, Ppsi, SrcF, Srcf);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

namespace {

// Per block: sum of squares and max |v| of the block's nb^3 values.
template <int NB>
__global__ void __launch_bounds__(256) stats_kernel(const double *__restrict__ v, const int64_t *__restrict__ off,
                                                    double *__restrict__ out) {
    const int b = blockIdx.x;
    const double *p = v + (off ? off[b] : (int64_t)b * NB * NB * NB);
    double ss = 0.0, mx = 0.0;
    for (int i = threadIdx.x; i < NB * NB * NB; i += 256) {
        const double a = p[i];
        ss += a * a;
        mx = fmax(mx, fabs(a));
    }
    __shared__ double s_ss[256], s_mx[256];
    s_ss[threadIdx.x] = ss;
    s_mx[threadIdx.x] = mx;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_ss[threadIdx.x] += s_ss[threadIdx.x + w];
            s_mx[threadIdx.x] = fmax(s_mx[threadIdx.x], s_mx[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[2 * b] = s_ss[0];
        out[2 * b + 1] = s_mx[0];
    }
}

}  // namespace

hipError_t block_stats(int nb, const double *v, const int64_t *off, int n_blocks, double *out, hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    if (nb == 8)
        stats_kernel<8><<<n_blocks, 256, 0, s>>>(v, off, out);
    else
        stats_kernel<16><<<n_blocks, 256, 0, s>>>(v, off, out);
    return hipGetLastError();
}

}  // namespace lgf
