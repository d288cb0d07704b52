// Mixed-precision refinement of one blockwise LGF convolution (gfx950).
//
// Wanted: u = L_dx^-1 g on the target set T (g: the source, on its own
// blocks).  The lattice Green's function inverts L_dx exactly on compactly
// supported functions, so for ANY w supported on T
//
//     L_dx^-1 g = w + L_dx^-1 (g - L_dx w).
//
// Take u~ = a float32 solve on T (relative error ~1e-7) and, with depth(c)
// the L1 distance from cell c to the complement of T,
//
//     w = u~ on cells of depth >= 2,   0 elsewhere.
//
// rho = g - L_dx w is then small (float32 noise of u~) on cells of depth >= 3,
// where every stencil point sees w = u~; on depths 1 and 2 (the cut, which
// lies in the shell blocks of T) and on source blocks outside T it is of the
// size of g and u.  So
//
//     u = w + L_dx^-1 (rho on the cut + g outside T)      float64 convolution
//           + L_dx^-1 (rho on depth >= 3)                  float32 convolution
//
// The first convolution has only the cut and the outside sources as
// sources (a thin set, handled by the MAC's sparse rows); the second one's
// source is ~1e-7 of g, so float32 leaves ~1e-14 relative error.  Float64 is
// used for the Green's function table, the residual, the cut convolution and
// the accumulation.
#include "lgf_device.hpp"
#include "lgf_kernels.hpp"

namespace lgf {

namespace {

__device__ __forceinline__ int fdiv_d(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

struct Lookup {
    RefGeom g;
    const int *map;
    __device__ int tidx(int bx, int by, int bz) const {
        const int mx = bx - g.lo[0], my = by - g.lo[1], mz = bz - g.lo[2];
        if (mx < 0 || my < 0 || mz < 0 || mx >= g.dim[0] || my >= g.dim[1] || mz >= g.dim[2]) return -1;
        return map[((size_t)mz * g.dim[1] + my) * g.dim[0] + mx];
    }
};

// depth of every cell of the listed shell blocks: L1 distance to the
// complement of T, capped at 3
template <int NB>
__global__ void __launch_bounds__(256) depth_kernel(RefGeom g, const int *__restrict__ map,
                                                    const int *__restrict__ shblk, unsigned char *__restrict__ depth) {
    const int b = blockIdx.x;
    Lookup L{g, map};
    const int Bx = shblk[3 * b], By = shblk[3 * b + 1], Bz = shblk[3 * b + 2];
    for (int i = threadIdx.x; i < NB * NB * NB; i += 256) {
        const int x = Bx * NB + i % NB, y = By * NB + (i / NB) % NB, z = Bz * NB + i / (NB * NB);
        int d = 3;
        for (int ox = -2; ox <= 2; ++ox)
            for (int oy = -2; oy <= 2; ++oy)
                for (int oz = -2; oz <= 2; ++oz) {
                    const int l1 = abs(ox) + abs(oy) + abs(oz);
                    if (l1 == 0 || l1 >= d) continue;
                    if (L.tidx(fdiv_d(x + ox, NB), fdiv_d(y + oy, NB), fdiv_d(z + oz, NB)) < 0) d = l1;
                }
        depth[(size_t)b * NB * NB * NB + i] = (unsigned char)d;
    }
}

template <int NB>
__global__ void __launch_bounds__(256) residual_kernel(RefGeom g, const int *__restrict__ map,
                                                       const int *__restrict__ tblk, const int *__restrict__ t2sh,
                                                       const unsigned char *__restrict__ depth,
                                                       const double *__restrict__ ut, const double *__restrict__ src,
                                                       const int64_t *__restrict__ gofs,
                                                       const int64_t *__restrict__ dofs, double *__restrict__ dst,
                                                       int accumulate, double *__restrict__ rin,
                                                       double *__restrict__ rcut) {
    constexpr int NB3 = NB * NB * NB;
    const int b = blockIdx.x;
    Lookup L{g, map};
    const int Bx = tblk[3 * b], By = tblk[3 * b + 1], Bz = tblk[3 * b + 2];
    const int sh_b = t2sh[b];
    const double idx2 = 1.0 / (g.dx * g.dx);
    // w at a lattice cell: u~ where depth >= 2, else 0 (also outside T)
    auto w_at = [&](int x, int y, int z) -> double {
        const int bx = fdiv_d(x, NB), by = fdiv_d(y, NB), bz = fdiv_d(z, NB);
        const int li = ((z - bz * NB) * NB + (y - by * NB)) * NB + (x - bx * NB);
        const int t = L.tidx(bx, by, bz);
        if (t < 0) return 0.0;
        const int sh = t2sh[t];
        if (sh >= 0 && depth[(size_t)sh * NB3 + li] < 2) return 0.0;
        return ut[(size_t)t * NB3 + li];
    };
    // w at local cell j of this block (no block lookup)
    auto w_own = [&](int j) -> double {
        if (sh_b >= 0 && depth[(size_t)sh_b * NB3 + j] < 2) return 0.0;
        return ut[(size_t)b * NB3 + j];
    };
    for (int i = threadIdx.x; i < NB3; i += 256) {
        const int lx = i % NB, ly = (i / NB) % NB, lz = i / (NB * NB);
        const int x = Bx * NB + lx, y = By * NB + ly, z = Bz * NB + lz;
        const int d = sh_b >= 0 ? depth[(size_t)sh_b * NB3 + i] : 3;
        const double wc = d >= 2 ? ut[(size_t)b * NB3 + i] : 0.0;
        // neighbours inside the block read it directly; across a face, by lookup
        const double wxp = lx + 1 < NB ? w_own(i + 1) : w_at(x + 1, y, z);
        const double wxm = lx > 0 ? w_own(i - 1) : w_at(x - 1, y, z);
        const double wyp = ly + 1 < NB ? w_own(i + NB) : w_at(x, y + 1, z);
        const double wym = ly > 0 ? w_own(i - NB) : w_at(x, y - 1, z);
        const double wzp = lz + 1 < NB ? w_own(i + NB * NB) : w_at(x, y, z + 1);
        const double wzm = lz > 0 ? w_own(i - NB * NB) : w_at(x, y, z - 1);
        const double lap = wxp + wxm + wyp + wym + wzp + wzm - 6.0 * wc;
        const double gv = gofs[b] >= 0 ? src[gofs[b] + i] : 0.0;
        const double r = gv - idx2 * lap;
        double *dp = dst + dofs[b] + i;
        *dp = accumulate ? *dp + wc : wc;
        if (d <= 2) {
            rcut[(size_t)sh_b * NB3 + i] = r;
            rin[(size_t)b * NB3 + i] = 0.0;
        } else {
            rin[(size_t)b * NB3 + i] = r;
            if (sh_b >= 0) rcut[(size_t)sh_b * NB3 + i] = 0.0;
        }
    }
}

}  // namespace

hipError_t refine_depth(int nb, const RefGeom &g, const int *map, const int *shblk, unsigned char *depth, int n_sh,
                        hipStream_t s) {
    if (n_sh <= 0) return hipSuccess;
    if (nb == 16)
        hipLaunchKernelGGL(depth_kernel<16>, dim3(n_sh), dim3(256), 0, s, g, map, shblk, depth);
    else if (nb == 8)
        hipLaunchKernelGGL(depth_kernel<8>, dim3(n_sh), dim3(256), 0, s, g, map, shblk, depth);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t refine_residual(int nb, const RefGeom &g, const int *map, const int *tblk, const int *t2sh,
                           const unsigned char *depth, const double *ut, const double *src, const int64_t *gofs,
                           const int64_t *dofs, double *dst, int accumulate, double *rin, double *rcut, int n_t,
                           hipStream_t s) {
    if (n_t <= 0) return hipSuccess;
    if (nb == 16)
        hipLaunchKernelGGL(residual_kernel<16>, dim3(n_t), dim3(256), 0, s, g, map, tblk, t2sh, depth, ut, src, gofs,
                           dofs, dst, accumulate, rin, rcut);
    else if (nb == 8)
        hipLaunchKernelGGL(residual_kernel<8>, dim3(n_t), dim3(256), 0, s, g, map, tblk, t2sh, depth, ut, src, gofs,
                           dofs, dst, accumulate, rin, rcut);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace lgf
