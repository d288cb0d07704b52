// Mixed-precision refinement of one blockwise LGF convolution (gfx950).
//
// u = L_dx^-1 g on the target set T is first computed with float32 spectra,
// FFTs and products (u~, relative error ~1e-7).  The error e = u - u~ is not
// recoverable from a residual on T alone: its discrete-harmonic part is
// fixed by values on the boundary of T.  So exact float64 values are taken
// on the shell blocks of T (blocks with any of their 26 neighbours outside
// T), and with depth(c) = L1 distance from cell c to the complement of T the
// function
//
//     e^ = e on cells of depth >= 3,  0 elsewhere
//
// is compactly supported, hence e^ = L_dx^-1 (L_dx e^) exactly (the lattice
// Green's function inverts L on compactly supported functions).  L_dx e^ is
// known in float64:
//     depth >= 4:  g - L_dx u~
//     depth == 3:  g - L_dx u~ - dx^-2 sum_{nbr depth 2} e(nbr)
//     depth == 2:  dx^-2 sum_{nbr depth 3} e(nbr)
//     depth <= 1:  0
// with e = u_exact - u~ on depths 2 and 3 (shell blocks).  One more float32
// convolution of this residual gives e^ with error ~1e-7 |e^| ~ 1e-14 |u|.
// The result is u_exact on shell blocks and u~ + e^ on the interior blocks.
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

template <int NB>
__global__ void __launch_bounds__(256) depth_kernel(RefGeom g, const int *__restrict__ map,
                                                    const int *__restrict__ shblk, unsigned char *__restrict__ depth) {
    const int b = blockIdx.x;
    Lookup L{g, map};
    const int Bx = shblk[3 * b], By = shblk[3 * b + 1], Bz = shblk[3 * b + 2];
    for (int i = threadIdx.x; i < NB * NB * NB; i += 256) {
        const int x = Bx * NB + i % NB, y = By * NB + (i / NB) % NB, z = Bz * NB + i / (NB * NB);
        int d = 4;
        for (int ox = -3; ox <= 3; ++ox)
            for (int oy = -3; oy <= 3; ++oy)
                for (int oz = -3; oz <= 3; ++oz) {
                    const int l1 = abs(ox) + abs(oy) + abs(oz);
                    if (l1 == 0 || l1 > 3 || l1 >= d) continue;
                    if (L.tidx(fdiv_d(x + ox, NB), fdiv_d(y + oy, NB), fdiv_d(z + oz, NB)) < 0) d = l1;
                }
        depth[(size_t)b * NB * NB * NB + i] = (unsigned char)d;
    }
}

template <int NB>
__global__ void __launch_bounds__(256) residual_kernel(RefGeom g, const int *__restrict__ map,
                                                       const int *__restrict__ tblk, const int *__restrict__ t2sh,
                                                       const unsigned char *__restrict__ depth,
                                                       const double *__restrict__ ut, const double *__restrict__ ush,
                                                       const double *__restrict__ src,
                                                       const int64_t *__restrict__ gofs, double *__restrict__ rho) {
    constexpr int NB3 = NB * NB * NB;
    const int b = blockIdx.x;
    Lookup L{g, map};
    const int Bx = tblk[3 * b], By = tblk[3 * b + 1], Bz = tblk[3 * b + 2];
    const double idx2 = 1.0 / (g.dx * g.dx);
    // (T index, local cell) of a lattice cell; T index -1 outside T
    auto locate = [&](int x, int y, int z, int &li) -> int {
        const int bx = fdiv_d(x, NB), by = fdiv_d(y, NB), bz = fdiv_d(z, NB);
        li = ((z - bz * NB) * NB + (y - by * NB)) * NB + (x - bx * NB);
        return L.tidx(bx, by, bz);
    };
    auto depth_of = [&](int t, int li) -> int {
        if (t < 0) return 0;
        const int sh = t2sh[t];
        return sh < 0 ? 4 : depth[(size_t)sh * NB3 + li];
    };
    auto err = [&](int t, int li) -> double {   // u_exact - u~ (shell cells only)
        return ush[(size_t)t2sh[t] * NB3 + li] - ut[(size_t)t * NB3 + li];
    };
    const int nbr[6][3] = {{1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1}};
    for (int i = threadIdx.x; i < NB3; i += 256) {
        const int x = Bx * NB + i % NB, y = By * NB + (i / NB) % NB, z = Bz * NB + i / (NB * NB);
        const int d = depth_of(b, i);
        double r = 0.0;
        if (d == 2) {
            double acc = 0.0;
            for (int q = 0; q < 6; ++q) {
                int li;
                const int t = locate(x + nbr[q][0], y + nbr[q][1], z + nbr[q][2], li);
                if (depth_of(t, li) == 3) acc += err(t, li);
            }
            r = idx2 * acc;
        } else if (d >= 3) {
            double lap = -6.0 * ut[(size_t)b * NB3 + i];
            double e2 = 0.0;
            for (int q = 0; q < 6; ++q) {
                int li;
                const int t = locate(x + nbr[q][0], y + nbr[q][1], z + nbr[q][2], li);
                lap += ut[(size_t)t * NB3 + li];
                if (d == 3 && depth_of(t, li) == 2) e2 += err(t, li);
            }
            const double gv = gofs[b] >= 0 ? src[gofs[b] + i] : 0.0;
            r = gv - idx2 * lap - idx2 * e2;
        }
        rho[(size_t)b * NB3 + i] = r;
    }
}

// dst block (per T block b) (+)= ush (shell) or ut (interior)
template <int NB>
__global__ void __launch_bounds__(256) assemble_kernel(const int *__restrict__ t2sh, const double *__restrict__ ut,
                                                       const double *__restrict__ ush,
                                                       const int64_t *__restrict__ dofs, double *__restrict__ dst,
                                                       int accumulate) {
    constexpr int NB3 = NB * NB * NB;
    const int b = blockIdx.x;
    const int sh = t2sh[b];
    const double *s = sh >= 0 ? ush + (size_t)sh * NB3 : ut + (size_t)b * NB3;
    double *d = dst + dofs[b];
    for (int i = threadIdx.x; i < NB3; i += 256) d[i] = accumulate ? d[i] + s[i] : s[i];
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
                           const unsigned char *depth, const double *ut, const double *ush, const double *src,
                           const int64_t *gofs, double *rho, int n_t, hipStream_t s) {
    if (n_t <= 0) return hipSuccess;
    if (nb == 16)
        hipLaunchKernelGGL(residual_kernel<16>, dim3(n_t), dim3(256), 0, s, g, map, tblk, t2sh, depth, ut, ush, src,
                           gofs, rho);
    else if (nb == 8)
        hipLaunchKernelGGL(residual_kernel<8>, dim3(n_t), dim3(256), 0, s, g, map, tblk, t2sh, depth, ut, ush, src,
                           gofs, rho);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t refine_assemble(int nb, const int *t2sh, const double *ut, const double *ush, const int64_t *dofs,
                           double *dst, int accumulate, int n_t, hipStream_t s) {
    if (n_t <= 0) return hipSuccess;
    if (nb == 16)
        hipLaunchKernelGGL(assemble_kernel<16>, dim3(n_t), dim3(256), 0, s, t2sh, ut, ush, dofs, dst, accumulate);
    else if (nb == 8)
        hipLaunchKernelGGL(assemble_kernel<8>, dim3(n_t), dim3(256), 0, s, t2sh, ut, ush, dofs, dst, accumulate);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace lgf
