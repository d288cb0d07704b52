// Velocity refresh (paper Sec. 4.1, eq. vel_update): u = -C^dagger L_E^-1 omega
// on one level.  The streamfunction psi = L_E^-1 omega is the LGF solve of
// each edge component (each lives on its own copy of the cell lattice);
// this kernel applies -C^dagger, the curl from edges to faces with backward
// differences (the adjoint of the forward-difference curl C, eq. mimetic):
//   u_x[n] = -(psi_z[n] - psi_z[n - e_y] - psi_y[n] + psi_y[n - e_z]) / dx
//   u_y[n] = -(psi_x[n] - psi_x[n - e_z] - psi_z[n] + psi_z[n - e_x]) / dx
//   u_z[n] = -(psi_y[n] - psi_y[n - e_x] - psi_x[n] + psi_x[n - e_y]) / dx
// A backward neighbour in another block is read through that block's
// offset; one outside the support makes the component NaN (psi is only
// known on the support).
#include <cstdint>

#include "lgf_kernels.hpp"

namespace lgf {

namespace {

template <int NB>
__global__ void __launch_bounds__(256) curl_back_kernel(const double *__restrict__ psi, double *__restrict__ u,
                                                        int64_t comp_len, const int64_t *__restrict__ blk_off,
                                                        const int64_t *__restrict__ nbr_off, double inv_dx) {
    const int b = blockIdx.x;
    const int64_t base = blk_off[b];
    const int64_t nb_[3] = {nbr_off[3 * b], nbr_off[3 * b + 1], nbr_off[3 * b + 2]};
    const double qnan = __longlong_as_double(0x7ff8000000000000LL);
    const double *pc[3] = {psi, psi + comp_len, psi + 2 * comp_len};
    for (int i = threadIdx.x; i < NB * NB * NB; i += 256) {
        const int c3[3] = {i % NB, (i / NB) % NB, i / (NB * NB)};
        const int stride[3] = {1, NB, NB * NB};
        // psi_c at the cell, and one cell back along axis a
        auto back = [&](int c, int a) -> double {
            if (c3[a] > 0) return pc[c][base + i - stride[a]];
            if (nb_[a] < 0) return qnan;
            return pc[c][nb_[a] + i + (NB - 1) * stride[a]];
        };
        const double px = pc[0][base + i], py = pc[1][base + i], pz = pc[2][base + i];
        u[base + i] = -((pz - back(2, 1)) - (py - back(1, 2))) * inv_dx;
        u[comp_len + base + i] = -((px - back(0, 2)) - (pz - back(2, 0))) * inv_dx;
        u[2 * comp_len + base + i] = -((py - back(1, 0)) - (px - back(0, 1))) * inv_dx;
    }
}

}  // namespace

hipError_t curl_backward_blocks(int nb, const double *psi, double *u, int64_t comp_len, const int64_t *blk_off,
                                const int64_t *nbr_off, int n_blocks, double inv_dx, hipStream_t s) {
    if (n_blocks <= 0) return hipSuccess;
    if (nb == 8)
        curl_back_kernel<8><<<n_blocks, 256, 0, s>>>(psi, u, comp_len, blk_off, nbr_off, inv_dx);
    else
        curl_back_kernel<16><<<n_blocks, 256, 0, s>>>(psi, u, comp_len, blk_off, nbr_off, inv_dx);
    return hipGetLastError();
}

}  // namespace lgf
