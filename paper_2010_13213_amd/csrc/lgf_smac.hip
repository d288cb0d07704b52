// Spectral multiply-accumulate of the blockwise LGF convolution (gfx950).
//
// After the forward block FFTs, the convolution of a level (paper Sec. 2.2,
// eq. lgf_convolution; every block pair of the level, Sec. 5) is, at each
// frequency omega, a convolution over the block lattice:
//
//     Uhat_t(omega) = sum_s Khat_{t-s}(omega) Fhat_s(omega).
//
// Data layout: slots s = (z * ey + y) * bx + x over a padded box of blocks,
// Fhat / Uhat [omega][slot], spectra table K[omega][dy][dz][dx] for
// dx, dy, dz >= 0 only.  A negative dy (dz) reflects the window along y (z):
// its spectrum is the stored one at ky -> -ky (kz -> -kz).  A negative dx
// reflects along x, which the half spectrum in kx serves as the complex
// conjugate at (ky, kz) -> (-ky, -kz).
//
// One workgroup owns one frequency and one tile of TY x TZ target rows (a
// row is the bx blocks along x at fixed (y, z)).  Lane (seg, ty, tz) keeps A
// consecutive targets of its row in registers; a per-tile lane table gives
// lanes only to the x-segments that hold targets, so thin supports do not
// pay for the empty part of their rows (a crowded tile is split over
// several workgroups).  The workgroup walks the
// source rows (sy, sz) in serpentine order; for each row every lane needs
// the kernel row K[., ty - sy, tz - sz] (2 bx - 1 values along x), which
// lives in an LDS ring buffer of (TY+1) x (TZ+1) kernel rows indexed by
// (dy mod (TY+1), dz mod (TZ+1)).  A step of +-1 in sy or sz brings exactly
// one new plane (TZ rows) or layer (TY rows); it is prefetched into
// registers while the current row is computed and written to the free ring
// slot, so each step costs one barrier.  Other jumps reload the window.
// Inside a row the Toeplitz product U[i] += K[x0 + i - j] F[j] reuses each
// loaded kernel value across the lane's A targets, and the source row F is
// read by all lanes from one LDS address (broadcast).
//
// Right-hand sides: up to three components with the same sources and
// targets (a vector Poisson solve) go through one launch; every kernel row
// staged in LDS then serves all of them, dividing the per-row cost of the
// ring, the barrier and the window reads by the component count.
//
// Occupancy: the ring is (TY+1)(TZ+1)(2 bx - 1) complex values.  For bx = 16
// in float64 a 16 x 8 tile needs 76 KB, so two workgroups share a CU's
// 160 KB and one's barrier is covered by the other's arithmetic.  The LDS
// reads of each step are issued two steps ahead of their use, which spreads
// a row's reads over its arithmetic instead of queueing all of them behind
// the barrier.
#include <type_traits>

#include "lgf_device.hpp"
#include "lgf_kernels.hpp"

namespace lgf {

namespace {

__device__ __forceinline__ int pmod(int a, int m) {
    const int r = a % m;
    return r < 0 ? r + m : r;
}

template <int BX, int A, int TY, int TZ> struct SmacCfg {
    static constexpr int NSEG = BX / A;
    static constexpr int NT = NSEG * TY * TZ;
    static constexpr int KW = 2 * BX - 1;
    static constexpr int SY = TY + 1, SZ = TZ + 1;
    static constexpr int PLANE = (TY > TZ ? TY : TZ) * KW;    // max elements of a plane / layer
    static constexpr int PER = (PLANE + NT - 1) / NT;          // per-lane prefetch slots
};

template <int BX, int A, int TY, int TZ, typename R, bool SPARSE, int NC>
__device__ __forceinline__ void smac_body(const SmacGeom &g, const cplx<R> *__restrict__ Fhat,
                                          cplx<R> *__restrict__ Uhat, const cplx<R> *__restrict__ Ktab,
                                          const SmacRow *__restrict__ rows, const SmacTile *__restrict__ tiles, int64_t wg) {
    using C = SmacCfg<BX, A, TY, TZ>;
    constexpr int KW = C::KW, SY = C::SY, SZ = C::SZ, NT = C::NT;
    __shared__ cplx<R> kbuf[SY * SZ * KW];
    __shared__ cplx<R> frow[2][NC][BX];

    // the tiles of one frequency are consecutive work items, and consecutive
    // frequencies form groups of four whose reflected offsets read the same
    // spectra-table rows: both then meet in the L2 of one XCD
    const int freq = g.perm[wg / g.n_tiles];
    const int tile = (int)(wg % g.n_tiles);
    const SmacTile tl = tiles[tile];
    const int ty0 = tl.ty0, tz0 = tl.tz0;
    const int l = threadIdx.x;
    // lanes past n_lanes only help with the cooperative loads
    const bool active = l < tl.n_lanes;
    // a wave without targets (lanes are packed from 0) only helps with the
    // cooperative loads and skips the arithmetic (uniform per wave)
    const bool wave_busy = (l & ~63) < tl.n_lanes;
    const int code = active ? g.lanes[tl.lane_off + l] : 0;
    const int seg = code & 255, tyl = (code >> 8) & 255, tzl = code >> 16;
    const int ty = ty0 + tyl, tz = tz0 + tzl;
    const int x0 = seg * A;

    const size_t kper = (size_t)g.XD * g.YD * g.ZD;
    const cplx<R> *Ff = Fhat + (size_t)freq * g.n_slots;
    // frequency rows reached by reflections (flip ky, flip kz): element
    // offsets into the table, selected arithmetically so that no array of
    // pointers lands in private memory
    const int H = g.N / 2 + 1;
    const int kx = freq % H, ky = (freq / H) % g.N, kz = freq / (H * g.N);
    const int kyr = (g.N - ky) % g.N, kzr = (g.N - kz) % g.N;
    auto frow_off = [&](int fy, int fz) -> size_t {
        return ((size_t)((fz ? kzr : kz) * g.N + (fy ? kyr : ky)) * H + kx) * kper;
    };
    // raw table value for the offset (dx, dy, dz) = (dxi - (BX - 1) + dox,
    // dy, dz) in the kernel's frame (x along the rows); g.axis = 1 runs the
    // rows along the lattice y axis, i.e. the lattice offset is (dy, dx, dz).
    // A negative lattice x offset also needs the conjugate, applied by kfix.
    const int dox = g.tx0 - g.sx0;   // x offset between the target and source segments
    auto kraw = [&](int dy, int dz, int dxi) -> cplx<R> {
        const int dx = dxi - (BX - 1) + dox;
        const int px = g.axis ? dy : dx, py = g.axis ? dx : dy;
        const bool fx = px < 0;
        const int fy = (py < 0) != fx, fz = (dz < 0) != fx;
        return Ktab[frow_off(fy, fz) + ((size_t)abs(py) * g.ZD + abs(dz)) * g.XD + abs(px)];
    };
    auto kfix = [&](cplx<R> v, int dy, int dxi) -> cplx<R> {
        const int dx = dxi - (BX - 1) + dox;
        if ((g.axis ? dy : dx) < 0) v.y = -v.y;
        return v;
    };
    auto kload = [&](int dy, int dz, int dxi) -> cplx<R> { return kfix(kraw(dy, dz, dxi), dy, dxi); };
    auto lds = [&](int dy, int dz, int dxi) -> int { return (pmod(dy, SY) * SZ + pmod(dz, SZ)) * KW + dxi; };

    // NC right-hand sides (components) share every kernel row
    cplx<R> acc[NC][A];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int i = 0; i < A; ++i) acc[c][i] = cmake<R>((R)0, (R)0);

    // full window load for row 0
    int sy = rows[0].y, sz = rows[0].z;
    unsigned msk = rows[0].mask;
    {
        const int dy0 = ty0 - sy, dz0 = tz0 - sz;
        for (int e = l; e < TY * TZ * KW; e += NT) {
            const int dxi = e % KW, q = e / KW;
            const int dy = dy0 + q % TY, dz = dz0 + q / TY;
            kbuf[lds(dy, dz, dxi)] = kload(dy, dz, dxi);
        }
        for (int e = l; e < NC * BX; e += NT)
            frow[0][e / BX][e % BX] = Ff[(size_t)(e / BX) * g.fstride + ((size_t)sz * g.ey + sy) * g.rs + g.sx0 + e % BX];
    }
    __syncthreads();

    for (int ri = 0; ri < g.n_rows; ++ri) {
        const int buf = ri & 1;
        int nsy = sy, nsz = sz;
        unsigned nmsk = 0;
        int kind = 0;   // 0: none, 1: plane (new dy), 2: layer (new dz), 3: full reload
        int ndy = 0, ndz = 0;
        if (ri + 1 < g.n_rows) {
            nsy = rows[ri + 1].y;
            nsz = rows[ri + 1].z;
            nmsk = rows[ri + 1].mask;
            const int ddy = nsy - sy, ddz = nsz - sz;
            if (ddz == 0 && (ddy == 1 || ddy == -1)) {
                kind = 1;
                ndy = (ddy == 1) ? ty0 - nsy : ty0 - nsy + TY - 1;
            } else if (ddy == 0 && (ddz == 1 || ddz == -1)) {
                kind = 2;
                ndz = (ddz == 1) ? tz0 - nsz : tz0 - nsz + TZ - 1;
            } else {
                kind = 3;
            }
        }
        // prefetch the new plane / layer and the next F row into registers
        cplx<R> pre[C::PER];
        cplx<R> fpre = cmake<R>((R)0, (R)0);
        if (kind == 1 || kind == 2) {
            const int cnt = (kind == 1 ? TZ : TY) * KW;
#pragma unroll
            for (int p = 0; p < C::PER; ++p) {
                const int e = l + p * NT;
                if (e < cnt) {
                    const int dxi = e % KW, q = e / KW;
                    const int dy = (kind == 1) ? ndy : (ty0 - nsy + q);
                    const int dz = (kind == 1) ? (tz0 - nsz + q) : ndz;
                    pre[p] = kraw(dy, dz, dxi);
                }
            }
            if (l < NC * BX) fpre = Ff[(size_t)(l / BX) * g.fstride + ((size_t)nsz * g.ey + nsy) * g.rs + g.sx0 + l % BX];
        }

        // compute: U[i] += K[x0 + i - j] * F[j], with a sliding register
        // window kw[i] = K[x0 + i - j] that gains one LDS value per step j;
        // the LDS reads of step j + 2 are issued at step j, so the reads of
        // all waves spread over the row instead of bunching after the barrier
        if (wave_busy) {
            const cplx<R> *krow = &kbuf[lds(ty - sy, tz - sz, 0)] + x0 + BX - 1;
            // a per-lane base register for the broadcast F row, so that its
            // sixteen reads use immediate offsets from one address
            int vzero;
            asm volatile("v_mov_b32 %0, 0" : "=v"(vzero));
            const cplx<R> *fr = &frow[buf][0][0] + vzero;
            cplx<R> kw[A];
#pragma unroll
            for (int i = 0; i < A; ++i) kw[i] = krow[i];
            cplx<R> fj[NC], fn1[NC], fn2[NC];
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                fj[c] = fr[c * BX];
                fn1[c] = fr[c * BX + 1];
                fn2[c] = fn1[c];
            }
            cplx<R> kn1 = krow[-1];
            cplx<R> kn2 = kn1;
#pragma unroll
            for (int j = 0; j < BX; ++j) {
                if (j + 2 < BX) {
                    kn2 = krow[-(j + 2)];
#pragma unroll
                    for (int c = 0; c < NC; ++c) fn2[c] = fr[c * BX + j + 2];
                }
                // on sparse rows a source position without a block is
                // skipped (uniform branch; dense rows take no branch)
                if (!SPARSE || ((msk >> j) & 1u)) {
#pragma unroll
                    for (int c = 0; c < NC; ++c)
#pragma unroll
                        for (int i = 0; i < A; ++i) acc[c][i] = cmac(acc[c][i], kw[i], fj[c]);
                }
                if (j + 1 < BX) {
#pragma unroll
                    for (int i = A - 1; i >= 1; --i) kw[i] = kw[i - 1];
                    kw[0] = kn1;
                    kn1 = kn2;
#pragma unroll
                    for (int c = 0; c < NC; ++c) {
                        fj[c] = fn1[c];
                        fn1[c] = fn2[c];
                    }
                }
                // keep each step's products here (IR passes would otherwise
                // sink them below the prefetch stores)
#pragma unroll
                for (int c = 0; c < NC; ++c)
#pragma unroll
                    for (int i = 0; i < A; ++i) asm volatile("" : "+v"(acc[c][i].x), "+v"(acc[c][i].y)::"memory");
            }
        }

        if (kind == 1 || kind == 2) {
            const int cnt = (kind == 1 ? TZ : TY) * KW;
#pragma unroll
            for (int p = 0; p < C::PER; ++p) {
                const int e = l + p * NT;
                if (e < cnt) {
                    const int dxi = e % KW, q = e / KW;
                    const int dy = (kind == 1) ? ndy : (ty0 - nsy + q);
                    const int dz = (kind == 1) ? (tz0 - nsz + q) : ndz;
                    kbuf[lds(dy, dz, dxi)] = kfix(pre[p], dy, dxi);
                }
            }
            if (l < NC * BX) frow[buf ^ 1][l / BX][l % BX] = fpre;
            __syncthreads();
        } else if (kind == 3) {
            __syncthreads();
            const int dy0 = ty0 - nsy, dz0 = tz0 - nsz;
            for (int e = l; e < TY * TZ * KW; e += NT) {
                const int dxi = e % KW, q = e / KW;
                const int dy = dy0 + q % TY, dz = dz0 + q / TY;
                kbuf[lds(dy, dz, dxi)] = kload(dy, dz, dxi);
            }
            for (int e = l; e < NC * BX; e += NT)
                frow[buf ^ 1][e / BX][e % BX] =
                    Ff[(size_t)(e / BX) * g.fstride + ((size_t)nsz * g.ey + nsy) * g.rs + g.sx0 + e % BX];
            __syncthreads();
        }
        sy = nsy;
        sz = nsz;
        msk = nmsk;
    }

    if (active) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            cplx<R> *Uf = Uhat + (size_t)c * g.fstride + (size_t)freq * g.n_slots + ((size_t)tz * g.ey + ty) * g.rs +
                          g.tx0 + x0;
            if (g.accum) {
#pragma unroll
                for (int i = 0; i < A; ++i) Uf[i] = cmake<R>(Uf[i].x + acc[c][i].x, Uf[i].y + acc[c][i].y);
            } else {
#pragma unroll
                for (int i = 0; i < A; ++i) Uf[i] = acc[c][i];
            }
        }
    }
}

template <int BX, int A, int TY, int TZ, typename R, bool SPARSE, int NC>
__global__ void __launch_bounds__((BX / A) * TY * TZ)
    smac_kernel(SmacGeom g, const cplx<R> *__restrict__ Fhat, cplx<R> *__restrict__ Uhat,
                const cplx<R> *__restrict__ Ktab, const SmacRow *__restrict__ rows, const SmacTile *__restrict__ tiles) {
    smac_body<BX, A, TY, TZ, R, SPARSE, NC>(g, Fhat, Uhat, Ktab, rows, tiles, xcd_order(blockIdx.x, gridDim.x));
}

// Several independent convolutions of one template in one grid: workgroup w
// belongs to the job with wg_begin <= w < next job's wg_begin.
template <int BX, int A, int TY, int TZ, typename R, bool SPARSE>
__global__ void __launch_bounds__((BX / A) * TY * TZ) smac_batch_kernel(const SmacJob *__restrict__ jobs, int n_jobs) {
    const int64_t w = xcd_order(blockIdx.x, gridDim.x);
    int lo = 0, hi = n_jobs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) / 2;
        if (jobs[mid].wg_begin <= w) lo = mid;
        else hi = mid - 1;
    }
    const SmacJob &j = jobs[lo];
    smac_body<BX, A, TY, TZ, R, SPARSE, 1>(j.g, (const cplx<R> *)j.F, (cplx<R> *)j.U, (const cplx<R> *)j.K, j.rows,
                                           j.tiles, w - j.wg_begin);
}

template <int BX, int A, int TY, int TZ, typename R, bool SPARSE, int NC>
hipError_t launch_cfg(const SmacGeom &g, const void *F, void *U, const void *K, const SmacRow *rows,
                      const SmacTile *tiles, hipStream_t s) {
    using C = SmacCfg<BX, A, TY, TZ>;
    if (g.n_rows <= 0 || g.n_tiles <= 0) return hipSuccess;
    const int64_t nwg = (int64_t)g.n_freq * g.n_tiles;
    hipLaunchKernelGGL((smac_kernel<BX, A, TY, TZ, R, SPARSE, NC>), dim3((unsigned)nwg), dim3(C::NT), 0, s, g,
                       (const cplx<R> *)F, (cplx<R> *)U, (const cplx<R> *)K, rows, tiles);
    return hipGetLastError();
}

template <int BX, int A, int TY, int TZ, typename R, bool SPARSE>
hipError_t launch_batch_cfg(const SmacJob *jobs, int n_jobs, int64_t total_wg, hipStream_t s) {
    using C = SmacCfg<BX, A, TY, TZ>;
    if (n_jobs <= 0 || total_wg <= 0) return hipSuccess;
    hipLaunchKernelGGL((smac_batch_kernel<BX, A, TY, TZ, R, SPARSE>), dim3((unsigned)total_wg), dim3(C::NT), 0, s,
                       jobs, n_jobs);
    return hipGetLastError();
}

// Templates (bx, A, TY, TZ): bx = 8 with 8 x 8 tiles; bx = 16 with 16 x 8
// (the default), 8 x 8 or 16 x 16 tiles (longer rows are cut into 16-wide
// segments by the runtime).  A = 8 targets per lane throughout.
template <typename F> hipError_t dispatch(int bx, int ty, int tz, bool fp32, bool sparse, const F &f) {
    auto pick = [&](auto bxc, auto tyc, auto tzc) -> hipError_t {
        constexpr int BX = decltype(bxc)::value, A = 8, TY = decltype(tyc)::value, TZ = decltype(tzc)::value;
        if (fp32)
            return sparse ? f.template operator()<BX, A, TY, TZ, float, true>()
                          : f.template operator()<BX, A, TY, TZ, float, false>();
        return sparse ? f.template operator()<BX, A, TY, TZ, double, true>()
                      : f.template operator()<BX, A, TY, TZ, double, false>();
    };
    using I8 = std::integral_constant<int, 8>;
    using I16 = std::integral_constant<int, 16>;
    if (bx == 8 && ty == 8 && tz == 8) return pick(I8{}, I8{}, I8{});
    if (bx == 16 && ty == 16 && tz == 8) return pick(I16{}, I16{}, I8{});
    if (bx == 16 && ty == 8 && tz == 8) return pick(I16{}, I8{}, I8{});
    if (bx == 16 && ty == 16 && tz == 16) return pick(I16{}, I16{}, I16{});
    return hipErrorInvalidValue;
}

struct BatchLaunch {
    const SmacJob *jobs;
    int n_jobs;
    int64_t total_wg;
    hipStream_t s;
    template <int BX, int A, int TY, int TZ, typename R, bool SP> hipError_t operator()() const {
        return launch_batch_cfg<BX, A, TY, TZ, R, SP>(jobs, n_jobs, total_wg, s);
    }
};

struct SingleLaunch {
    const SmacGeom &g;
    const void *F;
    void *U;
    const void *K;
    const SmacRow *rows;
    const SmacTile *tiles;
    int nc;
    hipStream_t s;
    template <int BX, int A, int TY, int TZ, typename R, bool SP> hipError_t operator()() const {
        switch (nc) {
        case 1: return launch_cfg<BX, A, TY, TZ, R, SP, 1>(g, F, U, K, rows, tiles, s);
        case 2: return launch_cfg<BX, A, TY, TZ, R, SP, 2>(g, F, U, K, rows, tiles, s);
        case 3: return launch_cfg<BX, A, TY, TZ, R, SP, 3>(g, F, U, K, rows, tiles, s);
        default: return hipErrorInvalidValue;
        }
    }
};

}  // namespace

hipError_t smac_batch_launch(int bx, int ty, int tz, bool fp32, bool sparse, const SmacJob *jobs, int n_jobs,
                             int64_t total_wg, hipStream_t s) {
    return dispatch(bx, ty, tz, fp32, sparse, BatchLaunch{jobs, n_jobs, total_wg, s});
}

int smac_seg_len(int bx) {
    (void)bx;
    return 8;
}

int smac_tiles(int bx, int (*tiles)[2], int max_tiles) {
    static const int t8[][2] = {{8, 8}};
    static const int t16[][2] = {{16, 8}, {8, 8}, {16, 16}};
    const int(*t)[2] = bx == 8 ? t8 : t16;
    const int n = bx == 8 ? 1 : 3;
    for (int i = 0; i < n && i < max_tiles; ++i) {
        tiles[i][0] = t[i][0];
        tiles[i][1] = t[i][1];
    }
    return n;
}

hipError_t smac_launch(const SmacGeom &g, bool fp32, bool sparse, int nc, const void *Fhat, void *Uhat,
                       const void *Ktab, const SmacRow *rows, const SmacTile *tiles, hipStream_t s) {
    return dispatch(g.bx, g.ty, g.tz, fp32, sparse, SingleLaunch{g, Fhat, Uhat, Ktab, rows, tiles, nc, s});
}

}  // namespace lgf
