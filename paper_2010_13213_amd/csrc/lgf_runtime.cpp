// Native runtime behind the C ABI of include/lgf.h: contexts (device LGF
// table, spectra cache, HBM budget), plans (validated block lists, level
// schedule, slot maps, work lists, workspaces) and the solve pipeline.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <stdexcept>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lgf.h"
#include "lgf_device.hpp"
#include "lgf_kernels.hpp"
#include "lgf_runtime.hpp"

namespace lgf {

thread_local std::string g_last_error;
thread_local bool g_no_timing = false;

void set_error(const std::string &m) { g_last_error = m; }

Failure::Failure(lgf_status s, const std::string &m) : std::runtime_error(m), status(s) {}

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) throw Failure(LGF_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// ------------------------------------------------------------------ memory

DeviceBuffer::~DeviceBuffer() { release(); }

void DeviceBuffer::release() {
    if (ptr) {
        (void)hipFree(ptr);
        if (owner) owner->used -= bytes;
    }
    ptr = nullptr;
    bytes = 0;
}

void DeviceBuffer::alloc(lgf_context *ctx, size_t n, const char *what) {
    release();
    if (n == 0) return;
    if (ctx->budget && ctx->used + n > ctx->budget)
        throw Failure(LGF_E_NOMEM, std::string("HBM budget exceeded allocating ") + what);
    hipError_t e = hipMalloc(&ptr, n);
    if (e != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        throw Failure(LGF_E_NOMEM, std::string("hipMalloc failed for ") + what);
    }
    bytes = n;
    owner = ctx;
    ctx->used += n;
}

// ------------------------------------------------------------------ timing

StageTimer::StageTimer(lgf_context *c, int st, hipStream_t s_) : ctx(c), stage(st), s(s_) {
    if (!ctx->timing || g_no_timing) return;
    hip_check(hipEventCreate(&a), "event");
    hip_check(hipEventRecord(a, s), "event record");
}

StageTimer::~StageTimer() {
    if (!a) return;
    hipEvent_t b = nullptr;
    if (hipEventCreate(&b) == hipSuccess && hipEventRecord(b, s) == hipSuccess) {
        ctx->pending.push_back(StageEvent{stage, a, b});
    } else {
        (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
}

void resolve_stage_times(lgf_context *ctx, double *ms, int64_t *launches) {
    for (int i = 0; i < kStages; ++i) {
        ms[i] = 0.0;
        launches[i] = 0;
    }
    for (auto &e : ctx->pending) {
        hip_check(hipEventSynchronize(e.b), "event sync");
        float t = 0.f;
        hip_check(hipEventElapsedTime(&t, e.a, e.b), "elapsed");
        ms[e.stage] += t;
        launches[e.stage] += 1;
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    ctx->pending.clear();
}

// ------------------------------------------------------------------ job ring

void ring_init(lgf_context *ctx) {
    JobRing &r = ctx->ring;
    const size_t n = JobRing::kSlots * JobRing::kSlotBytes;
    hip_check(hipHostMalloc(&r.host, n, hipHostMallocDefault), "hipHostMalloc job ring");
    hip_check(hipMalloc(&r.dev, n), "hipMalloc job ring");
    for (int i = 0; i < JobRing::kSlots; ++i)
        hip_check(hipEventCreateWithFlags(&r.done[i], hipEventDisableTiming), "ring event");
}

void ring_free(lgf_context *ctx) {
    JobRing &r = ctx->ring;
    for (int i = 0; i < JobRing::kSlots; ++i)
        if (r.done[i]) {
            (void)hipEventSynchronize(r.done[i]);
            (void)hipEventDestroy(r.done[i]);
            r.done[i] = nullptr;
        }
    if (r.host) (void)hipHostFree(r.host);
    if (r.dev) (void)hipFree(r.dev);
    r.host = r.dev = nullptr;
}

// ------------------------------------------------------------------ context

lgf_context_impl::lgf_context_impl(int dev, size_t budget_) : device(dev), budget(budget_) {}

void build_context_table(lgf_context *ctx) {
    const int S = kTableRadius + 1;
    ctx->gcube.alloc(ctx, sizeof(double) * (size_t)S * S * S, "LGF table");
    DeviceBuffer B, w;
    const int nodes = lgf_table_nodes();
    B.alloc(ctx, sizeof(double) * (size_t)nodes * S, "Bessel rows");
    w.alloc(ctx, sizeof(double) * nodes, "quadrature weights");
    hip_check(build_lgf_table((double *)ctx->gcube.ptr, (double *)B.ptr, (double *)w.ptr, ctx->stream),
              "build_lgf_table");
    hip_check(hipStreamSynchronize(ctx->stream), "table sync");
}

// The integrating-factor kernel cube for a (caller holds ctx->mu).
static const double *if_cube(lgf_context *ctx, double a) {
    auto it = ctx->if_cubes.find(a);
    if (it != ctx->if_cubes.end()) return (const double *)it->second->ptr;
    const int S = kTableRadius + 1;
    auto cube = std::make_unique<DeviceBuffer>();
    cube->alloc(ctx, sizeof(double) * (size_t)S * S * S, "integrating-factor table");
    DeviceBuffer row, w;
    row.alloc(ctx, sizeof(double) * S, "Bessel row");
    w.alloc(ctx, sizeof(double), "quadrature weight");
    hip_check(build_if_table((double *)cube->ptr, (double *)row.ptr, (double *)w.ptr, a, ctx->stream),
              "build_if_table");
    hip_check(hipStreamSynchronize(ctx->stream), "if table sync");
    const double *p = (const double *)cube->ptr;
    ctx->if_cubes[a] = std::move(cube);
    return p;
}

SpecTable *get_spectra(lgf_context *ctx, int nb, bool fp32, int XH, int YH, int ZH, const KernelId &ka) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto &t : ctx->tables)
        if (t->nb == nb && t->fp32 == fp32 && t->ka == ka && t->XH >= XH && t->YH >= YH && t->ZH >= ZH)
            return t.get();
    auto t = std::make_unique<SpecTable>();
    t->nb = nb;
    t->fp32 = fp32;
    t->ka = ka;
    t->XH = XH;
    t->YH = YH;
    t->ZH = ZH;
    const int N = 2 * nb;
    t->n_freq = N * N * (nb + 1);
    const size_t n_off = (size_t)(XH + 1) * (YH + 1) * (ZH + 1);
    const size_t elem = fp32 ? 8 : 16;
    t->data.alloc(ctx, elem * n_off * t->n_freq, "LGF block spectra");
    DeviceBuffer scratch;
    const size_t per_off = (size_t)t->n_freq * 16;
    const size_t want = std::min<size_t>(n_off, 2048) * per_off;
    scratch.alloc(ctx, want, "spectra scratch");
    const double *kern = ka.a > 0.0 ? if_cube(ctx, ka.a) : (const double *)ctx->gcube.ptr;
    hip_check(build_spectra(kern, ka.a <= 0.0, ka.stride, ka.band, ka.D, nb, XH, YH, ZH, fp32, t->data.ptr,
                            scratch.ptr, scratch.bytes, ctx->stream),
              "build_spectra");
    hip_check(hipStreamSynchronize(ctx->stream), "spectra sync");
    {
        // omega = (kz N + ky) H + kx; its partners (kx, -ky, kz), (kx, ky, -kz),
        // (kx, -ky, -kz) read the same octant rows of the table
        const int H = nb + 1;
        std::vector<int> perm;
        std::vector<char> seen(t->n_freq, 0);
        for (int w = 0; w < t->n_freq; ++w) {
            if (seen[w]) continue;
            const int kx = w % H, ky = (w / H) % N, kz = w / (H * N);
            const int kys[2] = {ky, (N - ky) % N}, kzs[2] = {kz, (N - kz) % N};
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    const int v = (kzs[b] * N + kys[a]) * H + kx;
                    if (!seen[v]) {
                        seen[v] = 1;
                        perm.push_back(v);
                    }
                }
        }
        t->perm.alloc(ctx, sizeof(int) * perm.size(), "frequency order");
        hip_check(hipMemcpy(t->perm.ptr, perm.data(), sizeof(int) * perm.size(), hipMemcpyHostToDevice),
                  "upload frequency order");
    }
    ctx->tables.push_back(std::move(t));
    return ctx->tables.back().get();
}

LatSpec *get_lat_spectra(lgf_context *ctx, int nb, bool fp32, int lx, int ly, int lz, const KernelId &ka) {
    auto find = [&]() -> LatSpec * {
        for (auto &t : ctx->lat_tables)
            if (t->nb == nb && t->fp32 == fp32 && t->ka == ka && t->lx == lx && t->ly == ly && t->lz == lz)
                return t.get();
        return nullptr;
    };
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        if (LatSpec *t = find()) return t;
    }
    // offsets up to L/2 - 1 per axis
    SpecTable *oct = get_spectra(ctx, nb, fp32, lx / 2 - 1, ly / 2 - 1, lz / 2 - 1, ka);
    auto t = std::make_unique<LatSpec>();
    t->nb = nb;
    t->fp32 = fp32;
    t->ka = ka;
    t->lx = lx;
    t->ly = ly;
    t->lz = lz;
    t->n_freq = oct->n_freq;
    {
        // the octant table's frequency order (reflection partners adjacent)
        // as positions of the block-major spectra
        const int N = 2 * nb, Hh = nb + 1;
        std::vector<int> perm(t->n_freq), pos(t->n_freq);
        hip_check(hipMemcpy(perm.data(), oct->perm.ptr, sizeof(int) * perm.size(), hipMemcpyDeviceToHost),
                  "read frequency order");
        for (int i = 0; i < t->n_freq; ++i) {
            const int w = perm[i];
            pos[i] = spec_pos(N, w % Hh, (w / Hh) % N, w / (Hh * N));
        }
        t->order_buf.alloc(ctx, sizeof(int) * pos.size(), "lattice frequency order");
        hip_check(hipMemcpy(t->order_buf.ptr, pos.data(), sizeof(int) * pos.size(), hipMemcpyHostToDevice),
                  "upload lattice frequency order");
        t->order = (const int *)t->order_buf.ptr;
    }
    const size_t per_w = (size_t)lx * ly * lz;
    const size_t n_stored = (size_t)lattice_stored_freqs(2 * nb);
    t->data.alloc(ctx, (fp32 ? 4 : 8) * per_w * n_stored, "lattice spectra");
    const size_t ec = fp32 ? 8 : 16;
    const size_t chunk = std::max<size_t>(1, std::min<size_t>(n_stored, (size_t(256) << 20) / (ec * per_w)));
    DeviceBuffer scratch;
    scratch.alloc(ctx, chunk * per_w * ec, "lattice spectra scratch");
    LatSpecGeom sg{2 * nb, lx, ly, lz, oct->XH + 1, oct->YH + 1, oct->ZH + 1};
    hip_check(lattice_spectra(sg, fp32, oct->data.ptr, t->data.ptr, scratch.ptr, scratch.bytes, ctx->stream),
              "lattice spectra");
    hip_check(hipStreamSynchronize(ctx->stream), "lattice spectra sync");
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (LatSpec *other = find()) return other;   // built meanwhile by another thread
    ctx->lat_tables.push_back(std::move(t));
    return ctx->lat_tables.back().get();
}

// ------------------------------------------------------------------ plan

static int roundup(int a, int m) { return (a + m - 1) / m * m; }

static void upload_slots(lgf_context *ctx, Conv &c, const std::vector<int> &s_slot, const std::vector<int> &t_slot,
                         const std::vector<int64_t> &s_off, const std::vector<int64_t> &t_off) {
    auto up = [&](DeviceBuffer &d, const void *h, size_t n) {
        if (n) hip_check(hipMemcpy(d.ptr, h, n, hipMemcpyHostToDevice), "upload");
    };
    c.d_src_slot.alloc(ctx, sizeof(int) * std::max<size_t>(1, s_slot.size()), "slots");
    c.d_tgt_slot.alloc(ctx, sizeof(int) * std::max<size_t>(1, t_slot.size()), "slots");
    c.d_src_off.alloc(ctx, sizeof(int64_t) * std::max<size_t>(1, s_off.size()), "offsets");
    c.d_tgt_off.alloc(ctx, sizeof(int64_t) * std::max<size_t>(1, t_off.size()), "offsets");
    up(c.d_src_slot, s_slot.data(), sizeof(int) * s_slot.size());
    up(c.d_tgt_slot, t_slot.data(), sizeof(int) * t_slot.size());
    up(c.d_src_off, s_off.data(), sizeof(int64_t) * s_off.size());
    up(c.d_tgt_off, t_off.data(), sizeof(int64_t) * t_off.size());
}

// Extents in blocks of the bounding box of src and tgt.
static void box_extent(const std::vector<Blk> &src, const std::vector<Blk> &tgt, int lo[3], int ext[3]) {
    int hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (int a = 0; a < 3; ++a) lo[a] = INT32_MAX;
    for (const auto *v : {&src, &tgt})
        for (const auto &b : *v)
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], b.ijk[a]);
                hi[a] = std::max(hi[a], b.ijk[a]);
            }
    for (int a = 0; a < 3; ++a) ext[a] = hi[a] - lo[a] + 1;
}

// The lattice method needs a compiled DFT length of at least 2E - 1 per axis.
static bool lattice_feasible(const std::vector<Blk> &src, const std::vector<Blk> &tgt) {
    if (src.empty() || tgt.empty()) return false;
    int lo[3], ext[3];
    box_extent(src, tgt, lo, ext);
    return lattice_len_ok(lattice_len(ext[0])) && lattice_len_ok(lattice_len(ext[1])) &&
           lattice_zlen_ok(lattice_len(ext[2]));
}

// Under an HBM budget the lattice is a candidate only if the spectra it
// would build still fit (the block-pair spectra of the same box are far
// smaller); spectra already in the context cost nothing.
static bool lattice_fits_budget(lgf_plan *plan, const std::vector<Blk> &src, const std::vector<Blk> &tgt,
                                bool fp32) {
    lgf_context *ctx = plan->ctx;
    if (!ctx->budget) return true;
    int lo[3], ext[3];
    box_extent(src, tgt, lo, ext);
    const int lx = lattice_len(ext[0]), ly = lattice_len(ext[1]), lz = lattice_len(ext[2]);
    std::lock_guard<std::mutex> lk(ctx->mu);
    for (auto &t : ctx->lat_tables)
        if (t->nb == plan->nb && t->fp32 == fp32 && t->ka == plan->build_ka && t->lx == lx && t->ly == ly &&
            t->lz == lz)
            return true;
    const size_t n_freq = (size_t)(2 * plan->nb) * (2 * plan->nb) * (plan->nb + 1);
    const size_t per_w = (size_t)lx * ly * lz;
    size_t need = (fp32 ? 4 : 8) * per_w * (size_t)lattice_stored_freqs(2 * plan->nb) +
                  std::min<size_t>(size_t(256) << 20, (fp32 ? 8 : 16) * per_w * n_freq);
    need += (fp32 ? 8 : 16) * (size_t)(lx / 2) * (ly / 2) * (lz / 2) * n_freq + 2048 * n_freq * 16;
    return ctx->used + need <= ctx->budget;
}

// A convolution whose MAC is the lattice FFT: slots over the tight bounding
// box, spectra for its DFT lengths.
static void build_conv_lattice(lgf_plan *plan, Conv &c, const std::vector<Blk> &src, const std::vector<Blk> &tgt,
                               bool fp32) {
    lgf_context *ctx = plan->ctx;
    int lo[3], ext[3];
    box_extent(src, tgt, lo, ext);
    c.method = kMethodLattice;
    c.axis = 0;
    c.bx = c.ty = c.tz = 0;
    c.rs = ext[0];
    c.ey = ext[1];
    c.ez = ext[2];
    for (int a = 0; a < 3; ++a) c.lo[a] = lo[a];
    c.lx = lattice_len(ext[0]);
    c.ly = lattice_len(ext[1]);
    c.lz = lattice_len(ext[2]);
    c.n_slots = (int64_t)ext[0] * ext[1] * ext[2];
    c.fp32 = fp32;
    c.n_src = (int)src.size();
    c.n_tgt = (int)tgt.size();
    c.lspec = get_lat_spectra(ctx, plan->nb, fp32, c.lx, c.ly, c.lz, plan->build_ka);
    c.spec = get_spectra(ctx, plan->nb, fp32, c.lx / 2 - 1, c.ly / 2 - 1, c.lz / 2 - 1, plan->build_ka);
    std::vector<int> s_slot, t_slot;
    std::vector<int64_t> s_off, t_off;
    auto slot_of = [&](const Blk &b) {
        return ((b.ijk[2] - lo[2]) * ext[1] + (b.ijk[1] - lo[1])) * ext[0] + (b.ijk[0] - lo[0]);
    };
    for (const auto &b : src) {
        s_slot.push_back(slot_of(b));
        s_off.push_back(b.off);
    }
    for (const auto &b : tgt) {
        t_slot.push_back(slot_of(b));
        t_off.push_back(b.off);
    }
    upload_slots(ctx, c, s_slot, t_slot, s_off, t_off);
    if ((int64_t)src.size() != c.n_slots) {
        std::vector<unsigned char> occ((size_t)c.n_slots, 0);
        for (int sl : s_slot) occ[(size_t)sl] = 1;
        c.d_src_occ.alloc(ctx, occ.size(), "source slots");
        hip_check(hipMemcpy(c.d_src_occ.ptr, occ.data(), occ.size(), hipMemcpyHostToDevice), "upload source slots");
    }
    c.lat_fused = ctx->lat_passes == 1 && lattice_fused_ok(lat_geom(c, 1));
}

const void *lattice_mac(lgf_context *ctx, const Conv &c, const LatGeom &g, const void *fhat, void *lat, void *uhat,
                        hipStream_t s) {
    if (c.lat_fused) {
        StageTimer t(ctx, kStageLatFused, s);
        hip_check(lattice_fused(g, c.fp32, fhat, c.lspec->data.ptr, uhat, lat, s),
                  "one-pass lattice MAC");
        return lat;
    }
    {
        StageTimer t(ctx, kStageLatX, s);
        hip_check(lattice_fwd(g, c.fp32, fhat, lat, s), "lattice x DFT");
    }
    {
        StageTimer t(ctx, kStageLatYZ, s);
        hip_check(lattice_yz(g, c.fp32, lat, c.lspec->data.ptr, c.lspec->order, s), "lattice y/z slabs");
    }
    StageTimer t(ctx, kStageLatInv, s);
    hip_check(lattice_inv(g, c.fp32, lat, uhat, s), "lattice inverse x DFT");
    return nullptr;
}

LatGeom lat_geom(const Conv &c, int nc) {
    LatGeom g;
    g.ex = c.rs;
    g.ey = c.ey;
    g.ez = c.ez;
    g.lx = c.lx;
    g.ly = c.ly;
    g.lz = c.lz;
    g.nc = nc;
    g.N = 2 * c.spec->nb;
    g.n_freq = c.spec->n_freq;
    g.n_slots = c.n_slots;
    g.fstride = (int64_t)c.spec->n_freq * c.n_slots;
    // slabs of a multiple of 32 elements are padded by 8 (one 128-byte line
    // in float64): unpadded, the lx slabs a lattice x line touches are a
    // power-of-two stride apart
    const int per_w = c.ey * c.ez;
    g.hslab = per_w % 32 == 0 ? per_w + 8 : per_w;
    g.hstride = (int64_t)c.spec->n_freq * c.lx * g.hslab;
    g.occ = (const unsigned char *)c.d_src_occ.ptr;
    return g;
}

// Build a convolution: sources `src` and targets `tgt` (block coords of one
// level), field offsets (in elements, per component) of each block.
//
// Rows longer than 16 blocks are cut into 16-wide x-segments; every pair
// (target segment, source segment) with targets and sources is one part,
// run by the 16-wide MAC template.  Part (ts, ss) runs in phase
// (ss - ts) mod n_seg, so the parts of one target segment never run in the
// same launch; the first of them stores into Uhat, later ones add.  Empty
// source segments of a row and empty target segments of a tile cost nothing.
static void build_conv_tile(lgf_plan *plan, Conv &c, const std::vector<Blk> &src, const std::vector<Blk> &tgt,
                            bool fp32, int axis, int TY, int TZ) {
    lgf_context *ctx = plan->ctx;
    const int nb = plan->nb;
    // coordinates in the MAC's frame: rows along x (axis 0) or along the
    // lattice y axis (axis 1: x and y swapped)
    c.axis = axis;
    auto P = [axis](const Blk &b, int a) -> int { return (axis == 1 && a < 2) ? b.ijk[1 - a] : b.ijk[a]; };
    int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (const auto *v : {&src, &tgt})
        for (const auto &b : *v)
            for (int a = 0; a < 3; ++a) {
                lo[a] = std::min(lo[a], P(b, a));
                hi[a] = std::max(hi[a], P(b, a));
            }
    const int ex = hi[0] - lo[0] + 1, ey = hi[1] - lo[1] + 1, ez = hi[2] - lo[2] + 1;
    if (ex > 64 || ey > 64 || ez > 64)
        throw Failure(LGF_E_UNSUPPORTED, "level extent above 64 blocks along an axis");
    const int bx = ex <= 8 ? 8 : 16;
    const int rs = roundup(ex, bx);
    const int n_seg = rs / bx;
    c.ty = TY;
    c.tz = TZ;
    c.bx = bx;
    c.rs = rs;
    c.ey = roundup(ey, TY);
    c.ez = roundup(ez, TZ);
    for (int a = 0; a < 3; ++a) c.lo[a] = lo[a];
    c.n_slots = (int64_t)rs * c.ey * c.ez;
    c.fp32 = fp32;
    auto slot_of = [&](const Blk &b) -> int {
        return ((P(b, 2) - lo[2]) * c.ey + (P(b, 1) - lo[1])) * rs + (P(b, 0) - lo[0]);
    };
    std::vector<int> s_slot, t_slot;
    std::vector<int64_t> s_off, t_off;
    // per source segment: row -> occupancy mask; per target segment: tile ->
    // occupied x-segments of A targets
    const int A = smac_seg_len(bx), NSEG = bx / A, NT = NSEG * TY * TZ;
    std::vector<std::map<std::pair<int, int>, unsigned>> rowmask(n_seg);
    std::vector<std::map<std::pair<int, int>, std::set<int>>> tileseg(n_seg);
    for (const auto &b : src) {
        s_slot.push_back(slot_of(b));
        s_off.push_back(b.off);
        const int x = P(b, 0) - lo[0];
        rowmask[x / bx][{P(b, 2) - lo[2], P(b, 1) - lo[1]}] |= 1u << (x % bx);
    }
    for (const auto &b : tgt) {
        t_slot.push_back(slot_of(b));
        t_off.push_back(b.off);
        const int y = P(b, 1) - lo[1], z = P(b, 2) - lo[2], x = P(b, 0) - lo[0];
        const int tzl = z % TZ, tyl = y % TY, seg = (x % bx) / A;
        tileseg[x / bx][{z / TZ * TZ, y / TY * TY}].insert((tzl * TY + tyl) * NSEG + seg);
    }
    auto up = [&](DeviceBuffer &d, const void *h, size_t n) {
        if (n) hip_check(hipMemcpy(d.ptr, h, n, hipMemcpyHostToDevice), "upload");
    };
    std::vector<bool> stored(n_seg, false);
    for (int ph = 0; ph < n_seg; ++ph)
        for (int ts = 0; ts < n_seg; ++ts) {
            const int ss = (ts + ph) % n_seg;
            if (rowmask[ss].empty() || tileseg[ts].empty()) continue;
            auto part = std::make_unique<SubConv>();
            part->tx0 = ts * bx;
            part->sx0 = ss * bx;
            part->phase = ph;
            part->accum = stored[ts];
            stored[ts] = true;
            // Source row order.  Consecutive rows one step apart in y or z
            // cost the MAC one new ring plane; any other step reloads the
            // whole ring.  Two orders are built and the one with fewer
            // reloads kept: the serpentine (z ascending, y alternating per z
            // group) and a greedy walk that keeps stepping to a neighbouring
            // row (same direction first) and jumps to the nearest row only
            // when it has none.
            int64_t n_src_seg = 0;
            std::vector<std::pair<int, int>> rowset;   // (y, z)
            for (auto &r : rowmask[ss]) {
                rowset.push_back({r.first.second, r.first.first});
                n_src_seg += __builtin_popcount(r.second);
            }
            auto jumps = [](const std::vector<std::pair<int, int>> &o) {
                int n = 0;
                for (size_t i = 1; i < o.size(); ++i)
                    n += std::abs(o[i].first - o[i - 1].first) + std::abs(o[i].second - o[i - 1].second) != 1;
                return n;
            };
            std::vector<std::pair<int, int>> serp;
            {
                std::map<int, std::vector<int>> byz;
                for (auto &r : rowset) byz[r.second].push_back(r.first);
                int gi = 0;
                for (auto &kv : byz) {
                    auto ys = kv.second;
                    std::sort(ys.begin(), ys.end());
                    if (gi & 1) std::reverse(ys.begin(), ys.end());
                    for (int y : ys) serp.push_back({y, kv.first});
                    ++gi;
                }
            }
            std::vector<std::pair<int, int>> walk;
            {
                std::set<std::pair<int, int>> left(rowset.begin(), rowset.end());
                std::pair<int, int> cur = serp.front(), dir = {1, 0};
                walk.push_back(cur);
                left.erase(cur);
                const std::pair<int, int> steps[4] = {{1, 0}, {-1, 0}, {0, 1}, {0, -1}};
                while (!left.empty()) {
                    std::pair<int, int> nxt{INT32_MIN, INT32_MIN};
                    const std::pair<int, int> ahead{cur.first + dir.first, cur.second + dir.second};
                    if (left.count(ahead)) nxt = ahead;
                    for (int q = 0; q < 4 && nxt.first == INT32_MIN; ++q) {
                        const std::pair<int, int> c2{cur.first + steps[q].first, cur.second + steps[q].second};
                        if (left.count(c2)) nxt = c2;
                    }
                    if (nxt.first == INT32_MIN) {   // jump to the nearest row left
                        int best = INT32_MAX;
                        for (auto &r : left) {
                            const int d = std::abs(r.first - cur.first) + std::abs(r.second - cur.second);
                            if (d < best) {
                                best = d;
                                nxt = r;
                            }
                        }
                        dir = {1, 0};
                    } else {
                        dir = {nxt.first - cur.first, nxt.second - cur.second};
                    }
                    walk.push_back(nxt);
                    left.erase(nxt);
                    cur = nxt;
                }
            }
            const auto &order = jumps(walk) < jumps(serp) ? walk : serp;
            std::vector<SmacRow> rows;
            for (auto &r : order) rows.push_back(SmacRow{r.first, r.second, rowmask[ss][{r.second, r.first}], 0});
            // lanes in (tz, ty, seg) order: a full tile gets lane l = (tzl * TY
            // + tyl) * NSEG + seg; tiles with more lanes than a workgroup split
            std::vector<SmacTile> tiles;
            std::vector<int> lanes;
            for (auto &t : tileseg[ts]) {
                std::vector<int> ls;
                for (int key : t.second) {
                    const int seg = key % NSEG, tyl = (key / NSEG) % TY, tzl = key / (NSEG * TY);
                    ls.push_back(seg | (tyl << 8) | (tzl << 16));
                }
                for (size_t i = 0; i < ls.size(); i += NT) {
                    const int n = (int)std::min<size_t>(NT, ls.size() - i);
                    tiles.push_back(SmacTile{t.first.second, t.first.first, (int)lanes.size(), n});
                    lanes.insert(lanes.end(), ls.begin() + i, ls.begin() + i + n);
                }
            }
            part->n_rows = (int)rows.size();
            part->n_tiles = (int)tiles.size();
            // skipping empty source positions costs a branch per position:
            // worth it once more than a few percent of them are empty
            part->sparse = n_src_seg * 10 < (int64_t)rows.size() * bx * 9;
            part->d_rows.alloc(ctx, sizeof(SmacRow) * std::max<size_t>(1, rows.size()), "rows");
            part->d_tiles.alloc(ctx, sizeof(SmacTile) * std::max<size_t>(1, tiles.size()), "tiles");
            part->d_lanes.alloc(ctx, sizeof(int) * std::max<size_t>(1, lanes.size()), "lanes");
            up(part->d_rows, rows.data(), sizeof(SmacRow) * rows.size());
            up(part->d_tiles, tiles.data(), sizeof(SmacTile) * tiles.size());
            up(part->d_lanes, lanes.data(), sizeof(int) * lanes.size());
            c.parts.push_back(std::move(part));
        }
    c.n_src = (int)src.size();
    c.n_tgt = (int)tgt.size();
    // the spectra table is indexed by lattice offsets
    c.spec = axis == 1 ? get_spectra(ctx, nb, fp32, c.ey - 1, rs - 1, c.ez - 1, plan->build_ka)
                       : get_spectra(ctx, nb, fp32, rs - 1, c.ey - 1, c.ez - 1, plan->build_ka);
    upload_slots(ctx, c, s_slot, t_slot, s_off, t_off);
}

// Shape key of a convolution for the tuning table.
static std::string tune_key(int nb, bool fp32, int nc, int axis, const std::vector<Blk> &src,
                            const std::vector<Blk> &tgt) {
    int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (const auto *v : {&src, &tgt})
        for (const auto &b : *v)
            for (int a = 0; a < 3; ++a) {
                const int c = (axis == 1 && a < 2) ? b.ijk[1 - a] : b.ijk[a];
                lo[a] = std::min(lo[a], c);
                hi[a] = std::max(hi[a], c);
            }
    char k[160];
    std::snprintf(k, sizeof k, "nb%d_%s_nc%d_ext%dx%dx%d_src%zu_tgt%zu", nb, fp32 ? "f32" : "f64", nc,
                  hi[0] - lo[0] + 1, hi[1] - lo[1] + 1, hi[2] - lo[2] + 1, src.size(), tgt.size());
    return k;
}

// Milliseconds per launch of the spectral MAC of c (its pair parts, or the
// lattice FFT), for the plan's components per launch, on the context
// stream, with throw-away spectral buffers.
static double time_mac(lgf_plan *plan, const Conv &c, int reps) {
    lgf_context *ctx = plan->ctx;
    const int nc = plan->mac_nc;
    const int64_t fs = (int64_t)c.spec->n_freq * c.n_slots;
    const size_t ec = c.fp32 ? 8 : 16;
    const size_t bytes = ec * (size_t)fs * nc;
    DeviceBuffer F, U, Hb;
    F.alloc(ctx, bytes, "tuning workspace");
    U.alloc(ctx, bytes, "tuning workspace");
    if (c.method == kMethodLattice)
        Hb.alloc(ctx, ec * (size_t)lat_geom(c, nc).hstride * nc, "tuning workspace");
    hip_check(zero_fill(F.ptr, bytes, ctx->stream), "tuning clear");
    auto run = [&] {
        if (c.method == kMethodLattice) {
            lattice_mac(ctx, c, lat_geom(c, nc), F.ptr, Hb.ptr, U.ptr, ctx->stream);
            return;
        }
        for (const auto &p : c.parts) {
            SmacGeom g = conv_geom(c, *p);
            g.fstride = fs;
            hip_check(smac_launch(g, c.fp32, p->sparse, nc, F.ptr, U.ptr, c.spec->data.ptr,
                                  (const SmacRow *)p->d_rows.ptr, (const SmacTile *)p->d_tiles.ptr, ctx->stream),
                      "tuning MAC");
        }
    };
    hipEvent_t a, b;
    hip_check(hipEventCreate(&a), "event");
    hip_check(hipEventCreate(&b), "event");
    auto timed = [&](int n) {
        hip_check(hipEventRecord(a, ctx->stream), "event record");
        for (int r = 0; r < n; ++r) run();
        hip_check(hipEventRecord(b, ctx->stream), "event record");
        hip_check(hipEventSynchronize(b), "event sync");
        float ms = 0.f;
        hip_check(hipEventElapsedTime(&ms, a, b), "elapsed");
        return (double)ms;
    };
    // warm-up; long launches get fewer repetitions (about 200 ms per shape)
    const double first = timed(1);
    const int n = std::max(1, std::min(reps, (int)(200.0 / std::max(first, 1e-3))));
    const double ms = timed(n) / n;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms;
}

// Models of a MAC launch in milliseconds, used when the tuning table has no
// entry: block pairs at the measured arithmetic rate of the pair kernel,
// the lattice FFT at half the HBM bandwidth over its streamed bytes (Fhat
// read, H written, read and written, read, Uhat written, the stored
// spectra read).
static double model_pairs_ms(const Conv &c, int nc) {
    double cmacs = 0;   // complex multiply-adds per frequency
    for (const auto &p : c.parts) cmacs += (double)p->n_rows * p->n_tiles * c.ty * c.tz * c.bx * c.bx;
    return 0.01 + 8.0 * cmacs * c.spec->n_freq * nc / (c.fp32 ? 80e9 : 45e9);
}
static double model_lattice_ms(int nb, bool fp32, int nc, const std::vector<Blk> &src, const std::vector<Blk> &tgt) {
    int lo[3], ext[3];
    box_extent(src, tgt, lo, ext);
    const double nf = 4.0 * nb * nb * (nb + 1), ns = lattice_stored_freqs(2 * nb);
    const double ec = fp32 ? 8 : 16, er = fp32 ? 4 : 8;
    const double lx = lattice_len(ext[0]), ly = lattice_len(ext[1]), lz = lattice_len(ext[2]);
    const double box = (double)ext[0] * ext[1] * ext[2], h = lx * ext[1] * ext[2];
    return 0.02 + (nf * ec * nc * (2 * box + 4 * h) + ns * er * lx * ly * lz) / 4e9;
}

// Build a convolution with the MAC method of the context's tuning table for
// its shape: block pairs with one of the compiled tile shapes, or (boxes up
// to 32 blocks along x and y, 64 along z) the lattice FFT.  With autotuning on and no entry
// yet, every candidate is built and timed on this convolution's own
// geometry; the fastest is recorded if it beats the default (pairs with the
// first tile shape) by more than the 3% that repeated timings of one
// candidate differ by, else the default is.  Without an entry the model
// above picks between the default pairs shape and the lattice FFT.  The
// context's method setting can restrict the candidates to block pairs or
// (where feasible) to the lattice FFT.
void build_conv(lgf_plan *plan, Conv &c, const std::vector<Blk> &src, const std::vector<Blk> &tgt, bool fp32,
                int axis) {
    lgf_context *ctx = plan->ctx;
    int xmin = INT32_MAX, xmax = INT32_MIN;
    for (const auto *v : {&src, &tgt})
        for (const auto &b : *v) {
            const int x = axis == 1 ? b.ijk[1] : b.ijk[0];
            xmin = std::min(xmin, x);
            xmax = std::max(xmax, x);
        }
    const int bx = (xmax - xmin + 1) <= 8 ? 8 : 16;
    int tiles[4][2];
    const int n_tiles = smac_tiles(bx, tiles, 4);
    std::vector<std::string> cand;
    for (int i = 0; i < n_tiles; ++i) cand.push_back("pairs " + std::to_string(tiles[i][0]) + "x" + std::to_string(tiles[i][1]));
    const bool lattice_ok = lattice_feasible(src, tgt) && lattice_fits_budget(plan, src, tgt, fp32);
    if (lattice_ok && ctx->mac_method != LGF_MAC_PAIRS) cand.push_back("lattice");
    if (lattice_ok && ctx->mac_method == LGF_MAC_LATTICE) cand.assign(1, "lattice");
    auto build = [&](Conv &into, const std::string &choice) {
        int ty = 0, tz = 0;
        if (parse_choice(choice, ty, tz)) build_conv_lattice(plan, into, src, tgt, fp32);
        else build_conv_tile(plan, into, src, tgt, fp32, axis, ty, tz);
    };
    std::string choice;
    // a table entry timed among block-pair shapes only is kept apart
    const std::string key = tune_key(plan->nb, fp32, plan->mac_nc, axis, src, tgt) +
                            (lattice_ok && ctx->mac_method == LGF_MAC_PAIRS ? "_pairs" : "");
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->tune.find(key);
        // a loaded entry must name a candidate of this convolution
        if (it != ctx->tune.end() && std::find(cand.begin(), cand.end(), it->second.choice) != cand.end())
            choice = it->second.choice;
    }
    if (choice.empty() && ctx->autotune_reps > 0 && cand.size() > 1 && !src.empty() && !tgt.empty()) {
        TuneEntry e;
        e.cand = cand;
        double best = 1e300;
        for (size_t i = 0; i < cand.size(); ++i) {
            Conv trial;
            build(trial, cand[i]);
            const double ms = time_mac(plan, trial, ctx->autotune_reps);
            e.ms.push_back(ms);
            if (i == 0 || (ms < 0.97 * e.ms[0] && ms < best)) {
                best = ms;
                choice = cand[i];
            }
        }
        e.choice = choice;
        std::lock_guard<std::mutex> lk(ctx->mu);
        ctx->tune[key] = e;
    }
    if (choice.empty() && cand.size() > 1 && cand.back() == "lattice") {
        Conv trial;
        build(trial, cand[0]);
        choice = model_lattice_ms(plan->nb, fp32, plan->mac_nc, src, tgt) < model_pairs_ms(trial, plan->mac_nc)
                     ? "lattice"
                     : cand[0];
    }
    if (choice.empty()) choice = cand[0];
    build(c, choice);
}

SmacGeom conv_geom(const Conv &c, const SubConv &p) {
    SmacGeom g;
    g.bx = c.bx;
    g.ty = c.ty;
    g.tz = c.tz;
    g.ey = c.ey;
    g.ez = c.ez;
    g.n_freq = c.spec->n_freq;
    g.n_slots = c.n_slots;
    g.XH = c.spec->XH;
    g.YH = c.spec->YH;
    g.ZH = c.spec->ZH;
    g.XD = g.XH + 1;
    g.YD = g.YH + 1;
    g.ZD = g.ZH + 1;
    g.N = 2 * c.spec->nb;
    g.perm = (const int *)c.spec->perm.ptr;
    g.n_rows = p.n_rows;
    g.n_tiles = p.n_tiles;
    g.lanes = (const int *)p.d_lanes.ptr;
    g.rs = c.rs;
    g.tx0 = p.tx0;
    g.sx0 = p.sx0;
    g.accum = p.accum ? 1 : 0;
    g.fstride = 0;
    g.axis = c.axis;
    return g;
}

// ------------------------------------------------------------------ ops

std::unique_ptr<ConvOp> build_op(lgf_plan *plan, const std::vector<Blk> &src, const std::vector<Blk> &tgt,
                                 bool refine) {
    lgf_context *ctx = plan->ctx;
    const int nb = plan->nb;
    const int64_t nb3 = (int64_t)nb * nb * nb;
    auto op = std::make_unique<ConvOp>();
    using Key = std::tuple<int, int, int>;
    std::map<Key, int> tix;
    for (size_t i = 0; i < tgt.size(); ++i) tix[Key(tgt[i].ijk[0], tgt[i].ijk[1], tgt[i].ijk[2])] = (int)i;
    std::vector<int> t2sh(tgt.size(), -1);
    std::vector<Blk> sh, interior, tcomp(tgt.size());
    int n_sh = 0;
    for (size_t i = 0; i < tgt.size(); ++i) {
        const auto &b = tgt[i];
        bool shell = false;
        for (int dz = -1; dz <= 1 && !shell; ++dz)
            for (int dy = -1; dy <= 1 && !shell; ++dy)
                for (int dx = -1; dx <= 1 && !shell; ++dx)
                    if (!tix.count(Key(b.ijk[0] + dx, b.ijk[1] + dy, b.ijk[2] + dz))) shell = true;
        tcomp[i] = b;
        tcomp[i].off = (int64_t)i * nb3;
        if (shell) {
            Blk q = b;
            q.off = (int64_t)n_sh * nb3;
            sh.push_back(q);
            t2sh[i] = n_sh++;
        } else {
            interior.push_back(b);
        }
    }
    if (!refine || interior.empty()) {
        op->c64 = std::make_unique<Conv>();
        build_conv(plan, *op->c64, src, tgt, false);
        plan->convs_view.push_back(op->c64.get());
        return op;
    }
    op->refined = true;
    op->n_t = (int)tgt.size();
    op->n_sh = n_sh;
    // float64 sources: the shell blocks (cut residual), then the source
    // blocks outside T (copied from the source field at solve time)
    std::vector<Blk> cut = sh;
    std::vector<int64_t> out_src, out_dst;
    for (const auto &b : src)
        if (!tix.count(Key(b.ijk[0], b.ijk[1], b.ijk[2]))) {
            Blk q = b;
            q.off = (int64_t)(n_sh + (int)out_src.size()) * nb3;
            out_src.push_back(b.off);
            out_dst.push_back(q.off);
            cut.push_back(q);
        }
    op->n_out = (int)out_src.size();
    // The cut is a thin shell: rows along x through the x-faces of T hold
    // only a block or two of it.  Each cut block goes to the orientation
    // (rows along x or along y) whose row through it holds more cut blocks,
    // and each orientation is one float64 convolution.
    std::map<std::pair<int, int>, int> xrow, yrow;
    for (const auto &b : cut) {
        ++xrow[{b.ijk[1], b.ijk[2]}];
        ++yrow[{b.ijk[0], b.ijk[2]}];
    }
    std::vector<Blk> cutx, cuty;
    for (const auto &b : cut)
        (yrow[{b.ijk[0], b.ijk[2]}] > xrow[{b.ijk[1], b.ijk[2]}] ? cuty : cutx).push_back(b);
    // Keep the split only when it saves MAC work.  Work ~ source rows x
    // target tiles of each convolution; both have all of T as targets, so
    // on thin supports (cut ~ all of T) one convolution is cheaper.
    {
        auto n_rows = [](const std::vector<Blk> &v, int a) {
            std::set<std::pair<int, int>> r;
            for (const auto &b : v) r.insert({b.ijk[a], b.ijk[2]});
            return (int64_t)r.size();
        };
        auto n_tiles = [&](int a, int ty) {
            std::set<std::pair<int, int>> t;
            for (const auto &b : tgt) t.insert({(b.ijk[a] + 1024 * ty) / ty, (b.ijk[2] + 1024 * 8) / 8});
            return (int64_t)t.size();
        };
        const int ty = 16;   // rows per tile of the default 16-wide template
        const int64_t single = n_rows(cut, 1) * n_tiles(1, ty);
        const int64_t split = n_rows(cutx, 1) * n_tiles(1, ty) + (cuty.empty() ? 0 : n_rows(cuty, 0) * n_tiles(0, ty));
        // the lattice FFT costs the same for any sources in the box
        if (cuty.empty() || split * 5 >= single * 4 || lattice_feasible(cut, tgt)) {
            cutx = cut;
            cuty.clear();
        }
    }
    op->c32 = std::make_unique<Conv>();
    build_conv(plan, *op->c32, src, tcomp, true);
    if (!cutx.empty()) {
        op->c64 = std::make_unique<Conv>();
        build_conv(plan, *op->c64, cutx, tgt, false, 0);
    }
    if (!cuty.empty()) {
        op->c64y = std::make_unique<Conv>();
        build_conv(plan, *op->c64y, cuty, tgt, false, 1);
    }
    op->ccorr = std::make_unique<Conv>();
    build_conv(plan, *op->ccorr, tcomp, tgt, true);
    for (const Conv *c : {op->c32.get(), op->c64.get(), op->c64y.get(), op->ccorr.get()})
        if (c) plan->convs_view.push_back(c);
    // dense map of T over its bounding box
    int lo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, hi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (const auto &b : tgt)
        for (int a = 0; a < 3; ++a) {
            lo[a] = std::min(lo[a], b.ijk[a]);
            hi[a] = std::max(hi[a], b.ijk[a]);
        }
    RefGeom &g = op->geom;
    for (int a = 0; a < 3; ++a) {
        g.lo[a] = lo[a];
        g.dim[a] = hi[a] - lo[a] + 1;
    }
    std::vector<int> map((size_t)g.dim[0] * g.dim[1] * g.dim[2], -1);
    std::vector<int> tblk, shblk;
    std::vector<int64_t> dofs;
    for (size_t i = 0; i < tgt.size(); ++i) {
        const auto &b = tgt[i];
        map[((size_t)(b.ijk[2] - lo[2]) * g.dim[1] + (b.ijk[1] - lo[1])) * g.dim[0] + (b.ijk[0] - lo[0])] = (int)i;
        for (int a = 0; a < 3; ++a) tblk.push_back(b.ijk[a]);
        dofs.push_back(b.off);
    }
    for (const auto &b : sh)
        for (int a = 0; a < 3; ++a) shblk.push_back(b.ijk[a]);
    std::map<Key, int64_t> sof;
    for (const auto &b : src) sof[Key(b.ijk[0], b.ijk[1], b.ijk[2])] = b.off;
    std::vector<int64_t> gofs;
    for (const auto &b : tgt) {
        auto it = sof.find(Key(b.ijk[0], b.ijk[1], b.ijk[2]));
        gofs.push_back(it == sof.end() ? -1 : it->second);
    }
    auto up = [&](DeviceBuffer &d, const void *h, size_t n, const char *what) {
        d.alloc(ctx, std::max<size_t>(n, 8), what);
        if (n) hip_check(hipMemcpy(d.ptr, h, n, hipMemcpyHostToDevice), "upload");
    };
    up(op->d_map, map.data(), sizeof(int) * map.size(), "target map");
    up(op->d_tblk, tblk.data(), sizeof(int) * tblk.size(), "target blocks");
    up(op->d_t2sh, t2sh.data(), sizeof(int) * t2sh.size(), "shell index");
    up(op->d_gofs, gofs.data(), sizeof(int64_t) * gofs.size(), "source offsets");
    up(op->d_dofs, dofs.data(), sizeof(int64_t) * dofs.size(), "target offsets");
    up(op->d_out_src, out_src.data(), sizeof(int64_t) * out_src.size(), "outside sources");
    up(op->d_out_dst, out_dst.data(), sizeof(int64_t) * out_dst.size(), "outside sources");
    DeviceBuffer d_shblk;
    up(d_shblk, shblk.data(), sizeof(int) * shblk.size(), "shell blocks");
    op->d_depth.alloc(ctx, (size_t)std::max(1, n_sh) * nb3, "shell depth");
    hip_check(refine_depth(nb, g, (const int *)op->d_map.ptr, (const int *)d_shblk.ptr,
                           (unsigned char *)op->d_depth.ptr, n_sh, ctx->stream),
              "shell depth");
    hip_check(hipStreamSynchronize(ctx->stream), "depth sync");
    return op;
}

void refine_middle(lgf_plan *plan, const ConvOp &op, const double *src, double *dst, const double *ut, double *rin,
                   double *cut, double dx, int accumulate, hipStream_t s) {
    const int nb = plan->nb;
    RefGeom g = op.geom;
    g.dx = dx;
    StageTimer t(plan->ctx, 3, s);
    hip_check(refine_residual(nb, g, (const int *)op.d_map.ptr, (const int *)op.d_tblk.ptr, (const int *)op.d_t2sh.ptr,
                              (const unsigned char *)op.d_depth.ptr, ut, src, (const int64_t *)op.d_gofs.ptr,
                              (const int64_t *)op.d_dofs.ptr, dst, accumulate, rin, cut, op.n_t, s),
              "refinement residual");
    if (op.n_out > 0)
        hip_check(copy_blocks(nb, src, cut, (const int64_t *)op.d_out_src.ptr, (const int64_t *)op.d_out_dst.ptr,
                              op.n_out, s),
                  "outside sources");
}

void run_op(lgf_plan *plan, const ConvOp &op, const double *src, int64_t sstride, double *dst, int64_t dstride,
            int nc, double dx, int accumulate, hipStream_t s) {
    for (int c0 = 0; c0 < nc; c0 += kMacComponents) {
        const int ng = std::min(kMacComponents, nc - c0);
        const double *sg = src + (size_t)c0 * sstride;
        double *dg = dst + (size_t)c0 * dstride;
        if (!op.refined) {
            run_conv(plan, *op.c64, sg, sstride, dg, dstride, ng, dx, accumulate, s);
            continue;
        }
        double *ut = (double *)plan->ws_ut.ptr, *rin = (double *)plan->ws_rho.ptr, *cut = (double *)plan->ws_ush.ptr;
        run_conv(plan, *op.c32, sg, sstride, ut, plan->ut_len, ng, dx, 0, s);
        for (int c = 0; c < ng; ++c)
            refine_middle(plan, op, sg + (size_t)c * sstride, dg + (size_t)c * dstride, ut + (size_t)c * plan->ut_len,
                          rin + (size_t)c * plan->ut_len, cut + (size_t)c * plan->cut_len, dx, accumulate, s);
        if (op.c64) run_conv(plan, *op.c64, cut, plan->cut_len, dg, dstride, ng, dx, 1, s);
        if (op.c64y) run_conv(plan, *op.c64y, cut, plan->cut_len, dg, dstride, ng, dx, 1, s);
        run_conv(plan, *op.ccorr, rin, plan->ut_len, dg, dstride, ng, dx, 1, s);
    }
}

void plan_alloc_refine(lgf_plan *plan, const std::vector<const ConvOp *> &ops) {
    int64_t nt = 0, ncut = 0;
    for (const ConvOp *o : ops)
        if (o && o->refined) {
            nt = std::max<int64_t>(nt, o->n_t);
            ncut = std::max<int64_t>(ncut, (int64_t)o->n_sh + o->n_out);
        }
    if (nt == 0) return;
    const int64_t nb3 = (int64_t)plan->nb * plan->nb * plan->nb;
    plan->ut_len = nt * nb3;
    plan->cut_len = std::max<int64_t>(1, ncut) * nb3;
    plan->ws_ut.alloc(plan->ctx, sizeof(double) * plan->ut_len * plan->mac_nc, "u float32 pass");
    plan->ws_rho.alloc(plan->ctx, sizeof(double) * plan->ut_len * plan->mac_nc, "refinement residual");
    plan->ws_ush.alloc(plan->ctx, sizeof(double) * plan->cut_len * plan->mac_nc, "cut residual");
}

// Spectral workspace large enough for every convolution of the plan, for
// mac_nc components.
SpecWs spectral_need(const lgf_plan *plan) {
    SpecWs w;
    size_t need = 0, hneed = 0;
    for (const Conv *c : plan->convs_view) {
        const size_t elem = c->fp32 ? 8 : 16;
        need = std::max(need, elem * (size_t)c->spec->n_freq * (size_t)c->n_slots);
        if (c->method == kMethodLattice) hneed = std::max(hneed, elem * (size_t)lat_geom(*c, 1).hstride);
    }
    w.fhat_bytes = w.uhat_bytes = need * (size_t)plan->mac_nc;
    w.lat_bytes = hneed * (size_t)plan->mac_nc;
    return w;
}

void plan_alloc_spectral(lgf_plan *plan) {
    const SpecWs w = spectral_need(plan);
    plan->Fhat.alloc(plan->ctx, w.fhat_bytes, "Fhat workspace");
    plan->Uhat.alloc(plan->ctx, w.uhat_bytes, "Uhat workspace");
    if (w.lat_bytes) plan->ws_lat.alloc(plan->ctx, w.lat_bytes, "lattice workspace");
}

// Run one convolution for nc <= kMacComponents components:
// dst_c (+)= dx^2 * G * src_c on the conv's blocks, component c at
// src + c*sstride / dst + c*dstride, spectra at Fhat / Uhat + c*fs.
void run_conv(lgf_plan *plan, const Conv &c, const double *src, int64_t sstride, double *dst, int64_t dstride,
              int nc, double dx, int accumulate, hipStream_t s) {
    const int nb = plan->nb;
    const double N3 = 8.0 * nb * nb * nb;
    const size_t elem = c.fp32 ? 8 : 16;
    const int64_t fs = (int64_t)c.spec->n_freq * c.n_slots;   // elements per component region
    SpecWs own;
    own.fhat = plan->Fhat.ptr;
    own.uhat = plan->Uhat.ptr;
    own.lat = plan->ws_lat.ptr;
    own.fhat_bytes = plan->Fhat.bytes;
    own.uhat_bytes = plan->Uhat.bytes;
    own.lat_bytes = plan->ws_lat.bytes;
    const SpecWs &ws = plan->ws_scratch ? *plan->ws_scratch : own;
    if (nc < 1 || nc > kMacComponents || (size_t)nc * fs * elem > ws.fhat_bytes || (size_t)nc * fs * elem > ws.uhat_bytes)
        throw Failure(LGF_E_INVALID, "internal: component count outside the spectral workspace");
    // empty slots of Fhat must read as zero for the block-pair MAC; the
    // forward FFT writes only occupied slots, so clear when another slot map
    // used the buffer last (a convolution with a source in every slot
    // overwrites all it reads).  Shared scratch may hold anything: clear it
    // whenever a slot is empty.  The lattice x pass skips empty slots itself.
    const bool needs_zeros = !fhat_full(c) && c.method != kMethodLattice;
    if (plan->ws_scratch) {
        if (needs_zeros) hip_check(zero_fill(ws.fhat, (size_t)nc * fs * elem, s), "clear Fhat");
    } else if (plan->fhat_conv != &c) {
        if (needs_zeros) hip_check(zero_fill(ws.fhat, ws.fhat_bytes, s), "clear Fhat");
        plan->fhat_conv = needs_zeros ? &c : nullptr;
    }
    for (int k = 0; k < nc; ++k) {
        StageTimer t(plan->ctx, 0, s);
        hip_check(block_fft_forward(nb, c.fp32, src + (size_t)k * sstride, (const int64_t *)c.d_src_off.ptr,
                                    (const int *)c.d_src_slot.ptr, c.n_src, (char *)ws.fhat + k * fs * elem,
                                    c.n_slots, c.method == kMethodLattice, 1.0, s),
                  "forward block FFT");
    }
    const void *uhat2 = nullptr;   // the one-pass lattice MAC's second term
    if (c.method == kMethodLattice) {
        uhat2 = lattice_mac(plan->ctx, c, lat_geom(c, nc), ws.fhat, ws.lat, ws.uhat, s);
    } else if (c.parts.empty()) {   // no source or no target: the convolution is zero
        hip_check(zero_fill(ws.uhat, (size_t)nc * fs * elem, s), "clear Uhat");
    }
    for (const auto &p : c.parts) {
        StageTimer t(plan->ctx, 1, s);
        SmacGeom g = conv_geom(c, *p);
        g.fstride = fs;
        hip_check(smac_launch(g, c.fp32, p->sparse, nc, ws.fhat, ws.uhat, c.spec->data.ptr,
                              (const SmacRow *)p->d_rows.ptr, (const SmacTile *)p->d_tiles.ptr, s),
                  "spectral MAC");
    }
    for (int k = 0; k < nc; ++k) {
        StageTimer t(plan->ctx, 2, s);
        hip_check(block_fft_inverse(nb, c.fp32, (char *)ws.uhat + k * fs * elem,
                                    uhat2 ? (const char *)uhat2 + k * fs * elem : nullptr, c.n_slots,
                                    c.method == kMethodLattice, (const int *)c.d_tgt_slot.ptr, (const int64_t *)c.d_tgt_off.ptr, c.n_tgt,
                                    dst + (size_t)k * dstride, conv_scale(plan, dx) / N3, accumulate, s),
                  "inverse block FFT");
    }
}

}  // namespace lgf
