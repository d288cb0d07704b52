// extern "C" entry points of include/lgf.h.  Every call converts failures
// into an lgf_status and a thread-local message; no exception crosses.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lgf.h"
#include "lgf_device.hpp"
#include "lgf_runtime.hpp"

using namespace lgf;

namespace {

template <typename F> lgf_status guard(F &&f) {
    try {
        f();
        return LGF_OK;
    } catch (const Failure &e) {
        set_error(e.what());
        return e.status;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return LGF_E_NOMEM;
    } catch (const std::exception &e) {
        set_error(e.what());
        return LGF_E_DEVICE;
    }
}

void require(bool ok, const std::string &msg) {
    if (!ok) throw Failure(LGF_E_INVALID, msg);
}

struct DeviceScope {
    int prev = -1;
    explicit DeviceScope(int dev) {
        hip_check(hipGetDevice(&prev), "hipGetDevice");
        if (prev != dev) hip_check(hipSetDevice(dev), "hipSetDevice");
    }
    ~DeviceScope() {
        int cur = -1;
        if (hipGetDevice(&cur) == hipSuccess && cur != prev && prev >= 0) hipSetDevice(prev);
    }
};

using Key = std::tuple<int, int, int>;

// Device scratch of lgf_solve_scratch: the spectral workspace (Fhat, Uhat,
// lattice H) of one solve, shared by every such call on a device.  In host
// code `scratch` names a host-side stand-in; its device address is looked up
// once per device (hipGetSymbolAddress, with that device current) and only
// that address is handed to kernels.
constexpr size_t kScratchBytes = size_t(LGF_SCRATCH_MAX_BYTES);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;     // device -> address of its copy of `scratch`

void *scratch_address(int device) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(device);
    if (it != g_scratch_ptr.end()) return it->second;
    void *ptr = nullptr;
    hip_check(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) throw Failure(LGF_E_DEVICE, "no device address for the static scratch array");
    g_scratch_ptr[device] = ptr;
    return ptr;
}

size_t align256(size_t n) { return (n + 255) & ~size_t(255); }

void validate_and_copy(lgf_plan *p, const lgf_problem *d) {
    require(d != nullptr, "null problem");
    require(d->n_levels >= 1 && d->n_levels <= 8, "n_levels must be in [1, 8]");
    require(d->nb == 8 || d->nb == 16, "nb must be 8 or 16");
    require(d->dx0 > 0 && std::isfinite(d->dx0), "dx0 must be positive");
    require(d->n_components >= 1 && d->n_components <= 8, "n_components must be in [1, 8]");
    require(d->precision == LGF_FP64 || d->precision == LGF_FP32_REFINE, "unknown precision");
    require(d->ne_blocks >= 0 && d->ne_blocks <= 4, "ne_blocks must be in [0, 4]");
    require(d->levels != nullptr, "null levels");
    p->K = d->n_levels;
    p->nb = d->nb;
    p->nc = d->n_components;
    p->prec = d->precision;
    p->ne = d->ne_blocks == 0 ? 1 : d->ne_blocks;
    p->dx0 = d->dx0;
    const int64_t nb3 = (int64_t)d->nb * d->nb * d->nb;
    int64_t base = 0;
    std::vector<std::set<Key>> sets(p->K);
    for (int k = 0; k < p->K; ++k) {
        const lgf_level &L = d->levels[k];
        require(L.n_blocks >= 1, "every level needs at least one block");
        require(L.block_ijk != nullptr, "null block list");
        std::vector<Blk> v;
        v.reserve(L.n_blocks);
        for (int i = 0; i < L.n_blocks; ++i) {
            Blk b;
            for (int a = 0; a < 3; ++a) {
                b.ijk[a] = L.block_ijk[3 * i + a];
                require(b.ijk[a] > -(1 << 20) && b.ijk[a] < (1 << 20), "block coordinate out of range");
            }
            b.off = base + (int64_t)i * nb3;
            require(sets[k].insert(Key(b.ijk[0], b.ijk[1], b.ijk[2])).second, "duplicate block in a level");
            v.push_back(b);
        }
        p->level_base.push_back(base);
        base += (int64_t)L.n_blocks * nb3;
        p->levels.push_back(std::move(v));
    }
    p->comp_len = base;
    // nesting: a level-(k+1) block's parent octant lies in a level-k block
    auto fdiv = [](int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); };
    for (int k = 1; k < p->K; ++k)
        for (const auto &b : p->levels[k])
            require(sets[k - 1].count(Key(fdiv(b.ijk[0], 2), fdiv(b.ijk[1], 2), fdiv(b.ijk[2], 2))) > 0,
                    "level " + std::to_string(k) + " block outside level " + std::to_string(k - 1));
    // cell masks: 0 / 1 only, and no 1 under a finer block (levels overlap)
    p->cell_mask.assign(p->K, {});
    for (int k = 0; k < p->K; ++k) {
        const lgf_level &L = d->levels[k];
        if (!L.cell_mask) continue;
        const size_t n = (size_t)L.n_blocks * nb3;
        p->cell_mask[k].assign(L.cell_mask, L.cell_mask + n);
        for (size_t i = 0; i < n; ++i)
            require(p->cell_mask[k][i] <= 1, "cell mask values must be 0 or 1 (level " + std::to_string(k) + ")");
        if (k + 1 < p->K) {
            std::map<Key, int> idx;
            for (int i = 0; i < (int)p->levels[k].size(); ++i) {
                const auto &b = p->levels[k][i];
                idx[Key(b.ijk[0], b.ijk[1], b.ijk[2])] = i;
            }
            const int nb = p->nb, H = nb / 2;
            for (const auto &fb : p->levels[k + 1]) {
                const int px = fdiv(fb.ijk[0], 2), py = fdiv(fb.ijk[1], 2), pz = fdiv(fb.ijk[2], 2);
                const int bi = idx.at(Key(px, py, pz));
                const int ox = (fb.ijk[0] - 2 * px) * H, oy = (fb.ijk[1] - 2 * py) * H, oz = (fb.ijk[2] - 2 * pz) * H;
                for (int z = 0; z < H; ++z)
                    for (int y = 0; y < H; ++y)
                        for (int x = 0; x < H; ++x)
                            require(p->cell_mask[k][(size_t)bi * nb3 + ((oz + z) * nb + (oy + y)) * nb + (ox + x)] == 0,
                                    "levels overlap after masking: a level-" + std::to_string(k) +
                                        " cell under a level-" + std::to_string(k + 1) + " block is kept");
            }
        }
    }
}

}  // namespace

size_t lgf_plan::workspace_bytes() const {
    size_t b = Fhat.bytes + Uhat.bytes + ws_fhat.bytes + ws_F.bytes + ws_psi[0].bytes + ws_psi[1].bytes +
               ws_ppsi.bytes + ws_srcF.bytes + ws_srcf.bytes + ws_ut.bytes + ws_ush.bytes + ws_rho.bytes +
               ws_lat.bytes;
    for (const Conv *c : convs_view) {
        b += c->d_src_slot.bytes + c->d_tgt_slot.bytes + c->d_src_off.bytes + c->d_tgt_off.bytes;
        for (const auto &p : c->parts) b += p->d_rows.bytes + p->d_tiles.bytes + p->d_lanes.bytes;
    }
    for (const auto &L : lv)
        b += L->d_cover.bytes + L->d_own_off.bytes + L->d_cf_fine.bytes + L->d_cf_coarse.bytes + L->d_cf_oct.bytes +
             L->d_fblk.bytes + L->d_ext_own.bytes + L->d_cmap.bytes + L->d_cu_src.bytes + L->d_cu_dst.bytes +
             L->d_cp_src.bytes + L->d_cp_dst.bytes;
    return b;
}

extern "C" {

lgf_status lgf_context_create(int device, size_t hbm_budget_bytes, lgf_context **out) {
    if (!out) {
        set_error("null out pointer");
        return LGF_E_INVALID;
    }
    *out = nullptr;
    lgf_context *ctx = nullptr;
    lgf_status st = guard([&] {
        int n = 0;
        hip_check(hipGetDeviceCount(&n), "hipGetDeviceCount");
        require(device >= 0 && device < n, "no such device");
        DeviceScope ds(device);
        ctx = new lgf_context(device, hbm_budget_bytes);
        hip_check(hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking), "hipStreamCreate");
        build_context_table(ctx);
        ring_init(ctx);
        scratch_address(device);     // set-up of lgf_solve_scratch on this device
    });
    if (st != LGF_OK) {
        if (ctx) lgf_context_destroy(ctx);
        return st;
    }
    *out = ctx;
    return LGF_OK;
}

void lgf_context_destroy(lgf_context *ctx) {
    if (!ctx) return;
    int prev = -1;
    hipGetDevice(&prev);
    hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    for (auto &e : ctx->pending) {
        (void)hipEventSynchronize(e.b);
        (void)hipEventDestroy(e.a);
        (void)hipEventDestroy(e.b);
    }
    ctx->pending.clear();
    ring_free(ctx);
    ctx->lat_tables.clear();
    ctx->tables.clear();
    ctx->if_cubes.clear();
    ctx->gcube.release();
    if (ctx->stream) hipStreamDestroy(ctx->stream);
    delete ctx;
    if (prev >= 0) hipSetDevice(prev);
}

size_t lgf_context_bytes(const lgf_context *ctx) { return ctx ? ctx->used : 0; }

lgf_status lgf_plan_create(lgf_context *ctx, const lgf_problem *desc, lgf_plan **out) {
    if (!ctx || !out) {
        set_error("null context or out pointer");
        return LGF_E_INVALID;
    }
    *out = nullptr;
    lgf_plan *p = new lgf_plan();
    p->ctx = ctx;
    lgf_status st = guard([&] {
        DeviceScope ds(ctx->device);
        validate_and_copy(p, desc);
        build_schedule(p);
    });
    if (st != LGF_OK) {
        lgf_plan_destroy(p);
        return st;
    }
    *out = p;
    return LGF_OK;
}

lgf_status lgf_plan_create_if(lgf_context *ctx, const lgf_problem *desc, double a0, lgf_plan **out) {
    if (!ctx || !out) {
        set_error("null context or out pointer");
        return LGF_E_INVALID;
    }
    *out = nullptr;
    lgf_plan *p = new lgf_plan();
    p->ctx = ctx;
    lgf_status st = guard([&] {
        require(a0 > 0.0 && std::isfinite(a0) && a0 <= 1.0e6, "a0 must be positive and at most 1e6");
        DeviceScope ds(ctx->device);
        validate_and_copy(p, desc);
        if (p->prec != LGF_FP64)
            throw Failure(LGF_E_UNSUPPORTED, "the integrating factor is applied in float64 only");
        p->if_a0 = a0;
        build_schedule(p);
    });
    if (st != LGF_OK) {
        lgf_plan_destroy(p);
        return st;
    }
    *out = p;
    return LGF_OK;
}

lgf_status lgf_plan_create_flgf(lgf_context *ctx, const lgf_problem *desc, int near_blocks, lgf_plan **out) {
    if (!ctx || !out) {
        set_error("null context or out pointer");
        return LGF_E_INVALID;
    }
    *out = nullptr;
    lgf_plan *p = new lgf_plan();
    p->ctx = ctx;
    lgf_status st = guard([&] {
        require(near_blocks >= 0 && near_blocks <= 8, "near_blocks must be in [0, 8]");
        DeviceScope ds(ctx->device);
        validate_and_copy(p, desc);
        if (p->K != 1 || p->nb != 16 || p->prec != LGF_FP64)
            throw Failure(LGF_E_UNSUPPORTED, "the fast-LGF approximation serves single-level float64 plans of 16^3 blocks");
        require(p->cell_mask[0].empty(), "the fast-LGF approximation takes no cell mask");
        p->flgf_D = near_blocks;
        p->kernel0.band = 1;
        p->kernel0.D = near_blocks;
        build_schedule(p);
    });
    if (st != LGF_OK) {
        lgf_plan_destroy(p);
        return st;
    }
    *out = p;
    return LGF_OK;
}

lgf_status lgf_problem_check(const lgf_problem *desc) {
    return guard([&] {
        lgf_plan tmp;
        validate_and_copy(&tmp, desc);
    });
}

void lgf_plan_destroy(lgf_plan *plan) {
    if (!plan) return;
    int prev = -1;
    hipGetDevice(&prev);
    hipSetDevice(plan->ctx->device);
    hipDeviceSynchronize();
    delete plan;
    if (prev >= 0) hipSetDevice(prev);
}

size_t lgf_plan_workspace_bytes(const lgf_plan *plan) { return plan ? plan->workspace_bytes() : 0; }

size_t lgf_plan_cells(const lgf_plan *plan, int level) {
    if (!plan || level < 0 || level >= plan->K) return 0;
    return plan->levels[level].size() * (size_t)plan->nb * plan->nb * plan->nb;
}

size_t lgf_plan_field_len(const lgf_plan *plan) { return plan ? (size_t)plan->comp_len * plan->nc : 0; }

lgf_status lgf_solve(lgf_plan *plan, const double *f, double *u, void *stream, lgf_report *rep) {
    return guard([&] {
        require(plan != nullptr, "null plan");
        require(f != nullptr && u != nullptr, "null field pointer");
        require(((uintptr_t)f % 8) == 0 && ((uintptr_t)u % 8) == 0, "misaligned field pointer");
        DeviceScope ds(plan->ctx->device);
        run_plan(plan, f, u, (hipStream_t)stream, rep);
    });
}

lgf_status lgf_solve_scratch(lgf_plan *plan, const double *f, double *u, void *stream) {
    return guard([&] {
        require(plan != nullptr, "null plan");
        require(f != nullptr && u != nullptr, "null field pointer");
        require(((uintptr_t)f % 8) == 0 && ((uintptr_t)u % 8) == 0, "misaligned field pointer");
        const SpecWs need = spectral_need(plan);
        const size_t total = align256(need.fhat_bytes) + align256(need.uhat_bytes) + align256(need.lat_bytes);
        if (total > kScratchBytes)
            throw Failure(LGF_E_INVALID, "plan needs " + std::to_string(total) +
                                             " bytes of spectral workspace; the static scratch holds " +
                                             std::to_string(kScratchBytes));
        DeviceScope ds(plan->ctx->device);
        char *base = (char *)scratch_address(plan->ctx->device);
        SpecWs ws = need;
        ws.fhat = base;
        ws.uhat = base + align256(need.fhat_bytes);
        ws.lat = need.lat_bytes ? base + align256(need.fhat_bytes) + align256(need.uhat_bytes) : nullptr;
        struct Restore {
            lgf_plan *p;
            ~Restore() {
                p->ws_scratch = nullptr;
                g_no_timing = false;
            }
        } restore{plan};
        plan->ws_scratch = &ws;
        g_no_timing = true;
        run_plan(plan, f, u, (hipStream_t)stream, nullptr);
    });
}

lgf_status lgf_velocity_refresh(lgf_plan *plan, const double *omega, double *psi, double *u, void *stream) {
    return guard([&] {
        require(plan != nullptr, "null plan");
        require(plan->K == 1 && plan->nc == 3 && plan->if_a0 == 0.0,
                "the velocity refresh needs a single-level LGF plan of 3 components");
        require(omega && psi && u, "null field pointer");
        require(((uintptr_t)omega % 8) == 0 && ((uintptr_t)psi % 8) == 0 && ((uintptr_t)u % 8) == 0,
                "misaligned field pointer");
        require(psi != omega && psi != u && u != omega, "omega, psi and u must be distinct arrays");
        DeviceScope ds(plan->ctx->device);
        hipStream_t s = (hipStream_t)stream;
        run_plan(plan, omega, psi, s, nullptr);
        StageTimer t(plan->ctx, kStageOther, s);
        hip_check(curl_backward_blocks(plan->nb, psi, u, plan->comp_len, (const int64_t *)plan->d_blk_off.ptr,
                                       (const int64_t *)plan->d_blk_back.ptr, (int)plan->levels[0].size(),
                                       1.0 / plan->dx0, s),
                  "curl");
    });
}

int64_t lgf_plan_source_blocks(const lgf_plan *plan, int level, int32_t *ijk) {
    if (!plan || level < 0 || level >= (int)plan->src_ijk.size()) return -1;
    const auto &v = plan->src_ijk[level];
    if (ijk) std::copy(v.begin(), v.end(), ijk);
    return (int64_t)v.size() / 3;
}

lgf_status lgf_solve_indicator(lgf_plan *plan, const double *f, double *u, void *stream, double *block_rms,
                               double *block_max) {
    return guard([&] {
        require(plan != nullptr, "null plan");
        require(f != nullptr && u != nullptr, "null field pointer");
        require(((uintptr_t)f % 8) == 0 && ((uintptr_t)u % 8) == 0, "misaligned field pointer");
        require(block_rms != nullptr && block_max != nullptr, "null statistics arrays");
        DeviceScope ds(plan->ctx->device);
        hipStream_t s = (hipStream_t)stream;
        hip_check(zero_fill(plan->d_ind.ptr, plan->d_ind.bytes, s), "clear indicator");
        struct Restore {
            lgf_plan *p;
            ~Restore() { p->collect = false; }
        } restore{plan};
        plan->collect = true;
        run_plan(plan, f, u, s, nullptr);
        const size_t n = (size_t)plan->ind_total * plan->nc;
        std::vector<double> h(2 * n);
        hip_check(hipMemcpyAsync(h.data(), plan->d_ind.ptr, sizeof(double) * 2 * n, hipMemcpyDeviceToHost, s),
                  "indicator copy");
        hip_check(hipStreamSynchronize(s), "indicator sync");
        const double nb3 = (double)plan->nb * plan->nb * plan->nb;
        for (size_t i = 0; i < n; ++i) {
            block_rms[i] = std::sqrt(h[2 * i] / nb3);
            block_max[i] = h[2 * i + 1];
        }
    });
}

struct lgf_graph {
    lgf_plan *plan = nullptr;                                  // single-plan graphs
    std::vector<lgf_plan *> plans;                             // batch graphs
    std::vector<std::unique_ptr<lgf::DeviceBuffer>> tables;    // job tables of a batch graph
    int device = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

lgf_status lgf_graph_create(lgf_plan *plan, const double *f, double *u, lgf_graph **out) {
    return guard([&] {
        require(out != nullptr, "null output");
        *out = nullptr;
        require(plan != nullptr, "null plan");
        require(f != nullptr && u != nullptr, "null field pointer");
        require(((uintptr_t)f % 8) == 0 && ((uintptr_t)u % 8) == 0, "misaligned field pointer");
        DeviceScope ds(plan->ctx->device);
        auto g = std::make_unique<lgf_graph>();
        g->plan = plan;
        g->device = plan->ctx->device;
        g->graph = capture_solve(plan, f, u);
        const hipError_t e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g->graph);
            hip_check(e, "graph instantiate");
        }
        *out = g.release();
    });
}

lgf_status lgf_graph_create_batch(lgf_context *ctx, int n, lgf_plan *const *plans, const double *const *f,
                                  double *const *u, lgf_graph **out) {
    return guard([&] {
        require(out != nullptr, "null output");
        *out = nullptr;
        require(ctx != nullptr && n >= 1, "bad batch arguments");
        require(plans && f && u, "null batch arrays");
        std::set<const lgf_plan *> seen;
        for (int i = 0; i < n; ++i) {
            require(plans[i] && plans[i]->ctx == ctx, "plan from another context");
            require(seen.insert(plans[i]).second, "a plan appears twice in one batch");
            require(f[i] && u[i], "null field pointer");
            require(((uintptr_t)f[i] % 8) == 0 && ((uintptr_t)u[i] % 8) == 0, "misaligned field pointer");
        }
        DeviceScope ds(ctx->device);
        auto g = std::make_unique<lgf_graph>();
        g->plans.assign(plans, plans + n);
        g->device = ctx->device;
        g->graph = capture_batch(ctx, n, plans, f, u, g->tables);
        const hipError_t e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g->graph);
            hip_check(e, "graph instantiate");
        }
        *out = g.release();
    });
}

lgf_status lgf_graph_launch(lgf_graph *g, void *stream) {
    return guard([&] {
        require(g != nullptr && g->exec != nullptr, "null graph");
        DeviceScope ds(g->device);
        // the graph clears the spectral workspace itself; the next eager
        // solve must not assume any slot map either
        if (g->plan) g->plan->fhat_conv = nullptr;
        for (lgf_plan *p : g->plans) p->fhat_conv = nullptr;
        hip_check(hipGraphLaunch(g->exec, (hipStream_t)stream), "graph launch");
    });
}

void lgf_graph_destroy(lgf_graph *g) {
    if (!g) return;
    DeviceScope ds(g->device);
    if (!g->tables.empty()) (void)hipDeviceSynchronize();   // no replay may still read the job tables
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

lgf_status lgf_solve_batch(lgf_context *ctx, int n, lgf_plan *const *plans, const double *const *f,
                           double *const *u, void *stream, lgf_report *reps) {
    return guard([&] {
        require(ctx != nullptr && n >= 0, "bad batch arguments");
        if (n == 0) return;
        require(plans && f && u, "null batch arrays");
        std::set<const lgf_plan *> seen;
        for (int i = 0; i < n; ++i) {
            require(plans[i] && plans[i]->ctx == ctx, "plan from another context");
            require(seen.insert(plans[i]).second, "a plan appears twice in one batch");
            require(f[i] && u[i], "null field pointer");
        }
        DeviceScope ds(ctx->device);
        run_batch(ctx, n, plans, f, u, (hipStream_t)stream, reps);
    });
}

int lgf_table_radius(void) { return kTableRadius; }

lgf_status lgf_table_values(lgf_context *ctx, int64_t n, const int32_t *ijk, double *out) {
    return guard([&] {
        require(ctx && n >= 0, "bad arguments");
        if (n == 0) return;
        require(ijk && out, "null arrays");
        DeviceScope ds(ctx->device);
        DeviceBuffer di, dout;
        di.alloc(ctx, sizeof(int32_t) * 3 * n, "points");
        dout.alloc(ctx, sizeof(double) * n, "values");
        hip_check(hipMemcpy(di.ptr, ijk, sizeof(int32_t) * 3 * n, hipMemcpyHostToDevice), "upload");
        hip_check(eval_lgf_points((const double *)ctx->gcube.ptr, (const int *)di.ptr, (double *)dout.ptr, n,
                                  ctx->stream),
                  "eval");
        hip_check(hipStreamSynchronize(ctx->stream), "sync");
        hip_check(hipMemcpy(out, dout.ptr, sizeof(double) * n, hipMemcpyDeviceToHost), "download");
    });
}

lgf_status lgf_block_spectrum(lgf_context *ctx, int nb, const int32_t d[3], double *out) {
    return guard([&] {
        require(ctx && d && out, "null arguments");
        require(nb == 8 || nb == 16, "nb must be 8 or 16");
        const int ax = std::abs(d[0]), ay = std::abs(d[1]), az = std::abs(d[2]);
        require(ax <= 64 && ay <= 64 && az <= 64, "offset too large");
        DeviceScope ds(ctx->device);
        // octant table covering |d|, then the reflection rule of the MAC loader
        SpecTable t;
        const int N = 2 * nb, H = nb + 1;
        const size_t n_freq = (size_t)N * N * H;
        const size_t n_off = (size_t)(ax + 1) * (ay + 1) * (az + 1);
        t.data.alloc(ctx, 16 * n_off * n_freq, "spectrum");
        DeviceBuffer scratch;
        scratch.alloc(ctx, 16 * n_freq * std::min<size_t>(n_off, 512), "spectrum scratch");
        hip_check(build_spectra((const double *)ctx->gcube.ptr, true, 1, 0, 0, nb, ax, ay, az, false, t.data.ptr, scratch.ptr,
                                scratch.bytes, ctx->stream),
                  "build_spectra");
        hip_check(hipStreamSynchronize(ctx->stream), "sync");
        const size_t o = ((size_t)ay * (az + 1) + az) * (ax + 1) + ax;
        std::vector<double> all(2 * n_off * n_freq);
        hip_check(hipMemcpy(all.data(), t.data.ptr, all.size() * 8, hipMemcpyDeviceToHost), "download");
        const bool fx = d[0] < 0, fy = (d[1] < 0) != fx, fz = (d[2] < 0) != fx;
        for (int kz = 0; kz < N; ++kz)
            for (int ky = 0; ky < N; ++ky)
                for (int kx = 0; kx < H; ++kx) {
                    const int ky2 = fy ? (N - ky) % N : ky, kz2 = fz ? (N - kz) % N : kz;
                    const size_t w = ((size_t)kz * N + ky) * H + kx, w2 = ((size_t)kz2 * N + ky2) * H + kx;
                    out[2 * w] = all[2 * (w2 * n_off + o)];
                    out[2 * w + 1] = fx ? -all[2 * (w2 * n_off + o) + 1] : all[2 * (w2 * n_off + o) + 1];
                }
    });
}

lgf_status lgf_context_set_timing(lgf_context *ctx, int enable) {
    return guard([&] {
        require(ctx != nullptr, "null context");
        ctx->timing = enable != 0;
    });
}

lgf_status lgf_context_stage_times(lgf_context *ctx, double *ms, int64_t *launches) {
    return guard([&] {
        require(ctx && ms && launches, "null arguments");
        DeviceScope ds(ctx->device);
        resolve_stage_times(ctx, ms, launches);
    });
}

lgf_status lgf_context_set_mac_method(lgf_context *ctx, int method) {
    return guard([&] {
        require(ctx != nullptr, "null context");
        require(method == LGF_MAC_AUTO || method == LGF_MAC_PAIRS || method == LGF_MAC_LATTICE,
                "unknown MAC method");
        ctx->mac_method = method;
    });
}

lgf_status lgf_context_set_lattice_passes(lgf_context *ctx, int passes) {
    return guard([&] {
        require(ctx != nullptr, "null context");
        require(passes == 1 || passes == 3, "lattice passes must be 1 or 3");
        ctx->lat_passes = passes;
    });
}

lgf_status lgf_context_set_autotune(lgf_context *ctx, int reps) {
    return guard([&] {
        require(ctx != nullptr, "null context");
        require(reps >= 0 && reps <= 1000, "autotune repetitions must be in [0, 1000]");
        ctx->autotune_reps = reps;
    });
}

lgf_status lgf_context_save_tuning(lgf_context *ctx, const char *path) {
    return guard([&] {
        require(ctx && path, "null arguments");
        std::string text;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            text = tuning_to_json(ctx->tune);
        }
        FILE *fp = std::fopen(path, "w");
        if (!fp) throw Failure(LGF_E_INVALID, std::string("cannot open ") + path + " for writing");
        const size_t n = std::fwrite(text.data(), 1, text.size(), fp);
        const int rc = std::fclose(fp);
        if (n != text.size() || rc != 0) throw Failure(LGF_E_INVALID, std::string("write failed: ") + path);
    });
}

lgf_status lgf_context_load_tuning(lgf_context *ctx, const char *path) {
    return guard([&] {
        require(ctx && path, "null arguments");
        std::ifstream in(path, std::ios::binary);
        if (!in) throw Failure(LGF_E_INVALID, std::string("cannot open ") + path);
        std::ostringstream ss;
        ss << in.rdbuf();
        std::map<std::string, TuneEntry> got = tuning_from_json(ss.str());
        std::lock_guard<std::mutex> lk(ctx->mu);
        for (auto &kv : got) ctx->tune[kv.first] = kv.second;
    });
}

lgf_status lgf_context_tuning_size(lgf_context *ctx, int64_t *n_entries) {
    return guard([&] {
        require(ctx && n_entries, "null arguments");
        std::lock_guard<std::mutex> lk(ctx->mu);
        *n_entries = (int64_t)ctx->tune.size();
    });
}

const char *lgf_last_error(void) { return g_last_error.c_str(); }

#ifndef LGF_SOURCE_SHA256
#define LGF_SOURCE_SHA256 "unknown"
#endif

const char *lgf_build_id(void) { return "sha256=" LGF_SOURCE_SHA256 " arch=gfx950"; }

const char *lgf_status_string(lgf_status s) {
    switch (s) {
    case LGF_OK: return "LGF_OK";
    case LGF_E_INVALID: return "LGF_E_INVALID";
    case LGF_E_NOMEM: return "LGF_E_NOMEM";
    case LGF_E_DEVICE: return "LGF_E_DEVICE";
    case LGF_E_UNSUPPORTED: return "LGF_E_UNSUPPORTED";
    }
    return "unknown status";
}

}  // extern "C"
