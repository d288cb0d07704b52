// Internal runtime types behind include/lgf.h.
#pragma once
#include <hip/hip_runtime.h>

#include <array>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/lgf.h"
#include "lgf_kernels.hpp"

namespace lgf {

extern thread_local std::string g_last_error;
// While set on a thread, launches record no stage-timing events.
extern thread_local bool g_no_timing;
void set_error(const std::string &m);

struct Failure : std::runtime_error {
    lgf_status status;
    Failure(lgf_status s, const std::string &m);
};

void hip_check(hipError_t e, const char *what);

// components that share one spectral-MAC launch (the MAC's right-hand sides)
constexpr int kMacComponents = 3;

struct lgf_context_impl;
}  // namespace lgf

struct lgf_context;

namespace lgf {

// Device allocation accounted against a context's HBM budget.
struct DeviceBuffer {
    void *ptr = nullptr;
    size_t bytes = 0;
    lgf_context *owner = nullptr;
    DeviceBuffer() = default;
    DeviceBuffer(const DeviceBuffer &) = delete;
    DeviceBuffer &operator=(const DeviceBuffer &) = delete;
    ~DeviceBuffer();
    void alloc(lgf_context *ctx, size_t n, const char *what);
    void release();
};

// The kernel of a convolution: the LGF (a = 0) or the integrating factor
// E(a) (a > 0), sampled at stride * n, and all block offsets (band 0), only
// those with max |d_i| <= D (band 1, near) or only those beyond (band 2, far).
struct KernelId {
    double a = 0.0;
    int stride = 1;
    int band = 0;
    int D = 0;
    bool operator==(const KernelId &o) const {
        return a == o.a && stride == o.stride && band == o.band && (band == 0 || D == o.D);
    }
};

struct SpecTable {
    int nb = 0;
    bool fp32 = false;
    KernelId ka;            // the kernel whose windows the table holds
    int XH = 0, YH = 0, ZH = 0;
    int n_freq = 0;
    DeviceBuffer data;
    DeviceBuffer perm;      // frequency order grouping (ky, kz) reflection partners
};

// Event pair around one kernel launch, resolved lazily.
struct StageEvent {
    int stage;
    hipEvent_t a, b;
};

// Pinned-host / device staging ring for the job tables of batched launches.
struct JobRing {
    static constexpr int kSlots = 32;
    static constexpr size_t kSlotBytes = 256 << 10;
    std::mutex mu;
    void *host = nullptr;           // hipHostMalloc, kSlots * kSlotBytes
    void *dev = nullptr;            // hipMalloc, same size
    hipEvent_t done[kSlots] = {};
    int next = 0;
};

// Real lattice spectra Khat[omega_r][kx][kz][ky] of the stored frequencies
// for lattice DFT lengths (lx, ly, lz) (lgf_lattice.hip), shared by every
// plan of the context.
struct LatSpec {
    int nb = 0;
    bool fp32 = false;
    KernelId ka;                  // kernel, as SpecTable::ka
    int lx = 0, ly = 0, lz = 0;
    int n_freq = 0;
    DeviceBuffer data;
    DeviceBuffer order_buf;       // the octant table's reflection-grouped order, as spectrum positions
    const int *order = nullptr;   // order_buf
};

// Tuning-table entry: the chosen MAC method ("pairs TYxTZ": the block-pair
// kernel with that tile shape, or "lattice"), and every candidate timed
// with its milliseconds per launch.
struct TuneEntry {
    std::string choice;
    std::vector<std::string> cand;
    std::vector<double> ms;
};
// "pairs TYxTZ" -> (ty, tz) and false; "lattice" -> true; anything else throws
bool parse_choice(const std::string &s, int &ty, int &tz);
// The table as JSON and back (lgf_tuning.cpp); the reader throws Failure
// (LGF_E_INVALID) on malformed text.
std::string tuning_to_json(const std::map<std::string, TuneEntry> &table);
std::map<std::string, TuneEntry> tuning_from_json(const std::string &text);

struct lgf_context_impl {
    int device;
    bool timing = false;
    int autotune_reps = 0;                       // > 0: time MAC candidates for new shapes
    int mac_method = LGF_MAC_AUTO;               // lgf_mac_method
    int lat_passes = 3;                          // lattice FFT split: 3, or 1 where the lengths allow
    std::map<std::string, TuneEntry> tune;       // shape key -> tile shape (guarded by mu)
    JobRing ring;
    std::vector<StageEvent> pending;
    size_t budget;
    size_t used = 0;
    hipStream_t stream = nullptr;
    DeviceBuffer gcube;
    std::vector<std::unique_ptr<SpecTable>> tables;
    std::vector<std::unique_ptr<LatSpec>> lat_tables;
    std::map<double, std::unique_ptr<DeviceBuffer>> if_cubes;   // integrating-factor kernels by a
    std::mutex mu;
    lgf_context_impl(int dev, size_t budget_);
};

// A block of one level: lattice block coordinates and the element offset of
// its first cell inside one component's field (or a workspace field).
struct Blk {
    int ijk[3];
    int64_t off;
};

// One (target x-segment, source x-segment) part of a convolution, run by the
// bx-wide MAC template: targets at x in [tx0, tx0 + bx), sources at x in
// [sx0, sx0 + bx) of the padded box.
struct SubConv {
    int tx0 = 0, sx0 = 0;
    int phase = 0;          // parts of one target segment run in different phases
    bool accum = false;     // add into Uhat (an earlier phase stored the segment)
    bool sparse = false;    // source rows have holes: the MAC skips empty positions
    int n_rows = 0, n_tiles = 0;
    DeviceBuffer d_rows, d_tiles, d_lanes;
};

// One blockwise LGF convolution on a level (sources -> targets).  The
// spectral MAC runs either as block pairs (parts, below) or, for boxes of at
// most 32 blocks along x and y and 64 along z, as an FFT over the block
// lattice (method 1).
constexpr int kMethodPairs = 0, kMethodLattice = 1;
struct Conv {
    int method = kMethodPairs;
    int lx = 0, ly = 0, lz = 0;     // lattice DFT lengths (method 1)
    LatSpec *lspec = nullptr;       // lattice spectra (method 1)
    bool lat_fused = false;         // method 1 in one pass per frequency (lattice_fused)
    int bx = 0;             // MAC row template (8 or 16)
    int ty = 0, tz = 0;     // MAC tile shape in rows
    int axis = 0;           // rows along lattice x (0) or y (1)
    int rs = 0;             // slots per row of the padded box: a multiple of bx (method 1: the box extent)
    int ey = 0, ez = 0;
    int lo[3] = {0, 0, 0};
    int64_t n_slots = 0;
    bool fp32 = false;
    int n_src = 0, n_tgt = 0;
    SpecTable *spec = nullptr;
    DeviceBuffer d_src_slot, d_tgt_slot, d_src_off, d_tgt_off;
    DeviceBuffer d_src_occ;   // lattice: 1 per source slot of the box (absent when every slot has a source)
    std::vector<std::unique_ptr<SubConv>> parts;   // in phase order
};

// One L_dx^-1 application on a source and a target block set: a plain
// float64 convolution, or the float32 + float64-refinement sequence.
struct ConvOp {
    bool refined = false;
    // plain: sources -> targets.  refined: the cut (depth <= 2 cells of the
    // shell blocks) and the sources outside T -> targets, in float64, split
    // into rows along x (c64) and rows along y (c64y); either may be null
    std::unique_ptr<Conv> c64, c64y;
    // refined: u~ (sources -> T) and the float32 residual (T -> targets)
    std::unique_ptr<Conv> c32, ccorr;
    int n_t = 0, n_sh = 0, n_out = 0;
    RefGeom geom{};
    DeviceBuffer d_map, d_tblk, d_t2sh, d_depth, d_gofs, d_dofs, d_out_src, d_out_dst;
};

// Spectral workspace of a solve: Fhat, Uhat (mac_nc component regions each)
// and the lattice workspace H.  By default the plan's own buffers; the
// static-scratch solve points them into the library's device array.
struct SpecWs {
    void *fhat = nullptr, *uhat = nullptr, *lat = nullptr;
    size_t fhat_bytes = 0, uhat_bytes = 0, lat_bytes = 0;
};

// Per-level schedule data of a composite plan.
struct LevelSched {
    int n_own = 0;
    bool any_cover = false;
    DeviceBuffer d_cmask;                            // the level's cell mask ([block][nb^3]), if given
    DeviceBuffer d_cover, d_own_off;                 // level blocks: octant cover bits, field offsets
    int n_cf = 0;
    DeviceBuffer d_cf_fine, d_cf_coarse, d_cf_oct;   // coarsening pairs from level k+1
    int n_ext = 0;
    DeviceBuffer d_fblk, d_ext_own;                  // R_k blocks and their own-level offsets (or -1)
    int n_dom = 0;                                   // dom(psi_k) blocks
    CorrGeom corr{};                                 // map of dom(psi_{k-1}) for this level's correction
    DeviceBuffer d_cmap;
    DeviceBuffer d_cu_src, d_cu_dst, d_cp_src, d_cp_dst;
    std::unique_ptr<ConvOp> convF, convPsi;
};

SpecTable *get_spectra(lgf_context *ctx, int nb, bool fp32, int XH, int YH, int ZH, const KernelId &ka);
LatSpec *get_lat_spectra(lgf_context *ctx, int nb, bool fp32, int lx, int ly, int lz, const KernelId &ka);
LatGeom lat_geom(const Conv &c, int nc);
// The lattice MAC of c (method 1) on the stream: Fhat -> Uhat through the
// workspace lat (H, or the second term of the one-pass split, which is then
// returned: the inverse block FFT adds it; else null).
const void *lattice_mac(lgf_context *ctx, const Conv &c, const LatGeom &g, const void *fhat, void *lat, void *uhat,
                        hipStream_t s);
// every slot of the convolution holds a source block: its forward FFTs
// write the whole spectral region it reads
inline bool fhat_full(const Conv &c) { return (int64_t)c.n_src == c.n_slots; }
SmacGeom conv_geom(const Conv &c, const SubConv &p);
// Factor of the spectral convolution's result: dx^2 for L_dx^-1 = dx^2 G *,
// 1 for the integrating factor (its kernel already carries dx through a).
inline double conv_scale(const lgf_plan *p, double dx);

}  // namespace lgf

struct lgf_context : lgf::lgf_context_impl {
    using lgf::lgf_context_impl::lgf_context_impl;
};

struct lgf_plan {
    lgf_context *ctx = nullptr;
    int K = 1, nb = 16, nc = 1, prec = 0, ne = 1;
    double dx0 = 1.0;
    std::vector<std::vector<lgf::Blk>> levels;     // per level, offsets within one component
    std::vector<std::vector<uint8_t>> cell_mask;   // per level: the caller's cell mask, or empty
    lgf::DeviceBuffer d_cmask0, ws_masked;         // single level with a mask: the mask, the masked source
    std::vector<int64_t> level_base;               // element offset of each level in a component
    int64_t comp_len = 0;                          // elements per component
    std::unique_ptr<lgf::ConvOp> op0;                       // single-level plans
    std::vector<std::unique_ptr<lgf::LevelSched>> lv;       // composite plans
    std::vector<const lgf::Conv *> convs_view;              // every convolution of the plan
    lgf::DeviceBuffer ws_fhat, ws_F, ws_psi[2], ws_ppsi, ws_srcF, ws_srcf;
    lgf::DeviceBuffer ws_ut, ws_ush, ws_rho;               // refinement workspaces
    int mac_nc = 1;                                // components per MAC launch: min(nc, 3)
    int64_t ut_len = 0, cut_len = 0;               // elements per component in ws_ut / ws_rho and ws_ush
    int64_t dom_len = 0, ext_len = 0;              // elements per component in ws_psi and ws_ppsi / ws_src*
    lgf::DeviceBuffer Fhat, Uhat;                  // mac_nc component regions each
    lgf::DeviceBuffer ws_lat;                      // lattice-DFT workspace H, mac_nc regions
    const lgf::Conv *fhat_conv = nullptr;          // conv whose slot map Fhat currently holds
    const lgf::SpecWs *ws_scratch = nullptr;       // set only during a static-scratch solve
    double if_a0 = 0.0;                            // > 0: integrating-factor plan, a on level 0 (a_k = 4^k a0)
    lgf::KernelId kernel0;                         // kernel of the plan's level-0 convolutions
    lgf::KernelId build_ka;                        // kernel of the convolutions being built
    int flgf_D = -1;                               // >= 0: two-grid fast-LGF plan with near radius D blocks
    std::unique_ptr<lgf_plan> flgf_coarse;         // its far field on the node lattice (nb/2 per block)
    lgf::DeviceBuffer ws_fc, ws_uc;                // node-lattice source and result
    int n_q0 = 0;                                  // integrating factor, composite: level-0 blocks in dom(psi_0)
    lgf::DeviceBuffer d_q0_src, d_q0_dst;
    lgf::DeviceBuffer d_blk_off, d_blk_back;       // single level: block offsets; with 3 components also the
                                                   // offsets of the blocks one back along x, y, z (or -1)
    // refinement indicator: the source blocks R_k of every level (level 0:
    // its blocks; k >= 1: its blocks dilated by ne layers) and, while
    // `collect` is set, per (component, level, R_k block) the sum of squares
    // and max |.| of the combined source of the level's phi convolution
    std::vector<std::vector<int32_t>> src_ijk;
    std::vector<int64_t> ind_base;
    int64_t ind_total = 0;
    lgf::DeviceBuffer d_ind;
    bool collect = false;
    size_t workspace_bytes() const;
};

namespace lgf {
inline double conv_scale(const lgf_plan *p, double dx) { return p->if_a0 > 0.0 ? 1.0 : dx * dx; }
// Timed stages: block FFT forward, block-pair MAC, block FFT inverse, other,
// lattice x DFTs, lattice y/z slabs (DFTs, product, inverse DFTs), lattice
// inverse x DFTs.
constexpr int kStages = 8;
enum { kStageFwd = 0, kStagePairs = 1, kStageInv = 2, kStageOther = 3, kStageLatX = 4, kStageLatYZ = 5,
       kStageLatInv = 6, kStageLatFused = 7 };
// Records an event before/after a stage launch when timing is on.
struct StageTimer {
    lgf_context *ctx;
    int stage;
    hipStream_t s;
    hipEvent_t a = nullptr;
    StageTimer(lgf_context *c, int st, hipStream_t s_);
    ~StageTimer();
};
void resolve_stage_times(lgf_context *ctx, double *ms, int64_t *launches);
void ring_init(lgf_context *ctx);
void ring_free(lgf_context *ctx);
void build_context_table(lgf_context *ctx);
void build_schedule(lgf_plan *plan);
void run_plan(lgf_plan *plan, const double *f, double *u, hipStream_t s, lgf_report *rep);
hipGraph_t capture_solve(lgf_plan *plan, const double *f, double *u);
// While set on a thread (batch capture), batched launches stage their job
// tables into new device buffers appended here instead of the ring.
extern thread_local std::vector<std::unique_ptr<DeviceBuffer>> *g_job_sink;
hipGraph_t capture_batch(lgf_context *ctx, int n, lgf_plan *const *plans, const double *const *f, double *const *u,
                         std::vector<std::unique_ptr<DeviceBuffer>> &tables);
void run_batch(lgf_context *ctx, int n, lgf_plan *const *plans, const double *const *f, double *const *u,
               hipStream_t s, lgf_report *reps);
void build_conv(lgf_plan *plan, Conv &c, const std::vector<Blk> &src, const std::vector<Blk> &tgt, bool fp32,
                int axis = 0);
void plan_alloc_spectral(lgf_plan *plan);
// Bytes of Fhat / Uhat / H every convolution of the plan needs (pointers null).
SpecWs spectral_need(const lgf_plan *plan);
std::unique_ptr<ConvOp> build_op(lgf_plan *plan, const std::vector<Blk> &src, const std::vector<Blk> &tgt, bool refine);
// Refinement workspaces (per component region) for the plan's refined ops.
void plan_alloc_refine(lgf_plan *plan, const std::vector<const ConvOp *> &ops);
// One component's residual step of a refined op: w into dst, rin / cut from
// ut (see lgf_refine.hip); ut, rin, cut are that component's regions.
void refine_middle(lgf_plan *plan, const ConvOp &op, const double *src, double *dst, const double *ut, double *rin,
                   double *cut, double dx, int accumulate, hipStream_t s);
// dst (+)= dx^2 G * src for nc components (component c at src + c*sstride,
// dst + c*dstride); groups of up to kMacComponents share one MAC launch.
void run_op(lgf_plan *plan, const ConvOp &op, const double *src, int64_t sstride, double *dst, int64_t dstride,
            int nc, double dx, int accumulate, hipStream_t s);
void run_conv(lgf_plan *plan, const Conv &c, const double *src, int64_t sstride, double *dst, int64_t dstride,
              int nc, double dx, int accumulate, hipStream_t s);
}  // namespace lgf
