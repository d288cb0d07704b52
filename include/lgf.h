/*
 * lgf.h -- C ABI of the MI355X (gfx950) lattice-Green's-function Poisson
 * library (liblgf.so).
 *
 * What it computes.  Yu, Dorschner & Colonius, "Multi-resolution lattice
 * Green's function method for incompressible flows":
 *   - Sec. 2.2, eqs. discrete_laplace / lgf_convolution: on an unbounded
 *     Cartesian lattice of spacing dx, the decaying solution of the 7-point
 *     Poisson problem  dx^-2 (sum_{+-e_i} u(n +- e_i) - 6 u(n)) = f(n)  is
 *     u = dx^2 * (G * f), G the lattice Green's function (LGF).
 *   - Sec. 3.4, eqs. AMR-LGF-2 ... FLGF-AMR: on a composite mesh of levels
 *     k = 0..K-1 (dx_k = dx0 / 2^k) the solution returned is
 *     phi^ = [Gamma L^-1 P] f^  -- every level solved with its own LGF, the
 *     coarse levels' contributions carried to finer levels by interpolation
 *     plus the correction source S (eq. source_correct), and the result
 *     restricted to each level's region Omega_k.
 *
 * Support.  The source support and the evaluation targets of level k are
 * the cells of a list of occupied blocks of nb^3 cells (nb = 8 or 16).  Block
 * (bx, by, bz) of level k holds lattice cells (bx*nb + x, by*nb + y, bz*nb + z),
 * x, y, z in [0, nb).  Level k+1 blocks must lie inside level-k blocks (each
 * fine block's parent octant belongs to a level-k block).  Omega_k is the
 * set of level-k cells not covered by a level-(k+1) block.
 *
 * Field layout (f and u).  One float64 array per call:
 *   [component][level][block][z][y][x],  x fastest,
 * blocks of a level in the order the plan was given them.  Cells of a
 * level-k block that are covered by finer blocks are ignored on input and
 * written as 0 on output.
 *
 * Ownership.  f and u are device pointers owned by the caller (e.g. PyTorch
 * tensors on the plan's device); the library never frees them.  Host arrays
 * passed to lgf_plan_create are copied.  Contexts and plans are opaque,
 * created and destroyed only through this API.
 *
 * Errors.  No C++ exception crosses the ABI.  Each call returns an
 * lgf_status; on failure lgf_last_error() (thread-local) holds a message.
 */
#ifndef LGF_H
#define LGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lgf_status {
    LGF_OK = 0,
    LGF_E_INVALID = 1,      /* bad argument, malformed block list        */
    LGF_E_NOMEM = 2,        /* HBM budget or device allocation exceeded  */
    LGF_E_DEVICE = 3,       /* a HIP runtime call failed                  */
    LGF_E_UNSUPPORTED = 4   /* a valid request this build does not serve */
} lgf_status;

typedef enum lgf_precision {
    LGF_FP64 = 0,           /* every step in float64                       */
    LGF_FP32_REFINE = 1     /* float32 block FFTs and spectral products,
                               float64 residual and accumulation           */
} lgf_precision;

typedef struct lgf_context lgf_context;
typedef struct lgf_plan lgf_plan;

/*
 * One refinement level: n_blocks block coordinates, [n_blocks][3] (x, y, z),
 * and an optional cell mask that states the level's part Omega_k of the
 * partition of Sec. 3.1 (eq. partition) cell by cell: [n_blocks][nb^3] bytes
 * in the field's [z][y][x] order, 1 = the cell belongs to Omega_k (its
 * source is used, its solution written), 0 = it does not (its source is
 * ignored and 0 is written).  NULL: Omega_k = every cell of the level's
 * blocks that no level-(k+1) block covers.  A mask may drop further cells
 * but may not keep a covered one: a 1 on a cell under a level-(k+1) block
 * makes the levels overlap and is refused (LGF_E_INVALID), as are values
 * other than 0 and 1.
 */
typedef struct lgf_level {
    int32_t n_blocks;
    const int32_t *block_ijk;
    const uint8_t *cell_mask;
} lgf_level;

/* Problem description (Sec. 3.1 composite grid, Sec. 5 block structure). */
typedef struct lgf_problem {
    int32_t n_levels;       /* K >= 1                                       */
    int32_t nb;             /* block edge in cells: 8 or 16                 */
    double dx0;             /* cell width of level 0 (> 0)                  */
    int32_t n_components;   /* 1..8 fields on the same support (3: vector) */
    int32_t precision;      /* an lgf_precision value                       */
    int32_t ne_blocks;      /* extended-correction layers in blocks (>= 1;
                               0 selects the default 1, i.e. N_E = nb)       */
    const lgf_level *levels;/* n_levels entries, coarsest first             */
} lgf_problem;

/* Optional per-solve report, filled after the solve's stream work is done. */
typedef struct lgf_report {
    double device_ms;       /* stream time of the solve (HIP events)        */
    double refine_rel_l2;   /* reserved: written as 0                      */
    int32_t passes;         /* LGF convolutions run per component           */
    int32_t reserved;
} lgf_report;

/*
 * Create a context on HIP device `device`.  The context owns the device-
 * resident LGF table (built here, in float64: the exact near field and the
 * asymptotic far field that Sec. 5 of the paper tabulates once and shares
 * between levels, since the 7-point LGF is the same on every level) and the
 * cache of LGF block spectra shared by every plan made from it.  `hbm_budget_bytes` caps what
 * plans and spectra may allocate (0 = no cap).  Errors: LGF_E_INVALID
 * (bad device or null out), LGF_E_DEVICE.
 */
lgf_status lgf_context_create(int device, size_t hbm_budget_bytes, lgf_context **out);
void lgf_context_destroy(lgf_context *ctx);

/* Bytes of device memory currently held by the context and its plans. */
size_t lgf_context_bytes(const lgf_context *ctx);

/*
 * Build an immutable plan for one support (all levels).  Validates the block
 * lists (duplicates, nesting, sizes -> LGF_E_INVALID), builds any LGF block
 * spectra missing from the context cache, and allocates the plan's
 * workspace (-> LGF_E_NOMEM if the budget would be exceeded).  Work runs on
 * the context's own stream and is complete when this returns.
 */
lgf_status lgf_plan_create(lgf_context *ctx, const lgf_problem *desc, lgf_plan **out);

/*
 * Integrating factor (Sec. 2.3, eqs. heat, IF-single; Sec. 3.5, eq.
 * FIF-AMR).  A plan whose solves apply H(a) = exp(a L), the solution
 * operator of the discrete heat equation over a time kappa (t - tau), with
 * a = kappa (t - tau) / dx^2 for the unscaled 7-point L, instead of L^-1:
 * u = E * f with the kernel E(n) = prod_i e^{-2a} I_{n_i}(2a) (tabulated in
 * float64 on the device for |n_i| <= lgf_table_radius(), 0 beyond, where it
 * is below 1e-300 for any a of interest).  a0 is a on level 0; level k uses
 * a_k = 4^k a0 (dx_k = dx0 / 2^k).  On a composite mesh the solve returns
 * Gamma H P f^: per level k the composite source on the level's blocks and
 * the extended region (the cumulative F_k plus the interpolation of the
 * coarser levels' sources, q_0 = f^_0, q_k = P q_{k-1} + f^_k), convolved
 * with E(a_k) and restricted to Omega_k.  The plan is used with lgf_solve,
 * lgf_solve_scratch, lgf_solve_batch (composite integrating-factor plans run
 * one after another inside a batch) and the graph calls.  precision must be
 * LGF_FP64 (else LGF_E_UNSUPPORTED); other errors as lgf_plan_create, and
 * LGF_E_INVALID for a0 not in (0, 1e6].
 */
lgf_status lgf_plan_create_if(lgf_context *ctx, const lgf_problem *desc, double a0, lgf_plan **out);

/*
 * Fast-LGF far-field approximation (Sec. 2.2 and Sec. 5: the paper sums the
 * LGF convolution with a fast multipole-type method on the block octree;
 * this is a two-grid reading of it).  Block pairs within near_blocks blocks
 * (max_i |t_i - s_i| <= near_blocks) are summed exactly; for the other pairs
 * the kernel is replaced by its cubic interpolation from a lattice of nodes
 * twice as coarse, (nb/2)^3 nodes per block at fine positions 2k + 1, every
 * block interpolating from its own nodes (the 4 nearest per axis, the window
 * kept inside the block):  u = u_near + I (G2_far * (A f)) with A = I^T
 * (anterpolation) and G2_far the LGF at the even lattice vectors between
 * nodes of far blocks, convolved over the node lattice by the same block
 * engine (blocks of nb/2).  Not exact: the error falls roughly with the
 * fourth power of the near radius; lgf_solve of a plan made by
 * lgf_plan_create gives the exact sum.  Single-level problems of 16^3
 * blocks in float64 without cell masks only (else LGF_E_UNSUPPORTED or
 * LGF_E_INVALID); near_blocks in [0, 8].  The plan is used with lgf_solve,
 * lgf_solve_scratch, lgf_solve_batch (it runs its own steps inside a batch)
 * and the graph calls.
 */
lgf_status lgf_plan_create_flgf(lgf_context *ctx, const lgf_problem *desc, int near_blocks, lgf_plan **out);

/*
 * Validate a problem description on the host only (no device work): the
 * same checks lgf_plan_create applies before it builds anything.  Returns
 * LGF_OK or LGF_E_INVALID with the reason in lgf_last_error().
 */
lgf_status lgf_problem_check(const lgf_problem *desc);
void lgf_plan_destroy(lgf_plan *plan);

/* Device bytes the plan's workspace holds (excluding shared spectra). */
size_t lgf_plan_workspace_bytes(const lgf_plan *plan);

/* Cells of level `level` (n_blocks * nb^3), i.e. the per-component length. */
size_t lgf_plan_cells(const lgf_plan *plan, int level);

/* Total float64 elements of f / u for this plan (all components, levels). */
size_t lgf_plan_field_len(const lgf_plan *plan);

/*
 * Solve (Sec. 2.2 one level, Sec. 3.4 composite).  f, u: device float64
 * arrays of lgf_plan_field_len() elements in the layout above; u is
 * overwritten.  Asynchronous on HIP stream `stream` (a hipStream_t; NULL =
 * the null stream).  If `rep` is non-null the call waits for its own work
 * and fills the report.  Errors: LGF_E_INVALID (null/misaligned pointers),
 * LGF_E_DEVICE.  Calls that share a plan must not overlap in time: the plan
 * owns one workspace.
 */
lgf_status lgf_solve(lgf_plan *plan, const double *f, double *u, void *stream,
                     lgf_report *rep);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as lgf_solve(plan, f, u, stream, NULL), bit for bit, with the
 * spectral workspace of every convolution (block spectra Fhat and Uhat and
 * the lattice workspace) taken from a static device array of
 * LGF_SCRATCH_MAX_BYTES bytes that the library holds on each device until
 * the process ends, instead of from the plan.  The call allocates nothing
 * and records no timing events; the plan's other workspaces (composite and
 * refinement fields) are its own, allocated by lgf_plan_create.
 * Limit: a plan whose Fhat + Uhat + lattice workspace (each rounded up to
 * 256 bytes) exceed LGF_SCRATCH_MAX_BYTES is refused with LGF_E_INVALID
 * before any device work.  Every such call on one device shares the one
 * array, which keeps the last call's contents (the call clears what must
 * start at zero): calls that overlap in time on one device race, whatever
 * their plans, streams or threads, so the caller orders them (one stream,
 * or events).  The context of the plan must have been created on the device
 * (lgf_context_create looks the array's device address up).
 */
#define LGF_SCRATCH_MAX_BYTES (64u << 20)
lgf_status lgf_solve_scratch(lgf_plan *plan, const double *f, double *u, void *stream);

/*
 * Velocity refresh (Sec. 4.1, eq. vel_update): u = -C^dagger L_E^-1 omega on
 * one level, the velocity recovered from the vorticity on the base level.
 * plan: a single-level plan with n_components = 3.  Staggering (Sec. 2.1:
 * vectors on the positive faces and edges of each cell): component c of a
 * field at cell n is the value on the c-edge (omega, psi) or c-face (u)
 * that cell owns, n + (e - e_c)/2 resp. n + e_c/2 with e = (1, 1, 1).
 * omega: device float64 edge vorticity in the plan's field layout
 * ([component][block][z][y][x]).  psi: caller-owned device array of the same
 * size that receives the streamfunction L_E^-1 omega (the LGF solve of every
 * component, as lgf_solve).  u: caller-owned device array of the same size
 * that receives -C^dagger psi, the curl from edges to faces with backward
 * differences scaled by 1/dx0 (the adjoint of the forward-difference curl C
 * of eq. mimetic).  A u component whose stencil needs psi one cell back in a
 * block outside the support is written as NaN.  omega, psi and u must be
 * distinct.  Asynchronous on `stream`.  Errors: LGF_E_INVALID (plan shape,
 * null, misaligned or aliased pointers), LGF_E_DEVICE.
 */
lgf_status lgf_velocity_refresh(lgf_plan *plan, const double *omega, double *psi, double *u, void *stream);

/*
 * Refinement indicator (Sec. 4.2, eqs. refine1, maximumS, refine2): the
 * criterion is evaluated on the combined source S_k of eq. combined_source,
 * the right-hand side of level k's phi convolution (k = 0: the cumulative
 * source F_0; k >= 1: S_k + F_k on the level's source blocks R_k, its blocks
 * and the extended correction region).
 *
 * lgf_plan_source_blocks: the blocks of R_k ([n][3] block coordinates of
 * level k, the level's blocks for k = 0, the level's blocks dilated by
 * ne_blocks layers for k >= 1, in the plan's order) into ijk (if non-null);
 * returns n, or -1 for a bad plan or level.
 *
 * lgf_solve_indicator: lgf_solve(plan, f, u, stream, NULL), and on the way,
 * per component, level and R_k block (host arrays of n_components *
 * sum_k n_k entries, [component][level][block]), the root mean square of
 * the combined source over the block's cells into block_rms and its largest
 * magnitude into block_max.  On one level S is the source f itself.  The
 * call waits for its stream.  Errors: LGF_E_INVALID (null or misaligned
 * pointers), LGF_E_DEVICE.
 */
int64_t lgf_plan_source_blocks(const lgf_plan *plan, int level, int32_t *ijk);
lgf_status lgf_solve_indicator(lgf_plan *plan, const double *f, double *u, void *stream, double *block_rms,
                               double *block_max);

/*
 * Solve n independent requests (each the problem of lgf_solve: Sec. 2.2 on
 * one level, the Sec. 3.4 recursion on a composite mesh) together.  Per block
 * size, the single-level requests run component by component, and the
 * composite ones level by level in the paper's order (every request's
 * restriction and coarsening; then for k = 0, 1, ...: every request's
 * correction source of level k, the phi_k convolutions of all requests,
 * their psi_k convolutions, the restriction).  Within one such step the
 * forward block FFTs of all requests run as one launch per precision, the
 * block-pair spectral products as one launch per (phase, precision, tile
 * shape, sparsity), the inverse block FFTs as one launch per precision;
 * lattice-FFT products and the stencil steps run per request.  These are
 * ordinary grids over a job table, not a persistent kernel, and the batch is
 * not captured into a graph (lgf_graph_create captures one plan's solve).
 * Each u[i] equals what lgf_solve(plans[i], f[i], u[i], ...) writes, bit for
 * bit (every request's reduction order is fixed by its own plan).  The
 * plans must be distinct and come from `ctx`.  `reps` (optional) has n
 * entries; each gets the device time of the whole batch.
 */
lgf_status lgf_solve_batch(lgf_context *ctx, int n, lgf_plan *const *plans,
                           const double *const *f, double *const *u, void *stream,
                           lgf_report *reps);

/*
 * Graph form of lgf_solve for fixed buffers: lgf_graph_create records every
 * launch of one lgf_solve(plan, f, u) into a HIP graph (captured on a
 * private stream; the device pointers f and u are bound into it) and
 * instantiates it; lgf_graph_launch replays the whole solve on `stream` with
 * one call, so repeated solves of one shape pay no per-kernel launch cost.
 * The graph reads f and writes u at replay time, so the caller refreshes f in
 * place between replays.  The plan must outlive the graph, and replays and
 * solves of one plan must not overlap in time (one workspace).  Errors of
 * create: LGF_E_INVALID (null/misaligned pointers), LGF_E_DEVICE (capture or
 * instantiation failed).  Timing (lgf_context_set_timing) does not see
 * graph replays.
 */
typedef struct lgf_graph lgf_graph;
lgf_status lgf_graph_create(lgf_plan *plan, const double *f, double *u, lgf_graph **out);
/*
 * Graph form of lgf_solve_batch: records one lgf_solve_batch(ctx, n, plans,
 * f, u, ...) on fixed buffers (the launches of every level and stage of
 * every request, in the batch's order) into one HIP graph; each
 * lgf_graph_launch replays the whole batch with one call.  The job tables of
 * the batched launches are copied at capture into device buffers owned by
 * the graph, so replays need no host staging.  Results equal
 * lgf_solve_batch bit for bit.  The plans and the context must outlive the
 * graph; replays must not overlap in time with each other or with other
 * uses of the same plans.  Errors as lgf_solve_batch and lgf_graph_create.
 */
lgf_status lgf_graph_create_batch(lgf_context *ctx, int n, lgf_plan *const *plans, const double *const *f,
                                  double *const *u, lgf_graph **out);
lgf_status lgf_graph_launch(lgf_graph *graph, void *stream);
void lgf_graph_destroy(lgf_graph *graph);

/*
 * Evaluate the context's device LGF table at n lattice points (host arrays:
 * ijk [n][3] int32 in, out [n] float64): the exact near field for
 * max|n_i| <= lgf_table_radius(), the asymptotic series beyond (Sec. 5:
 * the paper tabulates G near the origin and expands it asymptotically far
 * from it).
 */
lgf_status lgf_table_values(lgf_context *ctx, int64_t n, const int32_t *ijk, double *out);
int lgf_table_radius(void);

/*
 * One LGF block spectrum (host out, (2nb)^2 (nb+1) complex float64 as
 * interleaved re/im): the r2c FFT of the window G(d*nb + m),
 * m in [-(nb-1), nb-1]^3, laid circularly on a (2nb)^3 grid.  Index
 * [kz][ky][kx], kx in [0, nb].  The spectrum is computed on the device.
 */
lgf_status lgf_block_spectrum(lgf_context *ctx, int nb, const int32_t d[3], double *out);

/*
 * Stage timing for measurement.  While enabled, every solve on this context
 * records HIP events around each launch of the forward block FFT, the
 * spectral multiply-accumulate and the inverse block FFT, on the stream the
 * launch uses (no synchronisation is added).  lgf_context_stage_times waits
 * for the recorded events, returns the summed milliseconds and launch
 * counts per stage, and clears them.  ms and launches have LGF_N_STAGES
 * entries: 0 forward block FFT, 1 spectral MAC by block pairs, 2 inverse
 * block FFT, 3 everything else, 4 lattice x DFTs, 5 lattice y/z slabs (y
 * and z DFTs, product with the lattice spectra, inverse z and y DFTs), 6
 * lattice inverse x DFTs (stages 4-6 form the spectral MAC of lattice
 * convolutions in three passes), 7 the one-pass lattice MAC (all of 4-6 per
 * frequency, see lgf_context_set_lattice_passes).
 */
#define LGF_N_STAGES 8
lgf_status lgf_context_set_timing(lgf_context *ctx, int enable);
lgf_status lgf_context_stage_times(lgf_context *ctx, double *ms, int64_t *launches);

/*
 * MAC method and tuning.  The spectral multiply-accumulate of a level
 * convolution (at each block frequency, a convolution over the block
 * lattice) runs either as block pairs, compiled for a few tile shapes
 * (rectangles of target rows per workgroup), or, for boxes of at most 32
 * blocks along x and y and 64 along z, as a zero-padded FFT over the block lattice with
 * real lattice spectra (exact up to rounding, O(L^3 log L) per frequency
 * instead of the O(E^6) pairs).  Which is fastest depends on the shape of
 * the block set.  A context keeps a table from convolution shape (block
 * size, precision, components per MAC launch, extent of the box, source and
 * target block counts) to method.  Plans take the table's method when it
 * has one, else a model (pairs at the pair kernel's arithmetic rate, the
 * lattice FFT at half the HBM bandwidth over its bytes) picks between the
 * default tile shape and the lattice FFT.
 *
 * lgf_context_set_mac_method(ctx, m): LGF_MAC_AUTO (the default) as above;
 * LGF_MAC_PAIRS uses block pairs only; LGF_MAC_LATTICE uses the lattice FFT
 * wherever the box allows it.  Plans made before the call keep their method.
 *
 * lgf_context_set_autotune(ctx, reps): with reps > 0 (at most 1000), plan
 * creation on this context times every candidate (each compiled tile shape,
 * and the lattice FFT where allowed) on each convolution shape the table
 * lacks (one warm-up and up to reps launches, fewer where they would take
 * more than about 200 ms, on the context's own stream, with scratch spectra
 * the size of that convolution's, released after) and records the fastest,
 * or the default shape unless another candidate is faster by more than 3%;
 * 0 turns this off (the default).  Block-pair results do not depend on the
 * tile shape (each target sums its sources in the same order under every
 * shape); the lattice FFT differs from them by rounding only.
 * lgf_context_save_tuning / lgf_context_load_tuning write / merge the table
 * as JSON: {"version": 2, "entries": {key: {"choice": "pairs TYxTZ" or
 * "lattice", "candidates": [...], "ms": [ms per launch, ...]}}};
 * candidates and ms may be empty or absent in a loaded file.  Loading
 * rejects malformed text with LGF_E_INVALID (the message names the byte)
 * and changes nothing then; an entry whose choice is not a candidate of its
 * convolution is ignored at plan creation.  lgf_context_tuning_size returns
 * the number of entries.
 */
typedef enum { LGF_MAC_AUTO = 0, LGF_MAC_PAIRS = 1, LGF_MAC_LATTICE = 2 } lgf_mac_method;
lgf_status lgf_context_set_mac_method(lgf_context *ctx, int method);

/*
 * How the lattice FFT of a convolution is split into launches (same sum,
 * Sec. 2.2, eq. lgf_convolution, evaluated per block frequency as a
 * zero-padded lattice convolution).  passes = 3 (the default): lattice x
 * DFTs of the source spectra into a workspace, then its y/z slabs (y and z
 * DFTs, product with the lattice spectra, inverse z and y DFTs) in place,
 * then inverse x DFTs into the target spectra: the workspace is written
 * once and read twice.  passes = 1: where the DFT lengths are 32 x 32 x 32
 * (boxes of 9 to 16 blocks along every axis), one launch does all of it per
 * block frequency in on-chip memory, writing the terms of the even and the
 * odd lattice x frequencies to two target spectra that the inverse block
 * FFT adds; other lengths keep three passes.  It moves fewer bytes but, with
 * the block-major spectra, reads and writes 16 bytes per slot and
 * workgroup, and is slower on MI355X (3.8 against 2.8 ms per MAC on the
 * 256^3 box).  The two splits agree to rounding.  Plans made before the call
 * keep their split.  Returns LGF_E_INVALID for other values.
 */
lgf_status lgf_context_set_lattice_passes(lgf_context *ctx, int passes);
lgf_status lgf_context_set_autotune(lgf_context *ctx, int reps);
lgf_status lgf_context_save_tuning(lgf_context *ctx, const char *path);
lgf_status lgf_context_load_tuning(lgf_context *ctx, const char *path);
lgf_status lgf_context_tuning_size(lgf_context *ctx, int64_t *n_entries);

const char *lgf_last_error(void);
const char *lgf_status_string(lgf_status s);

/* Build provenance (no passage of the paper: it ties a library file to the
 * sources it was compiled from).  Returns a static NUL-terminated string
 * "sha256=<64 hex digits> arch=gfx950": the digest is the SHA-256 of every
 * kernel, runtime and header source and of the compiler flags, computed by
 * the build script before compiling.  Never NULL; callable without a GPU. */
const char *lgf_build_id(void);

#ifdef __cplusplus
}
#endif

#endif /* LGF_H */
