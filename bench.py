#!/usr/bin/env python3
"""Throughput benchmark of the LGF Poisson hot path on one MI355X.

Workload: a dense 256^3-cell single-level scalar solve (dx = R/64 over
[-2R, 2R]^3, 4096 blocks of 16^3 cells, source = x-vorticity of a thin
Gaussian-core vortex ring, R = 1, sigma = 0.1 R), the 256^3 configuration
of the headline metric.  A step is one full solve through the C ABI
(forward block FFTs, spectral multiply-accumulate over the 16.8M block
pairs -- by an FFT over the block lattice or pair by pair -- inverse block
FFTs), with the source already resident in HBM.

Prints one JSON line (rank 0, N = 1).  The timed solves run without
instrumentation (launched one by one, or replayed from a HIP graph with
--launch graph).  The roofline entry is for the dominant kernel of the
solve, timed in a second pass of the same solves with HIP events recorded by
the library around each of its launches on the solve stream: the lattice
y/z-slab kernel (HBM-bound) when the spectral product runs as an FFT over
the block lattice, the block-pair kernel (FP64 ALU-bound) when it runs as
block pairs.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "target cells solved/s at 256^3, FP32+refine vs FP64; p50/p99 solve latency"
FP64_VECTOR_PEAK_TFLOPS = 78.6     # MI355X FP64 vector FMA: 256 CU * 4 SIMD * 16 lanes * 2 * 2.4 GHz
HBM_PEAK_GBS = 8000.0
# Per dominant kernel: its name in profiles, the counter summary holding its
# HBM bytes per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE scaled by a 1 GiB
# copy) and the sources whose hash that summary must record to be used.
KERNELS = {
    "lat_fused": ("lat_fused<double,false>", "lat_fused_fp64_dense256_traffic.txt",
                  ["lgf_lattice.hip", "lgf_device.hpp", "lgf_kernels.hpp"]),
    "lat_yz": ("lat_yz<double,32,32>", "lat_yz_fp64_dense256_traffic.txt",
               ["lgf_lattice.hip", "lgf_device.hpp", "lgf_kernels.hpp"]),
    "smac": ("smac_kernel<16,8,16,8,double,dense,1 component>", "smac_fp64_dense256_traffic.txt",
             ["lgf_smac.hip", "lgf_device.hpp", "lgf_kernels.hpp"]),
}


def source_hash(kind):
    import hashlib
    h = hashlib.sha256()
    for name in KERNELS[kind][2]:
        with open(os.path.join(ROOT, "paper_2010_13213_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kind):
    """Counter-measured bytes per launch of the kernel, or None when the
    summary is missing or was taken for other kernel sources."""
    try:
        with open(os.path.join(ROOT, "profiles", KERNELS[kind][1])) as fh:
            kv = dict(l[1:].split(":", 1) for l in fh if l.startswith("@") and ":" in l)
    except OSError:
        return None
    kv = {k.strip(): v.strip() for k, v in kv.items()}
    if kv.get("source_sha256") != source_hash(kind):
        return None
    return float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"])


def lattice_len(extent):
    L = 4
    while L < 2 * extent - 1:
        L *= 2
    return L


WORKLOADS = ["gaussian_box_32^3", "ring_128^3_vector", "two_level_ring", "colliding_rings_quarter",
             "colliding_rings"]


def config_table(ctx, reps=3, only=None):
    """Every workload of the hot path, FP64 and FP32+refine: plan time, median
    solve time (wall, and device time between events on the solve stream),
    target cells/s and the error against stored oracle samples (tests/golden,
    written by scripts that call only the oracle) where such samples exist,
    else the difference to the FP64 result.  only: a list of workload names."""
    import numpy as np
    import torch
    from paper_2010_13213_amd import inputs, lgf

    gold = os.path.join(ROOT, "tests", "golden")
    cases = [
        ("gaussian_box_32^3", lambda: inputs.gaussian_box(), None),
        ("ring_128^3_vector", lambda: inputs.single_ring(), None),
        ("two_level_ring", lambda: inputs.two_level_ring(components=(0, 1)),
         os.path.join(gold, "two_level_ring_samples.npz")),
        ("colliding_rings_quarter", lambda: inputs.colliding_rings(nb=8, dx0=1.0 / 8, components=(0, 2)),
         os.path.join(gold, "colliding_rings_quarter_samples.npz")),
        ("colliding_rings", lambda: inputs.colliding_rings(), os.path.join(gold, "colliding_rings_full_samples.npz")),
    ]
    table = {}
    for name, make, gpath in cases:
        if only and name not in only:
            continue
        prob = make()
        f = torch.from_numpy(prob.flat_source()).cuda()
        cells = prob.n_cells() * prob.n_components
        row = {"blocks_per_level": [len(lv.blocks) for lv in prob.levels], "nb": prob.nb,
               "components": prob.n_components, "target_cells": cells}
        res = {}
        for prec in ("fp64", "fp32_refine"):
            t0 = time.perf_counter()
            plan = lgf.Plan.for_problem(ctx, prob, prec)
            t_plan = time.perf_counter() - t0
            u = torch.empty_like(f)
            plan.solve(f, u)
            torch.cuda.synchronize()
            ts, dev = [], []
            for _ in range(reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                t0 = time.perf_counter()
                e0.record()
                plan.solve(f, u)
                e1.record()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                dev.append(e0.elapsed_time(e1))
            ws = plan.workspace_bytes()
            plan.close()
            res[prec] = u.cpu().numpy().reshape(prob.n_components, -1)
            ms = 1e3 * float(np.median(ts))
            print("config %s %s: plan %.2f s, solve %.3f ms (device %.3f ms)"
                  % (name, prec, t_plan, ms, float(np.median(dev))), file=sys.stderr, flush=True)
            row[prec] = {"plan_s": round(t_plan, 3), "solve_ms": ms, "device_ms": float(np.median(dev)),
                         "cells_per_s": cells / (ms * 1e-3), "plan_workspace_bytes": int(ws),
                         "context_bytes": int(ctx.bytes())}
        if gpath is not None:
            g = np.load(gpath)
            # stored component c of the samples: the problem's component
            # g["components"][c] (all components of a 3-component problem),
            # else the problem's c-th
            pos = [int(x) for x in g["components"]] if "components" in g.files else list(range(prob.n_components))
            for prec in ("fp64", "fp32_refine"):
                errs = []
                base = 0
                for k, lv in enumerate(prob.levels):
                    n = len(lv.blocks) * prob.nb ** 3
                    idx = g["sample%d" % k]
                    for c in range(len(pos)):
                        ref = g["phi%d_c%d" % (k, c)]
                        got = res[prec][pos[c]][base:base + n][idx]
                        errs.append(float(np.linalg.norm(got - ref) / np.linalg.norm(ref)))
                    base += n
                row[prec]["err_vs_oracle_max_rel_l2"] = max(errs)
        d = res["fp32_refine"] - res["fp64"]
        row["fp32_refine"]["rel_l2_vs_fp64"] = float(np.linalg.norm(d) / np.linalg.norm(res["fp64"]))
        row["fp32_refine"]["ratio_vs_fp64"] = row["fp64"]["solve_ms"] / row["fp32_refine"]["solve_ms"]
        table[name] = row
        print("config %s: %s" % (name, json.dumps(row)), file=sys.stderr, flush=True)
        del f, res
    return table


def flgf_table(ctx, reps=3):
    """The fast-LGF approximation (lgf_plan_create_flgf) on the vector ring
    (208 blocks of 16^3) and the dense 256^3 box, near radii 1 and 2: device
    time per solve and the relative L2 error against the exact FP64 solve of
    the same context."""
    import numpy as np
    import torch
    from paper_2010_13213_amd import inputs, lgf

    def run(prob, near):
        plan = lgf.Plan.for_problem(ctx, prob, "fp64", flgf_near=near)
        f = torch.from_numpy(prob.flat_source()).cuda()
        u = torch.empty_like(f)
        plan.solve(f, u)
        torch.cuda.synchronize()
        dev = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.solve(f, u)
            e1.record()
            torch.cuda.synchronize()
            dev.append(e0.elapsed_time(e1))
        plan.close()
        return u.cpu().numpy().reshape(prob.n_components, -1), float(np.median(dev))

    out = {}
    for name, prob in (("ring_128^3_vector", inputs.single_ring(components=(0, 1))), ("dense_256^3", inputs.mstar())):
        exact, t_exact = run(prob, None)
        row = {"exact_device_ms": t_exact}
        for near in (1, 2):
            u, t = run(prob, near)
            err = max(float(np.linalg.norm(u[c] - exact[c]) / np.linalg.norm(exact[c])) for c in range(prob.n_components))
            row["near_%d" % near] = {"device_ms": t, "rel_l2_vs_exact": err}
        print("fast-LGF %s: %s" % (name, json.dumps(row)), file=sys.stderr, flush=True)
        out[name] = row
    return out


def _pct(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _time_direct(c, f, dx, rng, n):
    """Direct sums of all sources at n random targets: (targets, seconds)."""
    from oracle import direct
    tg = c[rng.choice(len(c), n, replace=False)]
    t0 = time.perf_counter()
    direct.direct_sum(c, f, tg, dx)
    return n, time.perf_counter() - t0


def cpu_baseline(problem, budget_s=10.0, seed=0):
    """Time the oracle direct sum on samples of targets (all sources), on all
    host cores and on one, plus the full 32^3 Gaussian box."""
    import numpy as np
    from oracle import direct
    from paper_2010_13213_amd import inputs
    c = inputs.cell_coords(problem.levels[0].blocks, problem.nb)
    f = problem.levels[0].values[0].reshape(-1)
    rng = np.random.default_rng(seed)
    direct.build(force=False)
    direct.direct_sum(c[:1], f[:1], c[:1], problem.dx0)      # loads the library and its table
    threads = direct.num_threads()
    # one thread first: its rate sizes both samples (the OpenMP loop hands
    # out targets 16 at a time, so a small all-core probe would idle cores)
    direct.set_num_threads(1)
    try:
        _, t_probe = _time_direct(c, f, problem.dx0, rng, 2)
        n1, dt1 = _time_direct(c, f, problem.dx0, rng, max(4, int(0.4 * budget_s / (t_probe / 2))))
    finally:
        direct.set_num_threads(threads)
    per1 = dt1 / n1
    n = int(max(16 * threads, min(len(c), (budget_s * threads / per1) // (16 * threads) * 16 * threads)))
    n, dt = _time_direct(c, f, problem.dx0, rng, n)
    gb = inputs.gaussian_box()
    cg = inputs.cell_coords(gb.levels[0].blocks, gb.nb)
    t0 = time.perf_counter()
    direct.direct_sum(cg, gb.flat_source(), cg, gb.dx0)
    t_gb = time.perf_counter() - t0
    # the vector ring (208 blocks of 16^3, two non-zero components): sampled
    # targets, both components, and the full solve extrapolated from them
    ring = inputs.single_ring()
    cr = inputs.cell_coords(ring.levels[0].blocks, ring.nb)
    nr = 32 * threads
    tr = cr[rng.choice(len(cr), nr, replace=False)]
    t0 = time.perf_counter()
    for comp in (0, 1):
        fr = ring.levels[0].values[comp].reshape(-1)
        nz = fr != 0
        direct.direct_sum(cr[nz], fr[nz], tr, ring.dx0)
    t_ring = time.perf_counter() - t0
    ring_rate = 2 * nr / t_ring
    tg = c[rng.choice(len(c), 64, replace=False)]
    u_tg = direct.direct_sum(c, f, tg, problem.dx0)
    return {"value": n / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": "%d random target cells of the 256^3 box, each summed over all %d source "
                      "cells (C/OpenMP direct sum, %d threads), %.1f s" % (n, len(c), threads, dt),
            "single_thread": {"value": n1 / dt1, "unit": "cells/s", "cores": 1,
                              "sample": "%d random target cells of the same box, %.1f s" % (n1, dt1)},
            "gaussian_box_32_full": {"value": len(cg) / t_gb, "unit": "cells/s", "cores": threads,
                                     "sample": "all %d cells against all %d sources, %.2f s"
                                               % (len(cg), len(cg), t_gb)},
            "ring_128_vector": {"value": ring_rate, "unit": "cells/s", "cores": threads,
                                "full_solve_s_extrapolated": 2 * len(cr) / ring_rate,
                                "sample": "%d random target cells of the 128^3 ring support (208 blocks of 16^3), "
                                          "components x and y against their non-zero sources, %.1f s; the z "
                                          "component is zero" % (nr, t_ring)},
            "fft_comparator": cpu_fft_comparator(problem, c, f, tg, u_tg)}


def cpu_fft_comparator(problem, c, f, check_tgt, check_ref):
    """A second, faster CPU number: the whole-box zero-padded FFT convolution
    (Hockney) in float64 with SciPy, G from the oracle's lattice Green's
    function at every offset of the box.  Only the solve (forward FFT of the
    padded source, product with the precomputed kernel spectrum, inverse FFT)
    is timed; building G and its spectrum is reported as setup."""
    import numpy as np
    import scipy.fft as sfft
    from oracle import direct
    workers = direct.num_threads()
    lo = c.min(axis=0)
    n = int((c.max(axis=0) - lo).max()) + 1
    t0 = time.perf_counter()
    ax = np.arange(n, dtype=np.int32)
    oct_pts = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), axis=-1).reshape(-1, 3)
    g_oct = direct.G_points(oct_pts).reshape(n, n, n)     # G(|dx|, |dy|, |dz|)
    del oct_pts
    wrap = np.concatenate([np.arange(n), [0], np.arange(n - 1, 0, -1)])   # index -> |offset|
    kern = g_oct[np.ix_(wrap, wrap, wrap)]
    kern[n, :, :] = 0.0
    kern[:, n, :] = 0.0
    kern[:, :, n] = 0.0                                   # offset -n never occurs
    khat = sfft.rfftn(kern, workers=workers)
    del kern, g_oct
    t_setup = time.perf_counter() - t0
    dense = np.zeros((2 * n,) * 3)
    rel = c - lo
    t0 = time.perf_counter()
    dense[rel[:, 0], rel[:, 1], rel[:, 2]] = f
    u = sfft.irfftn(sfft.rfftn(dense, workers=workers) * khat, s=dense.shape, workers=workers)
    u = u[:n, :n, :n] * problem.dx0 ** 2
    t_solve = time.perf_counter() - t0
    r = check_tgt - lo
    got = u[r[:, 0], r[:, 1], r[:, 2]]
    err = float(np.linalg.norm(got - check_ref) / np.linalg.norm(check_ref))
    return {"value": len(c) / t_solve, "unit": "cells/s", "cores": workers,
            "kind": "SciPy whole-box Hockney FFT convolution, float64 (not the oracle)",
            "solve_s": round(t_solve, 3), "setup_s": round(t_setup, 3),
            "fft_shape": [2 * n] * 3, "err_vs_oracle": err,
            "sample": "all %d cells of the box in one solve; error over %d oracle target cells"
                      % (len(c), len(check_ref))}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["both", "fp64", "fp32_refine"], default="both",
                    help="which precision paths to time (profiling runs use one)")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-budget-gb", type=float, default=48.0, help="HBM budget of the serving context")
    ap.add_argument("--configs", action="store_true",
                    help="also time every workload (FP64 and FP32+refine) into a 'configs' entry")
    ap.add_argument("--flgf", action="store_true",
                    help="time the fast-LGF approximation (near radii 1, 2) against the exact solve, print "
                         "one JSON line and exit")
    ap.add_argument("--workload", action="append", choices=WORKLOADS, default=None,
                    help="time only these workloads of the config table, print them as one JSON line and "
                         "exit (no headline measurement; for profiling one workload)")
    ap.add_argument("--print-hash", choices=sorted(KERNELS),
                    help="print the hash of that kernel's sources (as counter summaries record it) and exit")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one 1 GiB device copy first (counter calibration reference)")
    ap.add_argument("--launch", choices=["eager", "graph"], default="eager",
                    help="timed solves launched one by one, or replayed from a HIP graph of one solve (lgf_graph_create)")
    ap.add_argument("--lattice-passes", type=int, choices=[1, 3], default=3,
                    help="lattice MAC in three passes (3) or in one pass per frequency where the lengths allow (1)")
    ap.add_argument("--mac", choices=["auto", "pairs", "lattice"], default="auto",
                    help="spectral MAC method of the solves (auto: tuning table, else the cost model)")
    ap.add_argument("--autotune", type=int, default=0, metavar="REPS",
                    help="time every compiled MAC tile shape on each new convolution shape at plan "
                         "creation (REPS launches each) and keep the fastest")
    ap.add_argument("--save-tuning", default=None, help="write the context's tuning table here")
    args = ap.parse_args()
    if args.print_hash:
        print(source_hash(args.print_hash))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the LGF path here runs on a single MI355X and has no "
              "multi-GPU implementation (requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2010_13213_amd import inputs, lgf

    torch.cuda.init()
    ctx = lgf.Context(0)
    ctx.set_mac_method(args.mac)
    ctx.set_lattice_passes(args.lattice_passes)
    if args.autotune:
        ctx.set_autotune(args.autotune)
    if args.flgf:
        print(json.dumps({"flgf": flgf_table(ctx), "build": {"id": lgf.build_id()}}), flush=True)
        ctx.close()
        return
    if args.workload:
        print(json.dumps({"configs": config_table(ctx, only=args.workload),
                          "build": {"id": lgf.build_id()}}), flush=True)
        ctx.close()
        return
    prob = inputs.mstar()
    nb = prob.nb
    n_blocks = len(prob.levels[0].blocks)
    cells = n_blocks * nb ** 3 * prob.n_components
    f = torch.from_numpy(prob.flat_source()).cuda()
    if args.calib_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    def timed(precision):
        t_plan = time.perf_counter()
        plan = lgf.Plan.for_problem(ctx, prob, precision)
        t_plan = time.perf_counter() - t_plan
        u = torch.empty_like(f)
        stream = torch.cuda.current_stream()
        graph = lgf.Graph(plan, f, u) if args.launch == "graph" else None

        def run():
            if graph is not None:
                graph.launch(stream)
            else:
                plan.solve(f, u, stream=stream)

        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for a, b in evs:
            a.record(stream)
            run()
            b.record(stream)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        lat = [a.elapsed_time(b) for a, b in evs]
        host = u.cpu().numpy()
        # a second pass of the same solves with the library's stage events
        # (per launch of every kernel), outside the timed region above
        ctx.set_timing(True)
        ctx.stage_times()
        for _ in range(args.steps):
            plan.solve(f, u, stream=stream)
        st = ctx.stage_times()
        ctx.set_timing(False)
        if graph is not None:
            graph.close()
        plan.close()
        return {"wall": t1 - t0, "lat": lat, "stages": st, "plan_s": t_plan, "u": host}

    r64 = timed("fp64") if args.only in ("both", "fp64") else None
    r32 = timed("fp32_refine") if args.only in ("both", "fp32_refine") else None
    if r64 is None:
        r64 = r32

    # error of each result against the oracle on a sample of targets
    c = inputs.cell_coords(prob.levels[0].blocks, nb)
    rng = np.random.default_rng(1)
    idx = rng.choice(len(c), 48, replace=False)
    from oracle import direct
    direct.build(force=False)
    ref = direct.direct_sum(c, prob.levels[0].values[0].reshape(-1), c[idx], prob.dx0)

    def err(u):
        return float(np.linalg.norm(u[idx] - ref) / np.linalg.norm(ref))

    wall = r64["wall"]
    ms_step = 1e3 * wall / args.steps
    value = cells * args.steps / wall

    # roofline of the dominant kernel (per launch, HIP events on the solve stream)
    n_freq = (2 * nb) ** 2 * (nb + 1)
    st = r64["stages"]
    if st["lat_fused"][1] > 0:
        ext = [int(v) for v in (prob.levels[0].blocks.max(0) - prob.levels[0].blocks.min(0) + 1)]
        L = [lattice_len(e) for e in ext]
        n_stored = (nb + 1) ** 3               # lattice spectra kept for ky, kz in [0, N/2]
        n_slots = ext[0] * ext[1] * ext[2]
        # one pass per frequency: Fhat read once, the two terms of Uhat
        # written once (complex float64), the stored spectra read once (real float64)
        bytes_fu = n_freq * 16 * 3 * n_slots + n_stored * 8 * L[0] * L[1] * L[2]
        fu_ms = st["lat_fused"][0] / st["lat_fused"][1]
        achieved = bytes_fu / (fu_ms * 1e-3) / 1e9
        # the whole solve: block FFTs read/write the field (8 B per cell) and
        # the spectra (16 B per frequency per block); the inverse reads both terms
        bytes_fft = n_blocks * (nb ** 3 * 8 + n_freq * 16)
        solve_bytes = 2 * bytes_fft + n_blocks * n_freq * 16 + bytes_fu
        roof = {"bound": "hbm", "kernel": KERNELS["lat_fused"][0], "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("lat_fused"),
                "traffic_unit": "bytes per launch (HBM, counters)", "algorithmic_bytes_per_launch": bytes_fu,
                "avg_launch_ms": fu_ms, "lattice_lengths": L,
                "mac_stage_ms_per_step": st["lat_fused"][0] / args.steps,
                "solve_algorithmic_bytes": solve_bytes,
                "solve_frac": solve_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS}
    elif st["lat_yz"][1] > 0:
        ext = [int(v) for v in (prob.levels[0].blocks.max(0) - prob.levels[0].blocks.min(0) + 1)]
        L = [lattice_len(e) for e in ext]
        n_stored = (nb + 1) ** 3               # lattice spectra kept for ky, kz in [0, N/2]
        h = L[0] * ext[1] * ext[2]             # H per frequency: the box after the x DFT
        # y/z slabs: H read and written once (complex float64), stored spectra read once (real float64)
        bytes_yz = n_freq * 2 * 16 * h + n_stored * 8 * L[0] * L[1] * L[2]
        yz_ms = st["lat_yz"][0] / st["lat_yz"][1]
        achieved = bytes_yz / (yz_ms * 1e-3) / 1e9
        # the whole convolution (every kernel of a solve, algorithmic bytes):
        # block FFTs read/write the field (8 B per cell) and the spectra
        # (16 B per frequency per block), the lattice x passes read/write
        # Fhat/Uhat and H once each
        n_slots = ext[0] * ext[1] * ext[2]
        bytes_fft = n_blocks * (nb ** 3 * 8 + n_freq * 16)
        bytes_x = n_freq * 16 * (n_slots + h)
        solve_bytes = 2 * bytes_fft + 2 * bytes_x + bytes_yz
        roof = {"bound": "hbm", "kernel": KERNELS["lat_yz"][0], "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic("lat_yz"),
                "traffic_unit": "bytes per launch (HBM, counters)", "algorithmic_bytes_per_launch": bytes_yz,
                "avg_launch_ms": yz_ms, "lattice_lengths": L,
                "mac_stage_ms_per_step": sum(st[k][0] for k in ("lat_x", "lat_yz", "lat_xinv")) / args.steps,
                "solve_algorithmic_bytes": solve_bytes,
                "solve_frac": solve_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS}
    else:
        pairs = n_blocks * n_blocks
        flops_mac = 8.0 * pairs * n_freq                       # one complex MAC = 8 flops
        smac_avg = st["smac"][0] / max(1, st["smac"][1])
        achieved = flops_mac / (smac_avg * 1e-3) / 1e12
        roof = {"bound": "alu", "kernel": KERNELS["smac"][0], "achieved": achieved,
                "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
                "traffic": measured_traffic("smac"), "traffic_unit": "bytes per launch (HBM, counters)",
                "algorithmic_flops_per_launch": flops_mac, "avg_launch_ms": smac_avg}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "dense 256^3 box, 4096 blocks of 16^3, dx=R/64, ring x-vorticity, "
                               "single level, scalar; value = FP64 path",
                   "cells": cells, "block_pairs": n_blocks * n_blocks, "plan_s": round(r64["plan_s"], 3),
                   "mac_method": ("lattice, one pass" if st["lat_fused"][1] > 0 else
                                  "lattice, three passes" if st["lat_yz"][1] > 0 else "pairs")},
        "latency_ms": {"p50": _pct(r64["lat"], 50), "p99": _pct(r64["lat"], 99)},
        "err_vs_oracle": {"fp64": err(r64["u"]),
                          "fp32_refine": err(r32["u"]) if r32 else None,
                          "sample": "48 random target cells, relative L2"},
        "fp32_refine": None if r32 is None else {
            "value": cells * args.steps / r32["wall"], "unit": "cells/s",
            "ms_per_step": 1e3 * r32["wall"] / args.steps,
            "latency_ms": {"p50": _pct(r32["lat"], 50), "p99": _pct(r32["lat"], 99)},
            "stages_ms_per_step": {k: v[0] / args.steps for k, v in r32["stages"].items()},
            "ratio_vs_fp64": (cells * args.steps / r32["wall"]) / value},
        "stages_ms_per_step": {k: v[0] / args.steps for k, v in r64["stages"].items()},
        "roofline": roof,
        "build": {"library": os.path.relpath(lgf.LIB_PATH, os.path.dirname(os.path.abspath(__file__))),
                  "id": lgf.build_id()},
    }
    if not args.no_serving:
        from paper_2010_13213_amd import serve
        reqs = inputs.served_stream(args.serve_requests)
        budget = int(args.serve_budget_gb * (1 << 30))
        sctx = lgf.Context(0, hbm_budget_bytes=budget)
        pool = serve.PlanPool(sctx)
        # plans are resident state: one untimed pass at full concurrency
        # creates every plan the timed passes hold at once
        serve.serve(sctx, reqs, None, pool=pool)
        cap = serve.serve(sctx, reqs, None, pool=pool)
        sweep = []
        for frac in (0.25, 0.5, 0.75, 0.9, 1.0, 1.2):
            r = serve.serve(sctx, reqs, frac * cap["requests_per_s"], pool=pool)
            sweep.append({"rate_x_capacity": frac, "rate_requests_per_s": r["rate_req_per_s"],
                          "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
                          "throughput_cells_per_s": r["throughput_cells_per_s"], "mean_batch": r["mean_batch"],
                          "deferred": r["deferred"], "peak_context_bytes": r["peak_context_bytes"]})
            print("serving %.2f x capacity: p50 %.2f ms, p99 %.2f ms" % (frac, r["p50_ms"], r["p99_ms"]),
                  file=sys.stderr, flush=True)
        pool.close()
        sctx.close()
        at09 = [r for r in sweep if r["rate_x_capacity"] == 0.9][0]
        out["serving"] = {
            "workload": "%d independent dense-cube solves, side 16..128 cells (8^3 blocks), 1-4 Gaussian "
                        "blobs, half FP64 / half FP32+refine, Poisson arrivals; context HBM budget %.0f GiB"
                        % (len(reqs), args.serve_budget_gb),
            "capacity_requests_per_s": cap["requests_per_s"],
            "rate_requests_per_s": at09["rate_requests_per_s"],
            "p50_ms": at09["p50_ms"], "p99_ms": at09["p99_ms"],
            "throughput_cells_per_s": at09["throughput_cells_per_s"],
            "mean_batch": at09["mean_batch"], "budget_bytes": budget, "rate_sweep": sweep}
    if args.configs:
        out["configs"] = config_table(ctx)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob)
    if args.save_tuning:
        ctx.save_tuning(args.save_tuning)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
