"""Continuous-batching request loop over lgf_solve_batch.

Requests are independent single-level Poisson solves (different supports
and precisions).  The loop

* admits arrived requests in FIFO order while the HBM held by in-flight
  plan workspaces stays under a budget,
* keeps plans (and, through the context, the LGF block spectra) resident and
  reuses them for later requests of the same shape,
* launches every admitted group as one lgf_solve_batch call on one of
  several HIP streams, so a group admitted while others are still on the
  GPU overlaps with them on the device,
* records, per request, latency = completion seen by the host - arrival.

Source fields are staged in HBM before the clock starts (the measured path
is the solve, not the PCIe upload).

    python -m paper_2010_13213_amd.serve [--requests 512] [--sweep]
"""
import argparse
import collections
import json
import os
import sys
import time

import numpy as np

from . import inputs, lgf


def _pct(xs, q):
    if len(xs) == 0:
        return None
    return float(np.percentile(np.asarray(xs), q))


class PlanPool:
    """Idle plans per (blocks shape, nb, precision); created on demand."""

    def __init__(self, ctx):
        self.ctx = ctx
        self.idle = collections.defaultdict(list)
        self.ws_bytes = {}

    @staticmethod
    def key(req):
        p = req.problem
        return (len(p.levels[0].blocks), p.nb, req.precision)

    def estimate(self, req):
        return self.ws_bytes.get(self.key(req))

    def acquire(self, req):
        k = self.key(req)
        if self.idle[k]:
            return self.idle[k].pop()
        plan = lgf.Plan.for_problem(self.ctx, req.problem, req.precision)
        self.ws_bytes[k] = plan.workspace_bytes()
        return plan

    def release(self, req, plan):
        self.idle[self.key(req)].append(plan)

    def close(self):
        for v in self.idle.values():
            for p in v:
                p.close()
        self.idle.clear()


def serve(ctx, requests, rate, budget_bytes=48 << 30, n_streams=2, max_batch=64, pool=None,
          keep_results=False):
    """Run one stream of requests; arrival times = unit gaps / rate."""
    import torch
    own_pool = pool is None
    pool = pool or PlanPool(ctx)
    dev = [torch.from_numpy(r.problem.flat_source()).cuda() for r in requests]
    outs = [torch.empty_like(d) for d in dev]
    gaps = np.random.Generator(np.random.PCG64(17)).exponential(1.0, len(requests))
    arrival = np.cumsum(gaps) / rate if rate else np.zeros(len(requests))
    streams = [torch.cuda.Stream() for _ in range(n_streams)]
    torch.cuda.synchronize()

    pending = collections.deque(range(len(requests)))
    queue = collections.deque()
    inflight = []          # (event, ids, plans, stream index, bytes)
    busy = [False] * n_streams
    used = 0
    done_t = np.zeros(len(requests))
    batches = []
    t0 = time.perf_counter()
    while pending or queue or inflight:
        now = time.perf_counter() - t0
        while pending and arrival[pending[0]] <= now:
            queue.append(pending.popleft())
        still = []
        for ev, ids, plans, si, nbytes in inflight:
            if ev.query():
                t = time.perf_counter() - t0
                for i, pl in zip(ids, plans):
                    done_t[i] = t
                    pool.release(requests[i], pl)
                used -= nbytes
                busy[si] = False
            else:
                still.append((ev, ids, plans, si, nbytes))
        inflight = still
        launched = False
        if queue and not all(busy):
            si = busy.index(False)
            ids, plans, nbytes = [], [], 0
            while queue and len(ids) < max_batch:
                i = queue[0]
                est = pool.estimate(requests[i]) or 0
                if ids and used + nbytes + est > budget_bytes:
                    break
                queue.popleft()
                pl = pool.acquire(requests[i])
                ids.append(i)
                plans.append(pl)
                nbytes += pl.workspace_bytes()
            with torch.cuda.stream(streams[si]):
                lgf.solve_batch(ctx, plans, [dev[i] for i in ids], [outs[i] for i in ids],
                                stream=streams[si])
                ev = torch.cuda.Event()
                ev.record(streams[si])
            inflight.append((ev, ids, plans, si, nbytes))
            busy[si] = True
            used += nbytes
            batches.append(len(ids))
            launched = True
        if not launched:
            nxt = arrival[pending[0]] - (time.perf_counter() - t0) if pending else 0.0
            time.sleep(min(2e-4, max(0.0, nxt)) if inflight or nxt > 0 else 0.0)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lat = (done_t - arrival) * 1e3
    cells = sum(r.problem.n_cells() * r.problem.n_components for r in requests)
    res = {"requests": len(requests), "rate_req_per_s": rate, "wall_s": wall,
           "throughput_cells_per_s": cells / wall, "requests_per_s": len(requests) / wall,
           "p50_ms": _pct(lat, 50), "p99_ms": _pct(lat, 99), "mean_batch": float(np.mean(batches)),
           "batches": len(batches)}
    if keep_results:
        res["u"] = [o.cpu().numpy() for o in outs]
    if own_pool:
        pool.close()
    return res


def main():
    ap = argparse.ArgumentParser(description="served stream of independent LGF solves")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--sweep", action="store_true", help="sweep arrival rate around capacity")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    torch.cuda.init()
    ctx = lgf.Context(0)
    reqs = inputs.served_stream(args.requests)
    pool = PlanPool(ctx)
    serve(ctx, reqs, None, pool=pool)                     # create the resident plans and spectra
    cap = serve(ctx, reqs, None, pool=pool)               # all at t = 0: capacity
    rows = [dict(cap, label="all at once")]
    print(json.dumps({k: v for k, v in rows[0].items()}), flush=True)
    lam = cap["requests_per_s"]
    for f in ([0.25, 0.5, 0.75, 0.9, 1.0, 1.2] if args.sweep else [0.9]):
        r = serve(ctx, reqs, f * lam, pool=pool)
        r["label"] = "%.2f x capacity" % f
        rows.append(r)
        print(json.dumps(r), flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(rows, fh, indent=1)
    pool.close()
    ctx.close()


if __name__ == "__main__":
    main()
