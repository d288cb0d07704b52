"""Continuous-batching request loop over lgf_solve_batch.

Requests are independent single-level Poisson solves (different supports
and precisions).  The loop

* admits arrived requests in FIFO order within the HBM budget of the LGF
  context (table, spectra and every plan, idle or in flight): a plan that
  does not fit is made room for by freeing idle plans, else the request
  waits until in-flight work completes,
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
import hashlib
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
    """Idle plans per plan description; created on demand, evicted oldest first.

    The key is the whole problem description a plan is built from: block
    size, dx0, component count, precision and the block list of every
    level, so two supports with equal block counts never share a plan."""

    def __init__(self, ctx):
        self.ctx = ctx
        self.idle = collections.OrderedDict()      # key -> [plans], oldest release first
        self.created = 0
        self.evicted = 0

    @staticmethod
    def key(req):
        p = req.problem
        h = hashlib.sha256()
        for lv in p.levels:
            b = np.ascontiguousarray(lv.blocks, dtype=np.int32)
            h.update(np.int64(len(b)).tobytes())
            h.update(b.tobytes())
        return (int(p.nb), float(p.dx0), int(p.n_components), len(p.levels), req.precision, h.hexdigest())

    def acquire(self, req):
        """An idle plan of this description, else a new one (the context's
        HBM budget may refuse it with LGF_E_NOMEM)."""
        k = self.key(req)
        plans = self.idle.get(k)
        if plans:
            pl = plans.pop()
            if not plans:
                del self.idle[k]
            return pl
        pl = lgf.Plan.for_problem(self.ctx, req.problem, req.precision)
        self.created += 1
        return pl

    def release(self, req, plan):
        k = self.key(req)
        self.idle.setdefault(k, []).append(plan)
        self.idle.move_to_end(k)

    def evict_one(self):
        """Free the least recently released idle plan; False if none is idle."""
        if not self.idle:
            return False
        k, plans = next(iter(self.idle.items()))
        plans.pop(0).close()
        if not plans:
            del self.idle[k]
        self.evicted += 1
        return True

    def close(self):
        for v in self.idle.values():
            for p in v:
                p.close()
        self.idle.clear()


def _acquire_within_budget(pool, req, busy):
    """Plan for req without exceeding the context's HBM budget: on
    LGF_E_NOMEM free idle plans one by one and retry.  Returns None when
    the request must wait for in-flight work (busy) to release memory;
    raises when it cannot fit even with nothing else held."""
    while True:
        try:
            return pool.acquire(req)
        except lgf.LgfError as e:
            if e.status != lgf.LGF_E_NOMEM:
                raise
            if pool.evict_one():
                continue
            if busy:
                return None
            raise


def serve(ctx, requests, rate, n_streams=2, max_batch=64, pool=None, keep_results=False):
    """Run one stream of requests; arrival times = unit gaps / rate.

    Admission is by the HBM budget of `ctx` (lgf.Context(hbm_budget_bytes=...)),
    which bounds everything the context holds: LGF table, spectra, and every
    plan's workspace, idle or in flight.  A request whose plan does not fit
    after the idle plans are freed waits at the head of the queue until
    in-flight work completes."""
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
    inflight = []          # (event, ids, plans, stream index)
    busy = [False] * n_streams
    done_t = np.zeros(len(requests))
    batches = []
    deferred = 0
    blocked = False        # the queue head did not fit: wait for a completion
    peak_bytes = ctx.bytes()
    t0 = time.perf_counter()
    while pending or queue or inflight:
        now = time.perf_counter() - t0
        while pending and arrival[pending[0]] <= now:
            queue.append(pending.popleft())
        still = []
        for ev, ids, plans, si in inflight:
            if ev.query():
                t = time.perf_counter() - t0
                for i, pl in zip(ids, plans):
                    done_t[i] = t
                    pool.release(requests[i], pl)
                busy[si] = False
                blocked = False
            else:
                still.append((ev, ids, plans, si))
        inflight = still
        launched = False
        if queue and not all(busy) and not blocked:
            si = busy.index(False)
            ids, plans = [], []
            while queue and len(ids) < max_batch:
                pl = _acquire_within_budget(pool, requests[queue[0]], bool(inflight or ids))
                if pl is None:           # wait for memory: the head of the queue stays
                    deferred += 1
                    blocked = not ids
                    break
                ids.append(queue.popleft())
                plans.append(pl)
            peak_bytes = max(peak_bytes, ctx.bytes())
            if ids:
                with torch.cuda.stream(streams[si]):
                    lgf.solve_batch(ctx, plans, [dev[i] for i in ids], [outs[i] for i in ids],
                                    stream=streams[si])
                    ev = torch.cuda.Event()
                    ev.record(streams[si])
                inflight.append((ev, ids, plans, si))
                busy[si] = True
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
           "batches": len(batches), "deferred": deferred, "peak_context_bytes": int(peak_bytes),
           "budget_bytes": getattr(ctx, "hbm_budget_bytes", 0), "plans_created": pool.created,
           "plans_evicted": pool.evicted}
    if keep_results:
        res["u"] = [o.cpu().numpy() for o in outs]
    if own_pool:
        pool.close()
    return res


def main():
    ap = argparse.ArgumentParser(description="served stream of independent LGF solves")
    ap.add_argument("--requests", type=int, default=512)
    ap.add_argument("--budget-gb", type=float, default=48.0, help="HBM budget of the serving context")
    ap.add_argument("--sweep", action="store_true", help="sweep arrival rate around capacity")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    torch.cuda.init()
    ctx = lgf.Context(0, hbm_budget_bytes=int(args.budget_gb * (1 << 30)))
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
