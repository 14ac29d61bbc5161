"""Open-loop serving driver for the continuous-batching server.

Requests arrive on a seeded Poisson schedule (workloads.serving_trace); each
arrival is submitted at its arrival time, the server admits it when a slot
and pool space are free, and every loop iteration launches one step of every
admitted request (spin_server_tick), so requests of different orders and
precisions run concurrently with their block products and leaves batched
together.  Latency is measured from the scheduled arrival time to the moment
the host observes the request's completion event (open loop: a slow server
cannot delay arrivals).

Input matrices come from a pool keyed by (order, class, conditioning bucket),
generated on the GPU with seeded generators (diagonally dominant U(-1, 1) +
nI, or SPD with a geometric spectrum up to kappa), because generating a fresh
SPD matrix per request would dominate the host time.
"""
from __future__ import annotations

import collections
import math
import time

from . import FP64, MIXED_FP32, SYMMETRIC, Server, residual, server_request_bytes

KAPPA_BUCKETS = (10 ** 1.5, 10 ** 2.5, 10 ** 3.5)


class MatrixPool:
    def __init__(self, device="cuda", seed: int = 5):
        self.device = device
        self.seed = seed
        self.cache = {}

    def get(self, n: int, kind: str, kappa: float):
        import workloads as W
        if kind == "dd":
            key = (n, "dd", 0)
        else:
            b = min(range(len(KAPPA_BUCKETS)),
                    key=lambda i: abs(math.log10(KAPPA_BUCKETS[i]) - math.log10(max(kappa, 1.0))))
            key = (n, "spd", b)
        a = self.cache.get(key)
        if a is None:
            s = self.seed * 1_000_003 + n * 7 + key[2]
            if kind == "dd":
                a = W.torch_diag_dominant(n, s, self.device)
            else:
                a = W.torch_spd_spectrum(n, s, KAPPA_BUCKETS[key[2]], self.device)
            self.cache[key] = a
        return a


def percentile(xs, p):
    if not xs:
        return float("nan")
    xs = sorted(xs)
    k = (len(xs) - 1) * p / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)


def run_trace(trace, leaf: int = 128, ns_steps: int = 2, pool_bytes: int = 32 << 30,
              max_active: int = 64, max_ticks_in_flight: int = 64, pool: MatrixPool | None = None,
              split_n=None, symmetric: bool = False, check_every: int = 25):
    """Serves `trace` (list of dicts with t, n, kind, kappa, mixed) and returns
    latency / throughput statistics.

    split_n (an order or an increasing list of orders) divides the requests
    into lanes by order; each lane is its own server on its own stream, with
    the pool divided evenly.  The long step sequences of large requests and
    the many short steps of small ones then run side by side instead of
    taking turns in one stream; each request's result is the same either way.

    symmetric: FP64 requests for SPD matrices (exactly symmetric inputs) run
    the symmetric schedule (mode FP64 | SYMMETRIC), about half the flops.
    Mixed requests keep the plain schedule: their FP64 refinement dominates,
    so the symmetric one saves only a few percent there and leaves a larger
    residual after the same number of Newton steps.

    check_every: every check_every-th request (by arrival) keeps its result;
    after the run their residuals rho = |A X - I|_F / (|A|_F |X|_F) are
    computed on the GPU (spin_residual) and reported, split by mode.  Mixed
    requests are also checked by the library itself (rho <= 1e-12, else a
    refinement-divergence status)."""
    import torch
    pool = pool or MatrixPool()
    # materialise the inputs before the clock starts
    for r in trace:
        pool.get(r["n"], r["kind"], r["kappa"])
    torch.cuda.synchronize()
    bounds = [] if split_n is None else sorted([split_n] if isinstance(split_n, int) else list(split_n))
    if not bounds:
        lanes = [(Server(pool_bytes, max_active, leaf, ns_steps), torch.cuda.current_stream())]
    else:
        share = pool_bytes // (len(bounds) + 1)
        lanes = [(Server(share, max_active, leaf, ns_steps), torch.cuda.Stream())
                 for _ in range(len(bounds) + 1)]
    inflight = [collections.deque() for _ in lanes]
    lat, flops, statuses = [], 0.0, collections.Counter()
    outs, kept = {}, {}
    nxt = 0
    done = 0
    t0 = time.perf_counter()
    while done < len(trace):
        now = time.perf_counter() - t0
        while nxt < len(trace) and trace[nxt]["t"] <= now:
            r = trace[nxt]
            a = pool.get(r["n"], r["kind"], r["kappa"])
            x = torch.empty_like(a)
            lane = sum(1 for b in bounds if r["n"] >= b)
            if r["mixed"]:
                mode = MIXED_FP32
            elif symmetric and r["kind"] != "dd":
                mode = FP64 | SYMMETRIC
            else:
                mode = FP64
            lanes[lane][0].submit(a, x, mode, tag=nxt)
            outs[nxt] = x
            nxt += 1
        busy = False
        for (srv, stream), q in zip(lanes, inflight):
            st = srv.stats()
            if st["active"] or st["queued"]:
                busy = True
                srv.tick(stream)
                ev = torch.cuda.Event()
                ev.record(stream)
                q.append(ev)
                while len(q) > max_ticks_in_flight:
                    q.popleft().synchronize()
        if not busy and nxt < len(trace):
            time.sleep(min(1e-3, max(0.0, trace[nxt]["t"] - now)))
        for srv, _ in lanes:
            for tag, info in srv.poll():
                t_done = time.perf_counter() - t0
                lat.append(t_done - trace[tag]["t"])
                flops += 2.0 * trace[tag]["n"] ** 3
                statuses[info] += 1
                x = outs.pop(tag, None)
                if check_every and tag % check_every == 0:
                    kept[tag] = (x, info)
                done += 1
    makespan = time.perf_counter() - t0
    for srv, _ in lanes:
        srv.close()
    checked = {"fp64": [], "mixed": []}
    for tag, (x, info) in sorted(kept.items()):
        r = trace[tag]
        a = pool.get(r["n"], r["kind"], r["kappa"])
        checked["mixed" if r["mixed"] else "fp64"].append((residual(a, x), info))
    check = {k: {"count": len(v), "max_rho": max((rho for rho, _ in v), default=None),
                 "above_1e-12": sum(1 for rho, _ in v if not rho <= 1e-12),
                 "nonzero_status": sum(1 for _, info in v if info != 0)}
             for k, v in checked.items()}
    return {
        "requests": len(trace),
        "p50_ms": 1e3 * percentile(lat, 50),
        "p90_ms": 1e3 * percentile(lat, 90),
        "p99_ms": 1e3 * percentile(lat, 99),
        "max_ms": 1e3 * max(lat) if lat else float("nan"),
        "throughput_rps": len(lat) / makespan,
        "aggregate_tflops": flops / makespan / 1e12,
        "makespan_s": makespan,
        "status_counts": dict(statuses),
        "leaf": leaf,
        "ns_steps": ns_steps,
        "max_active": max_active,
        "lanes": len(lanes),
        "split_n": bounds,
        "symmetric": bool(symmetric),
        "residual_check": dict(check, every=check_every),
    }
