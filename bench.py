"""Benchmark: Strassen block-recursive inversion on one MI355X.

    python bench.py [--steps K] [--warmup W] [--n N] [--leaf L] [--kind spd|dd|spdk]
                    [--mode fp64|fp32] [--ns-steps S] [--no-cpu] [--no-trace]

Default workload: FP64 inversion of the SPD matrix A = B B^T / n + I
(B i.i.d. N(0, 1), seed 2), n = 8192, leaf 256 (recursion depth 5).  A step
is one complete inversion (every level of the recursion, every leaf) with A
already resident in HBM.  The metric is 2 n^3 / t (the method's exact flop
count) in TFLOP/s, with its fraction of the FP64 matrix-core peak.

Prints one JSON line.  Extra fields:
  roofline     -- dominant kernel (largest total time in a traced replay of
                  the same steps, HIP events on the launch stream): its
                  algorithmic flops per launch / average launch duration,
                  against the FP64 MFMA peak;
  cpu_baseline -- the CPU oracle (literal Alg. 1 recursion, OpenMP) timed on a
                  bounded sample of the same workload on the host cores;
  spd_variant  -- spin_invert_spd (four products and a transpose per node) on
                  the same symmetric matrix, timed the same way, beside the
                  plain method (which alone gives `value`).

With --spd the timed step itself is spin_invert_spd (for profiling it); the
default step is always the plain method of Alg. 1.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6    # MI355X dense FP64 matrix-core peak
PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 matrix-core peak
METRIC = "inversion TFLOP/s (2n³/t) & % of MFMA peak; p50/p99 latency under load"


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=10)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--n", type=int, default=8192)
    p.add_argument("--leaf", type=int, default=256)
    p.add_argument("--kind", default="spd", choices=["spd", "dd", "spdk"])
    p.add_argument("--mode", default="fp64", choices=["fp64", "fp32"])
    p.add_argument("--spd", action="store_true",
                   help="time spin_invert_spd as the step (symmetric inputs only)")
    p.add_argument("--no-spd-variant", action="store_true",
                   help="skip the spd_variant timing beside the plain method")
    p.add_argument("--ns-steps", type=int, default=2)
    p.add_argument("--seed", type=int, default=None)
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-trace", action="store_true")
    p.add_argument("--serve-seconds", type=float, default=60.0,
                   help="length of the open-loop serving run (0 disables it)")
    p.add_argument("--serve-rate", type=float, default=200.0, help="serving arrival rate, req/s")
    p.add_argument("--serve-plain", action="store_true",
                   help="serve SPD FP64 requests on the plain schedule instead of the symmetric one")
    p.add_argument("--mixed-n", type=int, default=16384,
                   help="order of the mixed-precision vs FP64 comparison (0 disables it)")
    p.add_argument("--mixed-leaf", type=int, default=256)
    p.add_argument("--mixed-reps", type=int, default=2)
    p.add_argument("--gemm-sweep", action="store_true",
                   help="only time spin_gemm alone (FP64, FP32, BF16, bf16x3) and spin_gemm_int8 "
                        "(FP64-accurate on INT8 cores), h = 2048, 4096, 8192, and exit")
    p.add_argument("--lu-compare", action="store_true",
                   help="only time Alg. 1 against inversion through a block LU factorisation "
                        "(U(-1,1) + n I, n = 8192 and 16384, leaf 128) and exit")
    p.add_argument("--cost-model", action="store_true",
                   help="only calibrate the recursion cost model, predict the leaf sweep at n = 16384 "
                        "(and n = 8192, leaf 256), time the same inversions and exit")
    p.add_argument("--calib-copy", action="store_true",
                   help="run one 512 MiB device-to-device copy first (HBM counter calibration)")
    return p.parse_args()


def make_input(kind: str, n: int, seed: int):
    import workloads as W
    if kind == "spd":
        return W.spd_gram(n, seed), f"spd_gram (B B^T/n + I, B ~ N(0,1)), seed {seed}"
    if kind == "dd":
        return W.diag_dominant(n, seed), f"diag_dominant (U(-1,1) + n I), seed {seed}"
    return W.spd_spectrum(n, seed, 1e4), f"spd_spectrum (Q diag(lam) Q^T, kappa 1e4), seed {seed}"


def host_cpu() -> dict:
    """Model name and core counts of the host the oracle runs on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return {"model": model, "logical_cpus": os.cpu_count(), "cpus_available": avail}


def _omp_threads() -> int:
    """Threads the oracle's OpenMP loops use by default."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def _set_threads(k: int) -> None:
    """Thread count of the oracle's OpenMP loops (the oracle links libgomp)."""
    import ctypes
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(k))


def _timed(fn, reps: int) -> float:
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2]


def cpu_baseline(kind: str, n: int, leaf: int, seed: int, a_host, x_gpu):
    """The CPU oracle on the host cores.

    * value: the oracle's Strassen recursion (O2: the block-inverse identity of
      Alg. 1 with Gauss-Jordan leaves, FP64, OpenMP) on the workload itself,
      one run, as 2 n^3 / t;
    * the GPU result against that oracle inverse: normwise forward error and
      the largest element-wise error relative to its column's largest entry;
    * smaller timings: O2 and O1 (Gauss-Jordan with partial pivoting on
      [A | I]) at n = 1024 and 2048 (O2) on all cores, median of 3, and both
      at n = 256 and 1024 on one thread.  O1 at the workload's order is not
      run: its n passes over an n x 2n array make it an hour-scale,
      memory-bound run."""
    import numpy as np

    import oracle
    lib = oracle.load()
    threads = _omp_threads()
    _set_threads(threads)
    t0 = time.perf_counter()
    x_orc, info = oracle.strassen_inv(a_host, min(leaf, n), lib)
    t = time.perf_counter() - t0
    out = {
        "value": 2.0 * n ** 3 / t / 1e12,
        "unit": "TFLOP/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"oracle O2 (Alg. 1 block-inverse recursion with Gauss-Jordan leaves, FP64, OpenMP) "
                  f"on the whole workload ({kind} n={n} leaf={min(leaf, n)}): one run, {t:.2f} s",
        "host": host_cpu(),
        "oracle_info": info,
    }
    if x_gpu is not None and info == 0:
        d = np.abs(x_gpu - x_orc)
        colmax = np.abs(x_orc).max(axis=0)
        out["forward_error_vs_oracle"] = float(np.linalg.norm(x_gpu - x_orc) / np.linalg.norm(x_orc))
        out["max_elementwise_error_vs_oracle"] = float((d.max(axis=0) / colmax).max())
    del x_orc
    rows = []
    for m in (1024, 2048):
        a, _ = make_input(kind, m, seed)
        rows.append({"oracle": "O2", "n": m, "leaf": min(leaf, m), "threads": threads,
                     "s_median_of_3": round(_timed(lambda: oracle.strassen_inv(a, min(leaf, m), lib), 3), 4)})
        if m == 1024:
            rows.append({"oracle": "O1", "n": m, "threads": threads,
                         "s_median_of_3": round(_timed(lambda: oracle.gj_inv(a, lib), 3), 4)})
    _set_threads(1)
    try:
        for m in (256, 1024):
            a, _ = make_input(kind, m, seed)
            rows.append({"oracle": "O2", "n": m, "leaf": min(leaf, m), "threads": 1,
                         "s_median_of_3" if m == 256 else "s_one_run":
                             round(_timed(lambda: oracle.strassen_inv(a, min(leaf, m), lib), 3 if m == 256 else 1), 4)})
            rows.append({"oracle": "O1", "n": m, "threads": 1,
                         "s_median_of_3" if m == 256 else "s_one_run":
                             round(_timed(lambda: oracle.gj_inv(a, lib), 3 if m == 256 else 1), 4)})
    finally:
        _set_threads(threads)
    for r in rows:
        secs = r.get("s_median_of_3", r.get("s_one_run"))
        r["gflops_2n3"] = round(2.0 * r["n"] ** 3 / secs / 1e9, 3)
    out["timings"] = rows
    return out


def serving(rate: float, seconds: float, symmetric: bool = True):
    """Open-loop serving run: Poisson arrivals at `rate` for `seconds`, orders
    log-uniform in [64, 4096] padded to 64, half diagonally dominant and half
    SPD (kappa log-uniform in [10, 1e4]), 70% mixed precision with 2 Newton
    steps and 30% FP64 (its SPD requests on the symmetric schedule), leaf
    128; orders below 512, from 512 to 2047 and from 2048 up are served by
    three server lanes on three streams; p50/p99 latency from arrival to
    completion, TFLOP/s from 2n^3 per request (the plain method's count, also
    for symmetric requests)."""
    import workloads as W
    from paper_1801_04723_amd import serve
    trace = W.serving_trace(rate=rate, duration=seconds, seed=5)
    st = serve.run_trace(trace, leaf=128, ns_steps=2, split_n=[512, 2048], symmetric=symmetric)
    st["workload"] = (f"Poisson {rate:g} req/s for {seconds:g} s, n log-uniform 64..4096 (x64), "
                      "50% diag-dominant / 50% SPD, 70% mixed FP32+2 Newton / 30% FP64 "
                      f"({'SPD FP64 requests on the symmetric schedule' if symmetric else 'plain schedule'}), leaf 128; "
                      "three server lanes on three streams (n < 512, 512 <= n < 2048, n >= 2048)")
    return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}


def mixed_vs_fp64(n: int, leaf: int, reps: int):
    """Mixed-precision inversions against the FP64 one on the same matrix and
    leaf: SPD A = Q diag(lam) Q^T, Q from the QR factorisation of a seeded
    Gaussian matrix (generated on the GPU), lam geometric over [1, 1e4].
    Each mode: rho before and after refinement (from the library's report),
    status, and the mean time of `reps` asynchronous calls after one warm-up."""
    import torch

    import paper_1801_04723_amd as spin
    import workloads as W
    t0 = time.perf_counter()
    dA = W.torch_spd_spectrum(n, seed=4, kappa=1e4, device="cuda")
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    dX = torch.empty_like(dA)
    runs = [("fp64", 0), ("fp32", 2), ("bf16x3", 3), ("bf16", 2), ("fp32_int8", 2), ("bf16x3_int8", 3)]
    out = {"workload": f"spd_spectrum (Q diag(lam) Q^T, kappa 1e4) n={n} generated on the GPU "
                       f"(seed 4, {gen_s:.1f} s), leaf {leaf}",
           "n": n, "leaf": leaf, "modes": {}}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for mode, steps in runs:
        if mode == "fp64":
            call = lambda: spin.invert(dA, leaf=leaf, out=dX)  # noqa: E731
        else:
            call = lambda: spin.invert_mixed(dA, leaf=leaf, mode=mode, ns_steps=steps,  # noqa: E731
                                             out=dX)
        call()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            call()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        rec = {"ms": round(ms, 2), "ns_steps": steps, "tflops_2n3": round(2.0 * n ** 3 / ms / 1e9, 2)}
        if mode == "fp64":
            rec["status"] = spin.info()
            rec["rho"] = spin.residual(dA, dX)
        else:
            _, rep = spin.invert_mixed(dA, leaf=leaf, mode=mode, ns_steps=steps, out=dX, report=True)
            rec.update(rho_before=rep["rho_before"], rho_after=rep["rho_after"],
                       r_fro=[float(v) for v in rep["r_fro"][:steps]], status=rep["status"])
        out["modes"][mode] = rec
    f = out["modes"]["fp64"]["ms"]
    for mode, _ in runs[1:]:
        out["modes"][mode]["time_vs_fp64"] = round(out["modes"][mode]["ms"] / f, 3)
    del dA, dX
    spin.release()
    torch.cuda.empty_cache()
    return out


def spd_variant(dA, n: int, leaf: int, steps: int, warmup: int, plain_ms: float):
    """spin_invert_spd on the same symmetric matrix: the same timing as the
    main step, its residual, and the schedule's own flop count."""
    import torch
    import paper_1801_04723_amd as spin
    dX = torch.empty_like(dA)
    for _ in range(warmup):
        spin.invert_spd(dA, leaf=leaf, out=dX)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        spin.invert_spd(dA, leaf=leaf, out=dX)
    stop.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop) / steps
    _, sched_flops = spin.plan_describe(n, leaf, spd=True)
    out = {
        "ms": round(ms, 4),
        "time_vs_plain": round(ms / plain_ms, 4),
        "tflops_2n3": round(2.0 * n ** 3 / (ms * 1e-3) / 1e12, 3),
        "schedule_flops": sched_flops,
        "schedule_tflops": round(sched_flops / (ms * 1e-3) / 1e12, 3),
        "status": spin.info(),
        "rho": spin.residual(dA, dX),
    }
    del dX
    return out


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when that summary is absent or the kernel's source file
    changed since the counters were taken."""
    import hashlib
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as f:
            rec = json.load(f).get(kernel)
        if not rec:
            return None
        with open(os.path.join(ROOT, rec["source"]), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
                return None
        return rec["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        return None


def roofline_from_trace(recs, n_steps: int):
    """Dominant kernel = largest total traced time; achieved = its algorithmic
    flops per launch / its average launch duration."""
    by = {}
    for r in recs:
        d = by.setdefault(r["kernel"], {"ms": 0.0, "flops": 0.0, "bytes": 0.0, "count": 0})
        d["ms"] += r["ms"]
        d["flops"] += r["flops"]
        d["bytes"] += r["bytes"]
        d["count"] += 1
    name, d = max(by.items(), key=lambda kv: kv[1]["ms"])
    avg_ms = d["ms"] / d["count"]
    flops_per_launch = d["flops"] / d["count"]
    achieved = flops_per_launch / (avg_ms * 1e-3) / 1e12
    peak = PEAK_FP64_TFLOPS if "f64" in name or "leaf" in name else PEAK_FP32_TFLOPS
    breakdown = {k: {"ms_per_step": round(v["ms"] / n_steps, 4), "launches_per_step": v["count"] // n_steps,
                     "tflops": round(v["flops"] / max(v["ms"], 1e-9) / 1e9, 3)}
                 for k, v in sorted(by.items(), key=lambda kv: -kv[1]["ms"])}
    return {
        "bound": "mfma",
        "kernel": name,
        "achieved": round(achieved, 3),
        "peak": peak,
        "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": measured_traffic(name),
        "algorithmic_bytes_per_launch": d["bytes"] / d["count"],
        "avg_launch_ms": round(avg_ms, 5),
        "flops_per_launch": flops_per_launch,
        "launches": d["count"],
    }, breakdown


def lu_compare_run():
    """Alg. 1 (spin_invert) against inversion through a block LU factorisation
    (spin_invert_lu) on the same matrices, the paper's SPIN-vs-LU comparison on
    one GPU: time per inversion (HIP events, 1 warm-up + 3), residual, and the
    schedule flops of each."""
    import torch
    import paper_1801_04723_amd as spin
    from paper_1801_04723_amd import costmodel as C
    import workloads as W
    rows = []
    for n, leaf in [(8192, 128), (16384, 128)]:
        A = W.torch_diag_dominant(n, seed=3)
        X = torch.empty_like(A)
        row = {"n": n, "leaf": leaf}
        for name, fn, desc in (("spin", spin.invert, {}), ("lu", spin.invert_lu, {"lu": True})):
            ms = C._time_ms(lambda: fn(A, leaf=leaf, out=X), reps=3, warm=1)
            _, fl = spin.plan_describe(n, leaf, **desc)
            row[name] = {"ms": round(ms, 3), "tflops_2n3": round(2.0 * n ** 3 / (ms * 1e-3) / 1e12, 3),
                         "schedule_flops": fl, "status": spin.info(), "rho": spin.residual(A, X)}
            print(f"n={n} {name}: {ms:.2f} ms", file=sys.stderr, flush=True)
        row["lu_over_spin"] = round(row["lu"]["ms"] / row["spin"]["ms"], 3)
        rows.append(row)
        del A, X
        spin.release()
        torch.cuda.empty_cache()
    return rows


def cost_model_run():
    """Calibrate the cost model (isolated leaves, nodes and products), then
    predict and time the leaf sweep of U(-1,1) + n I at n = 16384 and the
    n = 8192, leaf 256 step."""
    import torch
    import paper_1801_04723_amd as spin
    from paper_1801_04723_amd import costmodel as C
    import workloads as W
    t0 = time.perf_counter()
    rates = C.calibrate()
    print(f"calibrated in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    rows = []
    for n, leaf in [(16384, L) for L in (64, 128, 256, 512, 1024, 2048)] + [(8192, 256)]:
        A = W.torch_diag_dominant(n, seed=3)
        X = torch.empty_like(A)
        ms = C._time_ms(lambda: spin.invert(A, leaf=leaf, out=X), reps=3, warm=1)
        p = C.predict(n, leaf, rates)
        rows.append({"n": n, "leaf": leaf, "measured_ms": round(ms, 3), "predicted_ms": round(p["ms"], 3),
                     "leaf_term_ms": round(p["leaf_ms"], 3), "node_term_ms": round(p["node_ms"], 3),
                     "rel_error": round((p["ms"] - ms) / ms, 4), "leaves": p["leaves"], "nodes": p["nodes"]})
        print(f"n={n} leaf={leaf}: measured {ms:.2f} ms, predicted {p['ms']:.2f} ms", file=sys.stderr, flush=True)
        del A, X
        spin.release()
        torch.cuda.empty_cache()
    sweep = [r for r in rows if r["n"] == 16384]
    return {
        "leaf_ms": {str(k): round(v, 5) for k, v in sorted(rates.leaf_ms.items())},
        "node_ms": {str(k): round(v, 5) for k, v in sorted(rates.node_ms.items())},
        "cases": rows,
        "best_leaf_predicted": C.best_leaf(16384, rates, candidates=(64, 128, 256, 512, 1024, 2048)),
        "best_leaf_measured": min(sweep, key=lambda r: r["measured_ms"])["leaf"],
    }


def gemm_sweep():
    """Standalone block products D = A B (h x h x h, column-major, ld h) in each
    flavour: mean of 20 back-to-back calls after 3 warm-ups, HIP events on the
    launch stream.  TFLOP/s of 2h^3 (bf16x3 issues three times that)."""
    import torch

    import paper_1801_04723_amd as spin
    rows = []
    for h in (2048, 4096, 8192):
        for mode, dt in (("fp64", torch.float64), ("fp32", torch.float32), ("bf16", torch.float32),
                         ("bf16x3", torch.float32), ("int8emu", torch.float64)):
            g = torch.Generator(device="cuda")
            g.manual_seed(h)
            a = torch.rand(h, h, dtype=dt, device="cuda", generator=g)
            b = torch.rand(h, h, dtype=dt, device="cuda", generator=g)
            d = torch.empty(h, h, dtype=dt, device="cuda")
            if mode == "int8emu":
                # FP64-accurate product on INT8 matrix cores, 14 moduli
                call = lambda: spin.gemm_int8(h, h, h, a, h, b, h, 0, None, 1, d, h)  # noqa: E731
            else:
                call = lambda: spin.gemm_cm(h, h, h, 1.0, a, h, b, h, 0.0, None, h, d, h, False, mode)  # noqa: E731
            for _ in range(3):
                call()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                call()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 20
            rows.append({"h": h, "mode": mode, "ms": round(ms, 4), "tflops": round(2.0 * h ** 3 / ms / 1e9, 2)})
            del a, b, d
    return rows


def finite_json(x):
    """The output with every NaN or infinity replaced by None (strict JSON)."""
    import math
    if isinstance(x, float):
        return x if math.isfinite(x) else None
    if isinstance(x, dict):
        return {k: finite_json(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [finite_json(v) for v in x]
    return x


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; "
                                   f"--gpus {args.gpus} is not supported (use --gpus 1)"}))
        sys.exit(2)
    import torch

    import paper_1801_04723_amd as spin

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.gemm_sweep:
        print(json.dumps({"gemm_sweep": gemm_sweep()}), flush=True)
        return
    if args.cost_model:
        print(json.dumps(finite_json({"cost_model": cost_model_run()})), flush=True)
        return
    if args.lu_compare:
        print(json.dumps(finite_json({"lu_compare": lu_compare_run()})), flush=True)
        return
    dev = torch.device("cuda:0")
    seed = args.seed if args.seed is not None else {"spd": 2, "dd": 3, "spdk": 4}[args.kind]
    n, leaf = args.n, args.leaf
    a_host, desc = make_input(args.kind, n, seed)
    import numpy as np
    dA = torch.from_numpy(np.ascontiguousarray(a_host.T)).to(dev).t()  # column-major on device
    if args.no_cpu:
        del a_host
    dX = torch.empty_like(dA)
    stream = torch.cuda.current_stream()

    if args.calib_copy:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float64, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.spd and (args.mode != "fp64" or args.kind == "dd"):
        raise SystemExit("--spd needs --mode fp64 and a symmetric --kind (spd or spdk)")

    def step():
        if args.spd:
            spin.invert_spd(dA, leaf=leaf, out=dX)
        elif args.mode == "fp64":
            spin.invert(dA, leaf=leaf, out=dX)
        else:
            spin.invert_mixed(dA, leaf=leaf, mode="fp32", ns_steps=args.ns_steps, out=dX)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(args.steps):
        step()
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop) / args.steps
    status = spin.info()
    value = 2.0 * n ** 3 / (ms * 1e-3) / 1e12
    rho = spin.residual(dA, dX)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.mode == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{desc}, n={n}, leaf={leaf}, {args.mode}"
                        + (f", {args.ns_steps} Newton steps" if args.mode != "fp64" else "")
                        + (", symmetric variant (spin_invert_spd)" if args.spd else ""),
            "n": n, "leaf": leaf, "mode": args.mode,
            "depth": max(0, (n // leaf).bit_length() - 1) if n > leaf else 0,
        },
        "pct_fp64_peak": round(100.0 * value / PEAK_FP64_TFLOPS, 2),
        "rho": rho,
        "status": status,
        "wall_s_timed": round(wall, 4),
    }
    if not args.no_trace:
        spin.trace_enable(True)
        torch.cuda.synchronize()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        spin.trace_enable(False)
        recs = spin.trace_collect()
        roof, breakdown = roofline_from_trace(recs, args.steps)
        out["roofline"] = roof
        out["kernel_breakdown"] = breakdown
    else:
        out["roofline"] = None
    if args.mode == "fp64" and not args.spd and args.kind != "dd" and not args.no_spd_variant:
        out["spd_variant"] = spd_variant(dA, n, leaf, args.steps, args.warmup, ms)
    if args.serve_seconds > 0:
        out["serving"] = serving(args.serve_rate, args.serve_seconds, not args.serve_plain)
    # the timed result itself, compared with the oracle's inverse below
    x_gpu = dX.cpu().numpy() if not args.no_cpu else None
    if args.mixed_n > 0:
        del dA, dX
        spin.release()
        torch.cuda.empty_cache()
        out["mixed_precision"] = mixed_vs_fp64(args.mixed_n, args.mixed_leaf, args.mixed_reps)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.kind, n, leaf, seed, a_host, x_gpu)
        cb = out["cpu_baseline"]
        for k in ("forward_error_vs_oracle", "max_elementwise_error_vs_oracle"):
            if k in cb:
                out[k] = cb[k]
    print(json.dumps(finite_json(out), allow_nan=False), flush=True)


if __name__ == "__main__":
    main()
