"""Benchmark of the (min,+) power hot path on one MI355X.

Default workload (the headline metric): one chain step
    (N_k, R_k) = canon(N_(k-1) (x) A),   N = 16384, uint16,
on synthetic inputs (entries uniform in [0, 15], 30 % infinity, SplitMix64
seeds 1 and 2), i.e. one (min,+) product, its row-min normalisation and the
trace (Corollary 7) per step.  Throughput counts N^3 add+min pairs per step.

Prints ONE JSON line with the value, the roofline of the dominant kernel
(the product; VALU-bound, peak = CUs x 64 lanes x 2.4 GHz pairs/s, measured
with HIP events on the launch stream) and the CPU oracle timed on a bounded
sample of the same workload.

Other workloads (--workload config2|config3|config4|serve) print their own
line in the same format.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "min-plus GOPS (add+min pairs/s) at N=16384 uint16, % VALU peak; p99 query ms"
PEAK_CLOCK_GHZ = 2.4
LANES = 64


def valu_peak_gpairs(cus: int) -> float:
    """Packed-u16 VALU peak in G pairs/s: a pair is one add and one min, a
    packed instruction does two of either per lane, one wave64 instruction
    per SIMD per 4 clocks, 4 SIMDs per CU -> 64 pairs per CU per clock."""
    return cus * LANES * PEAK_CLOCK_GHZ


def cpu_baseline_gemm(X, Y, target_s: float = 15.0):
    """The oracle (as it stands) on sampled full rows of the same product;
    rate in the metric's unit (rows * N * N pairs / s)."""
    import oracle as O

    n = X.shape[0]
    Xi = O.from_u16(X)
    Yi = O.from_u16(Y)
    rng = np.random.default_rng(0)
    rows = max(1, O.threads())
    t0 = time.perf_counter()
    O.minplus(Xi[rng.integers(0, n, rows)], Yi)
    dt = time.perf_counter() - t0
    done_rows, done_t = rows, dt
    if dt < target_s / 3:
        more = int(rows * (target_s - dt) / max(dt, 1e-3))
        more = max(rows, min(more, 4096))
        t0 = time.perf_counter()
        O.minplus(Xi[rng.integers(0, n, more)], Yi)
        dt2 = time.perf_counter() - t0
        done_rows, done_t = more, dt2
    rate = done_rows * n * n / done_t / 1e9
    return {"value": round(rate, 3), "unit": "G pairs/s", "cores": O.threads(), "kind": "oracle",
            "sample": "%d random full rows of the N=%d product (%d x %d x %d pairs), %.1f s" %
                      (done_rows, n, done_rows, n, n, done_t)}


def bench_gemm(args, mpr, torch):
    import synth

    n = args.n
    dev = torch.device("cuda:0")
    t_gen = time.perf_counter()
    X = synth.random_matrix(n, n, 1, 0, 15, 0.30)
    Y = synth.random_matrix(n, n, 2, 0, 15, 0.30)
    A = mpr.to_device(Y)
    P = [mpr.to_device(X), mpr.alloc_matrix(n, n, dev)]
    R = torch.zeros(n, dtype=torch.int64, device=dev)
    gam = torch.empty(1, dtype=torch.int64, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    gen_s = time.perf_counter() - t_gen
    L = mpr.lib()
    stream = torch.cuda.current_stream()
    sptr = mpr._stream(stream)
    cfg = args.cfg

    def step(b, ev=None):
        src, dst = P[b], P[b ^ 1]
        if ev is not None:
            ev[0].record(stream)
        mpr._ok(L.mpr_minplus_gemm_cfg(cfg, n, n, n, mpr._ptr(src), mpr._ld(src), mpr._ptr(A), mpr._ld(A),
                                       mpr._ptr(dst), mpr._ld(dst), None, sptr), "gemm")
        if ev is not None:
            ev[1].record(stream)
        mpr._ok(L.mpr_normalise(n, n, mpr._ptr(dst), mpr._ld(dst), mpr._ptr(R), mpr._ptr(R), mpr._ptr(st), sptr),
                "normalise")
        mpr._ok(L.mpr_trace_min(mpr._ptr(dst), n, mpr._ld(dst), mpr._ptr(R), mpr._ptr(gam), sptr), "trace")
        return b ^ 1

    # canonical start: N_0 = canon(X)
    mpr.normalise(P[0], None, R)
    b = 0
    for _ in range(args.warmup):
        b = step(b)
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        b = step(b, events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mpr.check_status(st)
    gemm_ms = [e0.elapsed_time(e1) for e0, e1 in events]
    ms_step = wall * 1e3 / args.steps
    pairs = float(n) ** 3
    value = pairs / (ms_step * 1e-3) / 1e9
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    peak = valu_peak_gpairs(cus)
    kern_avg = float(np.mean(gemm_ms))
    achieved = pairs / (kern_avg * 1e-3) / 1e9
    traffic = None
    if args.traffic_json and os.path.exists(args.traffic_json):
        with open(args.traffic_json) as f:
            traffic = json.load(f).get("bytes_per_launch")
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "G pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u16",
        "data": "synthetic (SplitMix64 seeds 1, 2; uniform [0,15], 30% infinity)",
        "config": {"workload": "minplus chain step N=16384 uint16 (product + row-min normalisation + trace)",
                   "n": n, "tile_config": cfg if cfg >= 0 else "table"},
        "pct_valu_peak": round(100.0 * value / peak, 2),
        "roofline": {"bound": "alu", "achieved": round(achieved, 1), "peak": round(peak, 1), "unit": "G pairs/s",
                     "frac": round(achieved / peak, 4), "traffic": traffic,
                     "kernel": "gemm_kernel", "kernel_avg_ms": round(kern_avg, 3)},
        "input_gen_s": round(gen_s, 1),
    }
    if not args.skip_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_gemm(X, Y, args.cpu_seconds)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--cfg", type=int, default=-1, help="tile configuration (-1: tile table)")
    ap.add_argument("--workload", default="gemm", choices=["gemm"])
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "gemm_traffic.json"))
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one MI355X only: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2409_17658_amd as mpr

    torch.cuda.set_device(0)
    mpr.init(0)
    out = bench_gemm(args, mpr, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
