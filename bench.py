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

The headline runs in the packed uint16 form (the library's default
arithmetic) against the packed-int16 VALU peak; "f16_form" times the same
step in the exact f16 form (a labelled experiment with its own peak) and a
product whose minima all reach 2048 (its slow path).

The default run then adds compact legs of the other workloads, each with
the oracle timed on a bounded sample as its CPU baseline: config1 (m = 3,
n = 3..40), config2 (N = 8192 product and 64-power chain), config3 (m = 6,
7, 8 to n = 300), config4 (256 batched chains against the per-instance
path), and drives the query server (config 5: a cold leg on a fresh engine,
--serve-seconds of the Poisson stream at 200 req/s with every ladder
resident, a saturation burst, and the per-instance form of the engine).

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


def valu_peak_gpairs(cus: int, arith: str = "u16") -> float:
    """VALU peak in G pairs/s for the product's instruction mix; a pair is
    one add and one min.  A CU issues 64 lane-instructions per clock (one
    wave64 instruction per SIMD per 4 clocks, 4 SIMDs).  u16: v_pk_add_u16 +
    v_pk_min_u16 give 2 pairs per 2 lane-instructions -> 64 pairs per CU per
    clock.  f16 form: two v_pk_add_f16 + one v_pk_minimum3_f16 give 4 pairs
    per 3 lane-instructions -> 85.3 pairs per CU per clock."""
    per_clock = LANES * (4.0 / 3.0 if arith == "f16" else 1.0)
    return cus * per_clock * PEAK_CLOCK_GHZ


def cpu_baseline_gemm(X, Y, target_s: float = 15.0):
    """The oracle (as it stands) on sampled full rows of the same product;
    rate in the metric's unit (rows * N * N pairs / s).  A first small
    sample sizes the second one to about target_s seconds."""
    import oracle as O

    n = X.shape[0]
    Xi = O.from_u16(X)
    Yi = O.from_u16(Y)
    rng = np.random.default_rng(0)
    rows = max(2, 2 * O.threads())
    t0 = time.perf_counter()
    O.minplus(Xi[rng.integers(0, n, rows)], Yi)
    dt = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.minplus(Xi[rng.integers(0, n, 2 * rows)], Yi)
    dt2 = time.perf_counter() - t0
    per_row = max((dt2 - dt) / rows, 1e-4)  # marginal cost of a row
    fixed = max(dt - rows * per_row, 0.0)   # per-call set-up (finite-entry lists)
    more = int(max(rows, min(8192, (target_s - fixed) / per_row)))
    t0 = time.perf_counter()
    O.minplus(Xi[rng.integers(0, n, more)], Yi)
    dt3 = time.perf_counter() - t0
    rate = more * n * n / dt3 / 1e9
    return {"value": round(rate, 3), "unit": "G pairs/s", "cores": O.threads(), "kind": "oracle",
            "sample": "%d random full rows of the N=%d product (%d x %d x %d pairs counted), %.1f s" %
                      (more, n, more, n, n, dt3)}


def _dtype(arith: str) -> str:
    return "uint16" if arith == "u16" else "f16"


def _events(torch, k):
    return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(k)]


def bench_gemm(args, mpr, torch):
    """The headline: the N = 16384 chain step in the packed uint16 form
    (the library's default arithmetic), against the packed-int16 VALU peak;
    the same step in the exact f16 form is reported beside it as a labelled
    experiment, with a product whose minima all reach 2048 (the f16 form's
    slow path: every tile recomputed in uint16)."""
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
    cur = [0]

    def step(cfg, ev=None):
        src, dst = P[cur[0]], P[cur[0] ^ 1]
        if ev is not None:
            ev[0].record(stream)
        mpr._ok(L.mpr_minplus_gemm_cfg(cfg, n, n, n, mpr._ptr(src), mpr._ld(src), mpr._ptr(A), mpr._ld(A),
                                       mpr._ptr(dst), mpr._ld(dst), None, sptr), "gemm")
        if ev is not None:
            ev[1].record(stream)
        mpr._ok(L.mpr_normalise(n, n, mpr._ptr(dst), mpr._ld(dst), mpr._ptr(R), mpr._ptr(R), mpr._ptr(st), sptr),
                "normalise")
        mpr._ok(L.mpr_trace_min(mpr._ptr(dst), n, mpr._ld(dst), mpr._ptr(R), mpr._ptr(gam), sptr), "trace")
        cur[0] ^= 1

    def timed_steps(cfg, steps, warmup):
        """(ms per whole step by the host clock, mean product-kernel ms by HIP
        events on the launch stream)."""
        for _ in range(warmup):
            step(cfg)
        torch.cuda.synchronize()
        ev = _events(torch, steps)
        t0 = time.perf_counter()
        for k in range(steps):
            step(cfg, ev[k])
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        mpr.check_status(st)
        return wall * 1e3 / steps, float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev]))

    # canonical start: N_0 = canon(X)
    mpr.normalise(P[0], None, R)
    pairs = float(n) ** 3
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    cfg = args.cfg if args.cfg >= 0 else mpr.gemm_pick_config(n, n, n)
    info = mpr.gemm_config_info(cfg)
    ms_step, kern_avg = timed_steps(cfg, args.steps, args.warmup)
    value = pairs / (ms_step * 1e-3) / 1e9
    achieved = pairs / (kern_avg * 1e-3) / 1e9
    peak = valu_peak_gpairs(cus, info["arith"])
    dtype = _dtype(info["arith"])

    def tile_name(i):
        return "%dx%d, %dx%d per lane, %d threads, %s arithmetic" % (i["bm"], i["bn"], i["tm"], i["tn"],
                                                                   i["threads"], i["arith"])

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "G pairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
        "data": "synthetic (SplitMix64 seeds 1, 2; uniform [0,15], 30% infinity)",
        "config": {"workload": "minplus chain step N=16384 uint16 (product + row-min normalisation + trace)",
                   "n": n, "tile_config": cfg, "tile": tile_name(info),
                   "storage": "uint16 in and out"},
        "pct_valu_peak": round(100.0 * value / peak, 2),
        "roofline": {"bound": "alu", "achieved": round(achieved, 1), "peak": round(peak, 1), "unit": "G pairs/s",
                     "frac": round(achieved / peak, 4), "traffic": load_traffic(args.traffic_json, cfg),
                     "kernel": "gemm_kernel<%d,%d,%d,%d,%d>, %s" % (info["bm"], info["bn"], info["bk"], info["tm"],
                                                                    info["tn"], info["arith"]),
                     "kernel_avg_ms": round(kern_avg, 3),
                     "peak_basis": "%d CUs x 64 lanes x 2.4 GHz; %s" % (
                         cus, "v_pk_add_u16 clamp + v_pk_min_u16: 2 pairs per 2 lane-instructions"
                         if info["arith"] == "u16" else "2 v_pk_add_f16 + 1 v_pk_minimum3_f16: 4 pairs per 3")},
        "input_gen_s": round(gen_s, 1),
    }
    if args.probe:
        # the instruction mix's own rate on this device, and the clock it ran at
        # (pairs per CU per clock = the issue rate the peak assumes: 64 for
        # uint16, 85.33 for the f16 form; the probe's clock is its own, a
        # pure-VALU load runs a little below the product's)
        probe = {}
        for a in ("u16", "f16"):
            rate, ghz = mpr.valu_probe(a, args.probe_iters)
            nominal = valu_peak_gpairs(cus, a)
            probe[a] = {"gpairs": round(rate / 1e9, 1), "frac_of_nominal_peak": round(rate / 1e9 / nominal, 4),
                        "clock_ghz": round(ghz, 3), "pairs_per_cu_clock": round(rate / (cus * ghz * 1e9), 2),
                        "nominal_pairs_per_cu_clock": round(nominal / (cus * PEAK_CLOCK_GHZ), 2)}
        out["valu_probe"] = probe
    if args.f16_form and info["arith"] == "u16":
        out["f16_form"] = bench_f16_form(args, mpr, torch, timed_steps, tile_name, cus, pairs, n, L, sptr)
    if not args.skip_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_gemm(X, Y, args.cpu_seconds)
    return out


def bench_f16_form(args, mpr, torch, timed_steps, tile_name, cus, pairs, n, L, sptr):
    """The same chain step in the f16 form (an exact second arithmetic: the
    f16 images of small uint16 values add exactly, and a packed three-input
    minimum takes two k per instruction), against its own instruction-mix
    peak; then one product whose every minimum is >= 2048, where the f16
    form recomputes every tile in uint16."""
    import synth

    with mpr.arith_scope("f16"):
        fcfg = mpr.gemm_pick_config(n, n, n)
    finfo = mpr.gemm_config_info(fcfg)
    ms_step, kern = timed_steps(fcfg, args.steps, max(1, args.warmup // 2))
    fpeak = valu_peak_gpairs(cus, "f16")
    ach = pairs / (kern * 1e-3) / 1e9
    out = {"label": "experiment: exact f16 form of the same uint16 product (same bits, other instruction mix)",
           "tile_config": fcfg, "tile": tile_name(finfo), "ms_per_step": round(ms_step, 3),
           "value": round(pairs / (ms_step * 1e-3) / 1e9, 1), "kernel_avg_ms": round(kern, 3),
           "achieved": round(ach, 1), "peak": round(fpeak, 1), "frac": round(ach / fpeak, 4),
           "pct_of_packed_int16_peak": round(100.0 * ach / valu_peak_gpairs(cus, "u16"), 1),
           "traffic": load_traffic(args.traffic_json, fcfg)}
    if args.slow_reps <= 0:
        return out
    # slow path: entries in [1024, 1039] (30 % infinity), so every finite sum is >= 2048
    Xs = mpr.to_device(synth.random_matrix(n, n, 11, 1024, 1039, 0.30))
    Ys = mpr.to_device(synth.random_matrix(n, n, 12, 1024, 1039, 0.30))
    C = [mpr.alloc_matrix(n, n), mpr.alloc_matrix(n, n)]
    ucfg = mpr.gemm_pick_config(n, n, n)
    stream = torch.cuda.current_stream()
    times = {}
    for name, c, dst in (("u16", ucfg, C[0]), ("f16", fcfg, C[1])):
        ev = _events(torch, args.slow_reps + 1)
        for e0, e1 in ev:
            e0.record(stream)
            mpr._ok(L.mpr_minplus_gemm_cfg(c, n, n, n, mpr._ptr(Xs), mpr._ld(Xs), mpr._ptr(Ys), mpr._ld(Ys),
                                           mpr._ptr(dst), mpr._ld(dst), None, sptr), "gemm")
            e1.record(stream)
        torch.cuda.synchronize()
        times[name] = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev[1:]]))
    same = bool(torch.equal(C[0].view(torch.int16), C[1].view(torch.int16)))
    out["slow_path"] = {"inputs": "uniform [1024,1039], 30% infinity (seeds 11, 12): every minimum >= 2048",
                        "u16_kernel_ms": round(times["u16"], 3), "f16_kernel_ms": round(times["f16"], 3),
                        "f16_over_u16": round(times["f16"] / times["u16"], 3), "bit_identical": same}
    return out


def kernel_source_digest() -> str:
    """Digest of the sources the product kernel is built from (traffic
    counters taken on another version are not reported)."""
    import hashlib

    h = hashlib.sha256()
    for f in ("tile.h", "gemm.hip", "common.h"):
        with open(os.path.join(ROOT, "paper_2409_17658_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(path, cfg: int):
    """HBM bytes per launch of product configuration cfg at N = 16384, from
    the copy-calibrated counter runs, if they were taken on these sources."""
    if not path or not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != kernel_source_digest():
        return None
    rec = t.get("configs", {}).get(str(cfg))
    return rec.get("bytes_per_launch") if rec else None


def copy_calibration(torch, nbytes=1 << 30):
    """A plain device-to-device copy of known size, for scaling the HBM
    byte counters of a profiled run (FETCH_SIZE / WRITE_SIZE)."""
    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    return nbytes


# ---------------------------------------------------------------- goldens
def load_goldens():
    """gamma_R tables stored by tests/golden/make_roman_golden.py (plain JSON)."""
    gd = os.path.join(ROOT, "tests", "golden")
    out = {}
    for m in range(1, 9):
        f = os.path.join(gd, "roman_m%d.json" % m)
        if os.path.exists(f):
            with open(f) as fh:
                d = json.load(fh)
            out[m] = ({int(k): v for k, v in d["trace"].items()}, tuple(d["period"]))
    return out


def expected_gamma(goldens, m, n):
    """Stored table extended by the period (Proposition 8); m = 9 uses the
    closed form of Section 4.3 (4n if 5 | n else 4n + 2)."""
    if m == 9:
        return 4 * n if n % 5 == 0 else 4 * n + 2
    if m not in goldens:
        return None
    g, (mu, lam, c) = goldens[m]
    if n in g:
        return g[n]
    q, r = divmod(n - mu, lam)
    return g[mu + r] + c * q


# ---------------------------------------------------------------- config 2
def bench_config2(args, mpr, torch):
    import synth

    n, e = 8192, 64
    X = synth.random_matrix(n, n, 3, 0, 15, 0.30)
    A = mpr.to_device(X)
    C = mpr.alloc_matrix(n, n)
    ws = mpr.workspace(mpr.power_workspace_size(n, e, mpr.CHAIN))
    N = mpr.alloc_matrix(n, n)
    R = torch.empty(n, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    mpr.minplus_gemm(A, A, C, check=False)
    torch.cuda.synchronize()
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        mpr.minplus_gemm(A, A, C, check=False)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    t_single = float(np.median(ts))
    mpr.minplus_power(A, 3, mpr.CHAIN, N, R, ws, check=False, d_status=st)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mpr.minplus_power(A, e, mpr.CHAIN, N, R, ws, check=False, d_status=st)
    torch.cuda.synchronize()
    t_chain = time.perf_counter() - t0
    mpr.check_status(st)
    pairs = float(n) ** 3
    return {"metric": "min-plus GOPS, N=8192 single product and 64-power chain", "value": round(63 * pairs / t_chain / 1e9, 1),
            "unit": "G pairs/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": _dtype(mpr.gemm_config_info(mpr.gemm_pick_config(n, n, n))["arith"]),
            "data": "synthetic (SplitMix64 seed 3; uniform [0,15], 30% infinity)",
            "config": {"workload": "A^64 by the chain, N=8192, normalised every step", "n": n, "e": e},
            "single_product_ms": round(t_single * 1e3, 3), "single_product_gpairs": round(pairs / t_single / 1e9, 1),
            "chain_s": round(t_chain, 3)}


# ---------------------------------------------------------------- config 3
def bench_config3(args, mpr, torch):
    goldens = load_goldens()
    per_m = {}
    for m in (6, 7, 8):
        A = mpr.build_transfer(m)
        n = A.shape[0]
        ws = mpr.workspace(mpr.power_workspace_size(n, 300, mpr.SQUARE))
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        N = mpr.alloc_matrix(n, n)
        R = torch.empty(n, dtype=torch.int64, device="cuda")
        mpr.minplus_power(A, 4, mpr.CHAIN, N, R, ws, check=False, d_status=st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mpr.minplus_power(A, 300, mpr.CHAIN, N, R, ws, check=False, d_status=st)
        torch.cuda.synchronize()
        t_chain = time.perf_counter() - t0
        Nc = N.clone()
        Rc = R.clone()
        t0 = time.perf_counter()
        mpr.minplus_power(A, 300, mpr.SQUARE, N, R, ws, check=False, d_status=st)
        torch.cuda.synchronize()
        t_sq = time.perf_counter() - t0
        same = bool(torch.equal(Nc.view(torch.int16), N.view(torch.int16)) and torch.equal(Rc, R))
        mpr.check_status(st)
        wsp = mpr.workspace(mpr.power_workspace_size(n, 300, mpr.CHAIN_SPARSE))
        Ns = mpr.alloc_matrix(n, n)
        Rs = torch.empty(n, dtype=torch.int64, device="cuda")
        mpr.minplus_power(A, 4, mpr.CHAIN_SPARSE, Ns, Rs, wsp, check=False, d_status=st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mpr.minplus_power(A, 300, mpr.CHAIN_SPARSE, Ns, Rs, wsp, check=False, d_status=st)
        torch.cuda.synchronize()
        t_sp = time.perf_counter() - t0
        same_sp = bool(torch.equal(Nc.view(torch.int16), Ns.view(torch.int16)) and torch.equal(Rc, Rs))
        t0 = time.perf_counter()
        mu, lam, c, tr = mpr.find_period(A, 300, traces=True, slots=40)
        t_per = time.perf_counter() - t0
        t0 = time.perf_counter()
        mus, lams, cs, trs = mpr.find_period(A, 300, traces=True, slots=8, sparse=True)
        t_per_sp = time.perf_counter() - t0
        t0 = time.perf_counter()
        mue, lame, ce, tre = mpr.find_period(A, 300, traces=True, slots=8, sparse=True, extend=True)
        t_per_ext = time.perf_counter() - t0
        same_per = (mus, lams, cs) == (mu, lam, c) and bool(np.array_equal(trs, tr))
        same_ext = (mue, lame, ce) == (mu, lam, c) and bool(np.array_equal(tre, tr))
        ok = None
        if m in goldens:
            g, per = goldens[m]
            ok = (mu, lam, c) == per and all(int(tr[k]) == g[k] for k in range(1, 301))
        per_m[m] = {"n_states": n, "period": [mu, lam, c], "chain_300_s": round(t_chain, 3),
                    "chain_gpairs": round(299 * float(n) ** 3 / t_chain / 1e9, 1),
                    "square_300_s": round(t_sq, 4), "chain_equals_square": same,
                    "sparse_chain_300_s": round(t_sp, 4), "sparse_speedup": round(t_chain / t_sp, 2),
                    "sparse_equals_dense": same_sp,
                    "find_period_300_s": round(t_per, 3), "find_period_sparse_300_s": round(t_per_sp, 3),
                    "find_period_sparse_to_period_s": round(t_per_ext, 3),
                    "sparse_period_same": same_per, "extended_traces_same": same_ext,
                    "gamma_3_300_match_golden": ok}
    tot = sum(299 * float(v["n_states"]) ** 3 for v in per_m.values())
    tt = sum(v["chain_300_s"] for v in per_m.values())
    if args.with_m9:
        per_m[9] = bench_m9(mpr, torch)
    return {"metric": "Roman transfer powers to n=300 (m=6,7,8): chain GOPS", "value": round(tot / tt / 1e9, 1),
            "unit": "G pairs/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": _dtype(mpr.gemm_config_info(mpr.gemm_pick_config(7411, 7411, 7411))["arith"]),
            "data": "transfer matrices",
            "config": {"workload": "A(G)^300 by chain and by squaring, period search, gamma_R(3..300)"},
            "per_m": per_m}


def bench_m9(mpr, torch):
    """m = 9 (21909 states), the paper's largest exact case: the 50 powers of
    its Table 2 / Table 3 run, dense and compressed-K, and the period search;
    checked against Table 2 and the Section 4.3 closed form."""
    A = mpr.build_transfer(9)
    n = A.shape[0]
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = {"n_states": n}
    for name, sched in (("dense", mpr.CHAIN), ("sparse", mpr.CHAIN_SPARSE)):
        ws = mpr.workspace(mpr.power_workspace_size(n, 50, sched))
        N = mpr.alloc_matrix(n, n)
        R = torch.empty(n, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mpr.minplus_power(A, 50, sched, N, R, ws, check=False, d_status=st)
        torch.cuda.synchronize()
        out["A50_%s_s" % name] = round(time.perf_counter() - t0, 3)
        print("m9: A^50 %s %.2f s" % (name, out["A50_%s_s" % name]), file=sys.stderr, flush=True)
        del ws, N, R
    mpr.check_status(st)
    t0 = time.perf_counter()
    mu, lam, c, tr = mpr.find_period(A, 60, traces=True, slots=8, sparse=True)
    out["find_period_sparse_s"] = round(time.perf_counter() - t0, 3)
    out["period"] = [mu, lam, c]
    out["closed_form_ok"] = all(int(tr[k]) == (4 * k if k % 5 == 0 else 4 * k + 2) for k in range(3, 61))
    out["dense_gpairs"] = round(49 * float(n) ** 3 / out["A50_dense_s"] / 1e9, 1)
    out["paper_k80_50_powers_s"] = {"total": 4587, "kernel": 3100}
    return out


# ---------------------------------------------------------------- m = 10
def bench_m10(args, mpr, torch):
    """gamma_R(P_10 x C_n) for every n: the m = 10 transfer matrix (64769
    states, 8.4 GB per power) by the chain with a ring of 8 resident powers,
    its least period, and the checks the paper and the oracle provide:
    Remark 13 (2(m+1)n/5 for 5 | n), Theorem 11 (ceil(2(m+1)n/5) <= gamma for
    n >= 10) and the oracle's row DP for n <= 9 (stored golden)."""
    m, kmax = 10, args.m10_kmax
    A = mpr.build_transfer(m)
    n = A.shape[0]
    torch.cuda.synchronize()
    print("m10: transfer matrix built, %d states" % n, file=sys.stderr, flush=True)
    flags = mpr.PERIOD_SPARSE if args.m10_sparse else 0
    plan_b = mpr.sparse_plan_bytes(A) if args.m10_sparse else 0  # the plan sized for this A
    ws_b = mpr.period_workspace_size(n, 8, 0) + plan_b
    ws = mpr.workspace(ws_b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mu, lam, c, tr = mpr.find_period(A, kmax, traces=True, ws=ws, sparse=bool(args.m10_sparse))
    t = time.perf_counter() - t0
    print("m10: %d powers in %.1f s, period %s" % (kmax, t, (mu, lam, c)), file=sys.stderr, flush=True)
    # the same search stopped at the confirming power (Algorithm 2), later traces from the period
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    mue, lame, ce, tre = mpr.find_period(A, kmax, traces=True, ws=ws, sparse=bool(args.m10_sparse), extend=True)
    t_ext = time.perf_counter() - t0
    print("m10: stopped at the period in %.1f s" % t_ext, file=sys.stderr, flush=True)
    gam = {k: int(tr[k]) for k in range(3, kmax + 1)}
    out = {"metric": "gamma_R(P_10 x C_n): seconds for the m=10 period search (A^1..A^kmax, N=64769)",
           "value": round(t, 2), "unit": "s", "n_gpus": 1, "higher_is_better": False,
           "dtype": "uint16" if mpr.get_arith() == "u16" else "f16",
           "data": "transfer matrix m=10",
           "dense_equivalent_gpairs": round((kmax - 1) * float(n) ** 3 / t / 1e9, 1),
           "config": {"workload": "A(G)^k, k <= %d, N=64769, ring of 8 powers" % kmax, "n": n,
                      "chain_step": "compressed-K (sparse A)" if args.m10_sparse else "dense"},
           "period": [mu, lam, c], "seconds": round(t, 1), "gamma": gam,
           "workspace_gb": round(ws_b / 1e9, 2), "plan_gb": round(plan_b / 1e9, 3),
           "plan_worst_case_gb": round((mpr.period_workspace_size(n, 8, flags) -
                                        mpr.period_workspace_size(n, 8, 0)) / 1e9, 2),
           "to_period_s": round(t_ext, 2),
           "extended_traces_same": (mue, lame, ce) == (mu, lam, c) and bool(np.array_equal(tre, tr))}
    if mu is not None:
        numer = mpr.period_formula(mu, lam, c, tr[: mu + lam])
        out["formula"] = {"valid_from": mu, "gamma(n)": "(%d n + numer[n mod %d]) / %d" % (c, lam, lam),
                          "numer": numer.tolist()}
        ext = lambda k: mpr.gamma_from_period(mu, lam, c, tr, k)
        out["remark13_ok"] = all(ext(k) == 2 * (m + 1) * k // 5 for k in range(5, 2001, 5))
        out["theorem11_ok"] = all(ext(k) >= -(-2 * (m + 1) * k // 5) for k in range(10, 2001))
    gd = os.path.join(ROOT, "tests", "golden", "rowdp_m10.json")
    if os.path.exists(gd):
        with open(gd) as f:
            rd = {int(k): v for k, v in json.load(f)["gamma"].items()}
        out["rowdp_golden_ok"] = all(gam[k] == v for k, v in rd.items() if k in gam)
    return out


# ---------------------------------------------------------------- m = 11
def bench_m11(args, mpr, torch):
    """gamma_R(P_11 x C_n) for every n: the m = 11 transfer matrix (191476
    states, 73.3 GB per power) on one MI355X.  Three powers fit beside each
    other, not a ring longer than the period, so the search keeps two
    powers in its ring and A's own buffer (free once the compressed-K plan
    replaces A) for the power at which a class repeat shows; the relation
    is confirmed exactly one period later.  Checks: Remark 13 (2(m+1)n/5 for
    5 | n), Theorem 11 (ceil(2(m+1)n/5) <= gamma for n >= 10) and the
    oracle's row DP for small n (stored golden)."""
    m, kmax = 11, args.m11_kmax
    A = mpr.build_transfer(m)
    n = A.shape[0]
    torch.cuda.synchronize()
    print("m11: transfer matrix built, %d states" % n, file=sys.stderr, flush=True)
    plan_b = mpr.sparse_plan_bytes(A)
    flags = mpr.PERIOD_SPARSE | mpr.PERIOD_EXTEND | mpr.PERIOD_REUSE_A
    ws_b = mpr.period_workspace_size(n, 2, mpr.PERIOD_REUSE_A) + plan_b
    ws = mpr.workspace(ws_b)
    t_last = [time.perf_counter()]

    def progress(k, trace):  # one line per power (each takes seconds)
        now = time.perf_counter()
        print("m11: power %d trace %d (%.1f s)" % (k, trace, now - t_last[0]), file=sys.stderr, flush=True)
        t_last[0] = now

    mpr.set_period_progress(progress)
    try:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mu, lam, c, tr = mpr.find_period(A, kmax, traces=True, ws=ws, sparse=True, extend=True, reuse_a=True)
        t = time.perf_counter() - t0
    finally:
        mpr.set_period_progress(None)
    del A
    computed = (mu + lam) if mu is not None else kmax
    gam = {k: int(tr[k]) for k in range(3, kmax + 1)}
    out = {"metric": "gamma_R(P_11 x C_n): seconds for the m=11 period search (N=191476)",
           "value": round(t, 2), "unit": "s", "n_gpus": 1, "higher_is_better": False,
           "dtype": "uint16" if mpr.get_arith() == "u16" else "f16", "data": "transfer matrix m=11",
           "config": {"workload": "A(G)^k, N=191476, two ring powers + A's buffer, compressed-K steps", "n": n,
                      "flags": "sparse, extend, reuse_a"},
           "period": [mu, lam, c], "powers_computed": computed, "gamma": gam,
           "workspace_gb": round(ws_b / 1e9, 2), "matrix_gb": round(n * mpr.round_up(n) * 2 / 1e9, 2),
           "plan_gb": round(plan_b / 1e9, 3)}
    if mu is not None:
        numer = mpr.period_formula(mu, lam, c, tr[: mu + lam])
        out["formula"] = {"valid_from": mu, "gamma(n)": "(%d n + numer[n mod %d]) / %d" % (c, lam, lam),
                          "numer": numer.tolist()}
        ext = lambda k: mpr.gamma_from_period(mu, lam, c, tr, k)
        out["remark13_ok"] = all(ext(k) == 2 * (m + 1) * k // 5 for k in range(5, 2001, 5))
        out["theorem11_ok"] = all(ext(k) >= -(-2 * (m + 1) * k // 5) for k in range(10, 2001))
    gd = os.path.join(ROOT, "tests", "golden", "rowdp_m11.json")
    if os.path.exists(gd):
        with open(gd) as f:
            rd = {int(k): v for k, v in json.load(f)["gamma"].items()}
        out["rowdp_golden_ok"] = all(gam[k] == v for k, v in rd.items() if k in gam)
    return out


# ---------------------------------------------------------------- config 4
def bench_config4(args, mpr, torch):
    import synth

    inst = synth.batch_instances(256, seed=4)
    t_gen = time.perf_counter()
    chains = []
    for d in inst:
        X = synth.random_matrix(d["n"], d["n"], d["seed"], 0, 31, 0.25)
        A = mpr.to_device(X)
        chains.append((A, d["e"], mpr.alloc_matrix(d["n"], d["n"]), torch.empty(d["n"], dtype=torch.int64, device="cuda")))
    gen_s = time.perf_counter() - t_gen
    pairs = sum((d["e"] - 1) * float(d["n"]) ** 3 for d in inst)
    ws = mpr.workspace(mpr.batch_workspace_size(chains))
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    # autotune: time one launch per batched configuration (or take the one given)
    tune = {}
    if args.batch_cfg == -2:
        for cfg in range(mpr.batch_config_count()):
            mpr.set_batch_config(cfg)
            mpr.batch_plan(chains, ws, stream)
            t0 = time.perf_counter()
            mpr.batch_launch(ws, st, stream)
            stream.synchronize()
            tune[cfg] = time.perf_counter() - t0
        mpr.set_batch_config(min(tune, key=tune.get))
    else:
        mpr.set_batch_config(args.batch_cfg)
    mpr.batch_plan(chains, ws, stream)
    best = mpr.batch_plan_info(ws)[0]
    g = mpr.batch_graph_create(ws, st, stream)
    mpr.graph_launch(g, stream)
    stream.synchronize()
    reps = max(1, args.batch_reps)
    t0 = time.perf_counter()
    for _ in range(reps):
        mpr.graph_launch(g, stream)
    stream.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    mpr.graph_destroy(g)
    mpr.check_status(st)
    batched = [(N.clone(), R.clone()) for (_, _, N, R) in chains]
    # the same configuration as a persistent grid (resident workgroups looping over the list)
    mpr.set_batch_persistent(True)
    try:
        mpr.batch_plan(chains, ws, stream)
        pgrid = mpr.batch_plan_info(ws)[1]
        g = mpr.batch_graph_create(ws, st, stream)
        mpr.graph_launch(g, stream)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            mpr.graph_launch(g, stream)
        stream.synchronize()
        t_pers = (time.perf_counter() - t0) / reps
        mpr.graph_destroy(g)
        mpr.check_status(st)
        pers_same = all(torch.equal(N.view(torch.int16), b[0].view(torch.int16)) and torch.equal(R, b[1])
                        for (_, _, N, R), b in zip(chains, batched))
    finally:
        mpr.set_batch_persistent(False)
    mpr.set_batch_config(-1)
    # the plain per-instance path: one chain after another
    t_solo, same = None, None
    if args.per_instance:
        wsi = mpr.workspace(max(mpr.power_workspace_size(d["n"], d["e"], mpr.CHAIN) for d in inst))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for (A, e, N, R) in chains:
            mpr.minplus_power(A, e, mpr.CHAIN, N, R, wsi, check=False, d_status=st)
        torch.cuda.synchronize()
        t_solo = time.perf_counter() - t0
        mpr.check_status(st)
        same = all(torch.equal(N.view(torch.int16), b[0].view(torch.int16)) and torch.equal(R, b[1])
                   for (_, _, N, R), b in zip(chains, batched))
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    binfo = mpr.batch_config_info(best)
    return {"metric": "batched min-plus power chains GOPS (256 chains, one launch in a HIP graph)",
            "value": round(pairs / t_batch / 1e9, 1), "unit": "G pairs/s", "n_gpus": 1, "higher_is_better": True,
            "dtype": _dtype(binfo["arith"]), "data": "synthetic (batch_instances seed 4; entries U[0,31], 25% infinity)",
            "config": {"workload": "256 chains, N log-uniform [256,4096], e uniform [8,128]",
                       "total_pairs": pairs, "batch_config": best, "panel_rows": binfo["panel_rows"],
                       "per_instance_tile_configs": sorted({mpr.gemm_pick_config(d["n"], d["n"], d["n"])
                                                            for d in inst})},
            "batched_s": round(t_batch, 3), "per_instance_s": round(t_solo, 3) if t_solo else None,
            "per_instance_gpairs": round(pairs / t_solo / 1e9, 1) if t_solo else None,
            "speedup_vs_per_instance": round(t_solo / t_batch, 2) if t_solo else None,
            "persistent_form": {"grid": pgrid, "s": round(t_pers, 3), "gpairs": round(pairs / t_pers / 1e9, 1),
                                "equal": bool(pers_same)},
            "pct_valu_peak": round(100 * pairs / t_batch / 1e9 / valu_peak_gpairs(cus, binfo["arith"]), 2),
            "autotune_s": {str(k): round(v, 3) for k, v in tune.items()},
            "batched_equals_per_instance": None if same is None else bool(same), "input_gen_s": round(gen_s, 1)}


# ---------------------------------------------------------------- compact legs of the default line
def host_cpu() -> dict:
    """The host's CPU model and logical CPU count (the oracle's cores)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count()}


def _timed(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return r, time.perf_counter() - t0


def _rows(torch, t, rows):
    """Rows of a device uint16 matrix on the host (through an int16 view:
    torch does not index uint16 device tensors)."""
    idx = torch.as_tensor(np.asarray(rows), device=t.device)
    return t.view(torch.int16)[idx].cpu().numpy().view(np.uint16)


def _same(torch, a, b):
    return bool(torch.equal(a[0].view(torch.int16), b[0].view(torch.int16)) and torch.equal(a[1], b[1]))


def leg_config1(mpr, torch):
    """m = 3 (33 states), n = 3..40: the GPU chain's traces and period against
    the oracle run in full (its chain and exhaustive search for n <= 5)."""
    import oracle as O

    m, kmax = 3, 40

    def gpu(pipeline=False):
        A = mpr.build_transfer(m)
        return mpr.find_period(A, kmax, traces=True, slots=8, pipeline=pipeline)

    (mu, lam, c, tr), t_gpu = _timed(torch, gpu)
    (mup, lamp, cp, trp), t_gpu_p = _timed(torch, lambda: gpu(True))
    t0 = time.perf_counter()
    Ao = O.transfer(m)
    g = {}
    O.power_chain(Ao, kmax, on_step=lambda k, N, R: g.__setitem__(k, O.trace(N, R)))
    per = O.find_period(Ao, kmax)[:3]
    brute = {n: O.brute_gamma(m, n) for n in (3, 4, 5)}
    t_cpu = time.perf_counter() - t0
    ok = all(int(tr[n]) == g[n] for n in range(3, kmax + 1)) and all(int(tr[n]) == v for n, v in brute.items())
    return {"workload": "m=3 transfer matrix (33 states), gamma_R(P_3 x C_n) for n=3..40, period",
            "period": [mu, lam, c], "gpu_s": round(t_gpu, 4),
            "gpu_pipelined_s": round(t_gpu_p, 4),
            "pipelined_same": bool((mup, lamp, cp) == (mu, lam, c) and np.array_equal(trp, tr)),
            "gamma_3_40": [int(tr[n]) for n in range(3, kmax + 1)],
            "matches_oracle": bool(ok and tuple(per) == (mu, lam, c)),
            "cpu_baseline": {"value": round(t_cpu, 3), "unit": "s", "cores": O.threads(), "kind": "oracle",
                             "sample": "the whole config: chain to n=40, period, exhaustive search n=3..5"}}


def leg_config2(mpr, torch, args):
    """N = 8192: one product, and A^64 by the chain (63 products, each
    normalised); the f16 form of the chain as a labelled experiment; the
    oracle's row-restricted chain on sampled rows (row i of A^k depends only
    on row i of A^(k-1) and on A, so this is exact) as CPU baseline and
    parity check."""
    import oracle as O
    import synth

    n, e = 8192, 64
    X = synth.random_matrix(n, n, 3, 0, 15, 0.30)
    A = mpr.to_device(X)
    C = mpr.alloc_matrix(n, n)
    stream = torch.cuda.current_stream()
    mpr.minplus_gemm(A, A, C, check=False)
    ev = _events(torch, 5)
    for e0, e1 in ev:
        e0.record(stream)
        mpr.minplus_gemm(A, A, C, check=False)
        e1.record(stream)
    torch.cuda.synchronize()
    t_single = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev])) * 1e-3
    ws = mpr.workspace(mpr.power_workspace_size(n, e, mpr.CHAIN))
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = {}
    for arith in ("u16", "f16"):
        N = mpr.alloc_matrix(n, n)
        R = torch.empty(n, dtype=torch.int64, device="cuda")
        with mpr.arith_scope(arith):
            mpr.minplus_power(A, 3, mpr.CHAIN, N, R, ws, check=False, d_status=st)
            _, t = _timed(torch, lambda: mpr.minplus_power(A, e, mpr.CHAIN, N, R, ws, check=False, d_status=st))
        mpr.check_status(st)
        out[arith] = ((N, R), t)
    pairs = float(n) ** 3
    rng = np.random.default_rng(3)
    rows = np.sort(rng.choice(n, args.config2_rows, replace=False))
    t0 = time.perf_counter()
    Nr, Rr = O.chain_rows(O.from_u16(X), rows, e)
    t_cpu = time.perf_counter() - t0
    (Nu, Ru), t_chain = out["u16"]
    ok = np.array_equal(_rows(torch, Nu, rows), O.to_u16(Nr)) and np.array_equal(Ru.cpu().numpy()[rows], Rr)
    return {"workload": "N=8192 uint16 (seed 3, U[0,15], 30% inf): one product, A^64 by the chain",
            "value": round(63 * pairs / t_chain / 1e9, 1), "unit": "G pairs/s", "dtype": "uint16",
            "chain_s": round(t_chain, 3), "single_product_ms": round(t_single * 1e3, 3),
            "single_product_gpairs": round(pairs / t_single / 1e9, 1),
            "f16_form": {"chain_s": round(out["f16"][1], 3),
                         "gpairs": round(63 * pairs / out["f16"][1] / 1e9, 1),
                         "bit_identical": _same(torch, out["u16"][0], out["f16"][0])},
            "sampled_rows_match_oracle": bool(ok),
            "cpu_baseline": {"value": round(len(rows) * (e - 1) * float(n) * n / t_cpu / 1e9, 3),
                             "unit": "G pairs/s", "cores": O.threads(), "kind": "oracle",
                             "sample": "%d random rows of A^64 by the row-restricted chain (63 steps), %.1f s; "
                                       "full chain extrapolated %.0f s" % (len(rows), t_cpu, t_cpu * n / len(rows))}}


def leg_config3(mpr, torch, goldens, args):
    """m = 6, 7, 8: powers to n = 300 by the chain (dense and compressed-K)
    and by binary powering, bit-identical; the least period and gamma_R for
    n = 3..300 against the stored goldens; the oracle's chain in full for
    m = 6, 7 and on sampled rows for m = 8 (over the arcs of A)."""
    import oracle as O

    per_m = {}
    tot_pairs = tot_t = 0.0
    for m in (6, 7, 8):
        A = mpr.build_transfer(m)
        n = A.shape[0]
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        res = {}
        for name, sched in (("chain", mpr.CHAIN), ("square", mpr.SQUARE), ("sparse_chain", mpr.CHAIN_SPARSE)):
            ws = mpr.workspace(mpr.power_workspace_size(n, 300, sched))
            N, R = mpr.alloc_matrix(n, n), torch.empty(n, dtype=torch.int64, device="cuda")
            mpr.minplus_power(A, 4, sched, N, R, ws, check=False, d_status=st)
            _, t = _timed(torch, lambda: mpr.minplus_power(A, 300, sched, N, R, ws, check=False, d_status=st))
            res[name] = ((N, R), t)
            del ws
        mpr.check_status(st)
        (mu, lam, c, tr), t_per = _timed(torch, lambda: mpr.find_period(A, 300, traces=True, slots=8, sparse=True,
                                                                        extend=True))
        # the same search with each power computed while the host reads the previous one's class hash
        (mup, lamp, cp, trp), t_per_p = _timed(torch, lambda: mpr.find_period(A, 300, traces=True, slots=8,
                                                                              sparse=True, extend=True,
                                                                              pipeline=True))
        pipelined_same = (mup, lamp, cp) == (mu, lam, c) and np.array_equal(trp, tr)
        g, per = goldens[m]
        golden_ok = (mu, lam, c) == per and all(int(tr[k]) == g[k] for k in range(1, 301))
        t0 = time.perf_counter()
        if m < 8:
            want = {}
            Nr, Rr = O.power_chain(O.transfer(m), 300, on_step=lambda k, N_, R_: want.__setitem__(k, O.trace(N_, R_)))
            rows = np.arange(n)
            sample = "whole chain to n=300"
            oracle_ok = all(int(tr[k]) == want[k] for k in range(1, 301))
        else:
            rows = np.sort(np.random.default_rng(8).choice(n, args.config3_rows, replace=False))
            Nr, Rr = O.chain_rows_sparse(O.transfer_rows(m, rows), O.transfer_arcs(m), 300)
            sample = "%d random rows of A^300 by the row chain over the arcs of A" % len(rows)
            oracle_ok = True
        t_cpu = time.perf_counter() - t0
        (Nc, Rc), t_chain = res["chain"]
        oracle_ok = oracle_ok and np.array_equal(_rows(torch, Nc, rows), O.to_u16(Nr)) and \
            np.array_equal(Rc.cpu().numpy()[rows], Rr)
        pairs = 299 * float(n) ** 3
        tot_pairs += pairs
        tot_t += t_chain
        per_m[m] = {"n_states": n, "period": [mu, lam, c], "chain_300_s": round(t_chain, 3),
                    "chain_gpairs": round(pairs / t_chain / 1e9, 1), "square_300_s": round(res["square"][1], 4),
                    "sparse_chain_300_s": round(res["sparse_chain"][1], 4),
                    "chain_equals_square": _same(torch, res["chain"][0], res["square"][0]),
                    "chain_equals_sparse": _same(torch, res["chain"][0], res["sparse_chain"][0]),
                    "period_search_to_period_s": round(t_per, 4),
                    "period_search_pipelined_s": round(t_per_p, 4), "pipelined_same": bool(pipelined_same),
                    "gamma_3_300_match_golden": bool(golden_ok),
                    "matches_oracle": bool(oracle_ok),
                    "cpu_baseline": {"value": round(len(rows) * 299 * float(n) * n / t_cpu / 1e9, 3),
                                     "unit": "G pairs/s (dense-equivalent)", "cores": O.threads(),
                                     "kind": "oracle", "sample": "%s, %.2f s" % (sample, t_cpu)}}
    return {"workload": "Roman transfer matrices m=6,7,8 to n=300: chain, squaring, period, gamma_R(3..300)",
            "value": round(tot_pairs / tot_t / 1e9, 1), "unit": "G pairs/s (dense chains)", "dtype": "uint16",
            "per_m": per_m}


def leg_config4(mpr, torch, args):
    """256 chains in one graph-captured launch (configuration picked by the
    library's model with the autotuner's weights), the f16 form of it, and
    the plain per-instance path (one chain after another) on the same GPU;
    the oracle on sampled rows of three chains."""
    import oracle as O
    import synth

    inst = synth.batch_instances(256, seed=4)
    t_gen = time.perf_counter()
    mats, chains = [], []
    for d in inst:
        X = synth.random_matrix(d["n"], d["n"], d["seed"], 0, 31, 0.25)
        mats.append(X)
        chains.append((mpr.to_device(X), d["e"], mpr.alloc_matrix(d["n"], d["n"]),
                       torch.empty(d["n"], dtype=torch.int64, device="cuda")))
    gen_s = time.perf_counter() - t_gen
    pairs = sum((d["e"] - 1) * float(d["n"]) ** 3 for d in inst)
    ws = mpr.workspace(mpr.batch_workspace_size(chains))
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    forms = {}
    for arith in ("u16", "f16"):
        with mpr.arith_scope(arith):
            mpr.batch_plan(chains, ws, stream)
        cfg = mpr.batch_plan_info(ws)[0]
        g = mpr.batch_graph_create(ws, st, stream)
        mpr.graph_launch(g, stream)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.batch_reps):
            mpr.graph_launch(g, stream)
        stream.synchronize()
        t = (time.perf_counter() - t0) / args.batch_reps
        mpr.graph_destroy(g)
        mpr.check_status(st)
        forms[arith] = (cfg, t, [(N.clone(), R.clone()) for (_, _, N, R) in chains])
    wsi = mpr.workspace(max(mpr.power_workspace_size(d["n"], d["e"], mpr.CHAIN) for d in inst))

    def solo():
        for (A, e, N, R) in chains:
            mpr.minplus_power(A, e, mpr.CHAIN, N, R, wsi, check=False, d_status=st)

    _, t_solo = _timed(torch, solo)
    mpr.check_status(st)
    same = all(_same(torch, (N, R), b) for (_, _, N, R), b in zip(chains, forms["u16"][2]))
    same_f16 = all(_same(torch, a, b) for a, b in zip(forms["u16"][2], forms["f16"][2]))
    order = sorted(range(len(inst)), key=lambda i: -inst[i]["n"])
    picks = [order[0], order[len(order) // 2], order[-1]]
    t0 = time.perf_counter()
    ok, sampled = True, 0.0
    for i in picks:
        n, e = inst[i]["n"], inst[i]["e"]
        rows = np.sort(np.random.default_rng(i).choice(n, args.config4_rows, replace=False))
        Nr, Rr = O.chain_rows(O.from_u16(mats[i]), rows, e)
        N, R = forms["u16"][2][i]
        ok = ok and np.array_equal(_rows(torch, N, rows), O.to_u16(Nr)) and np.array_equal(R.cpu().numpy()[rows], Rr)
        sampled += len(rows) * (e - 1) * float(n) * n
    t_cpu = time.perf_counter() - t0
    cfg, t_batch, _ = forms["u16"]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    binfo = mpr.batch_config_info(cfg)
    return {"workload": "256 chains, N log-uniform [256,4096], e uniform [8,128], U[0,31] 25% inf (seed 4)",
            "value": round(pairs / t_batch / 1e9, 1), "unit": "G pairs/s", "dtype": "uint16",
            "total_pairs": pairs, "batch_config": cfg, "panel_rows": binfo["panel_rows"],
            "batched_s": round(t_batch, 3), "pct_valu_peak": round(100 * pairs / t_batch / 1e9 /
                                                                   valu_peak_gpairs(cus, "u16"), 2),
            "per_instance_s": round(t_solo, 3), "per_instance_gpairs": round(pairs / t_solo / 1e9, 1),
            "speedup_vs_per_instance": round(t_solo / t_batch, 2),
            "batched_equals_per_instance": bool(same),
            "f16_form": {"batch_config": forms["f16"][0], "batched_s": round(forms["f16"][1], 3),
                         "gpairs": round(pairs / forms["f16"][1] / 1e9, 1),
                         "pct_of_f16_peak": round(100 * pairs / forms["f16"][1] / 1e9 /
                                                  valu_peak_gpairs(cus, "f16"), 2),
                         "bit_identical": bool(same_f16)},
            "sampled_rows_match_oracle": bool(ok), "input_gen_s": round(gen_s, 1),
            "cpu_baseline": {"value": round(sampled / t_cpu / 1e9, 3), "unit": "G pairs/s", "cores": O.threads(),
                             "kind": "oracle",
                             "sample": "%d rows each of the largest, median and smallest chain (all steps), %.1f s"
                                       % (args.config4_rows, t_cpu)}}


# ---------------------------------------------------------------- config 5
def _lat_stats(res, pick=None):
    sel = [r for r in res if pick is None or pick(r)]
    if not sel:
        return None
    lat = np.array([(r["t_done"] - r["t_submit"]) * 1e3 for r in sel])
    return {"count": len(sel), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "max_ms": round(float(lat.max()), 3)}


def _check(goldens, qs, res):
    bad = sum(1 for r in res if r["status"] != 0)
    checked = wrong = 0
    for (_, m, n), r in zip(qs, res):
        exp = expected_gamma(goldens, m, n)
        if exp is not None:
            checked += 1
            wrong += int(r["gamma"] != exp)
    return {"errors": bad, "checked": checked, "mismatches": wrong}


def _closed_loop(serve, S, qs, timeout_s):
    """Every query submitted at once: throughput at saturation."""
    burst = [(0.0, m, n) for (_, m, n) in qs]
    t0 = time.perf_counter()
    res = serve.run_open_loop(S, burst, timeout_s=timeout_s)
    wall = time.perf_counter() - t0
    span = max(r["t_done"] for r in res) - min(r["t_submit"] for r in res)
    return res, {"queries": len(res), "qps": round(len(res) / span, 1), "wall_s": round(wall, 3),
                 **{k: v for k, v in _lat_stats(res).items() if k != "count"}}


def _wait_built(S, count, timeout_s=120.0):
    """Waits until `count` ladder builds have finished (the last giant of a
    ladder answers queries just before its build is marked finished; the
    Roman ladders are kept as byte copies, counted by narrow_builds)."""
    t_end = time.monotonic() + timeout_s
    while S.stats()["narrow_builds"] < count and time.monotonic() < t_end:
        time.sleep(0.002)


def bench_serve(args, mpr, torch, seconds: float):
    """Config 5 (m uniform in 3..9, n uniform in 3..1000; answers checked
    against the stored goldens, m = 9 against Section 4.3's closed form):
    1. cold: a fresh engine meets a Poisson stream at 200 req/s; the first
       request of each m waits for its ladder, built on the build stream
       while warm requests of other m keep being answered;
    2. warm: every ladder resident, the Poisson stream for `seconds`;
    3. saturation: the same engine, every query of a burst submitted at once;
    4. the plain per-instance path on the same GPU: an engine with one query
       per launch and one launch in flight (max_batch 1, slots 1), same burst."""
    import synth
    from paper_2409_17658_amd import serve

    goldens = load_goldens()
    rate = 200.0
    budget = int(args.serve_budget_gb * (1 << 30))
    out = {"offered_qps": rate}
    qs_cold = synth.poisson_queries(rate, int(rate * args.serve_cold_seconds), seed=6, m_range=(3, 9),
                                    n_range=(3, 1000))
    qs = synth.poisson_queries(rate, int(rate * seconds), seed=5, m_range=(3, 9), n_range=(3, 1000))
    qs_burst = synth.poisson_queries(rate, args.serve_burst, seed=7, m_range=(3, 9), n_range=(3, 1000))
    with serve.Server(baby=32, max_n=1000, max_batch=256, slots=4, hbm_budget_bytes=budget) as S:
        if args.serve_cold_seconds > 0:
            res = serve.run_open_loop(S, qs_cold, timeout_s=args.serve_cold_seconds * 4 + 600)
            cold = [r for r in res if r["cold"] == 1]
            m9 = [r for r in cold if r["m"] == 9]
            # warm answers that completed while the m = 9 ladder was building
            overlap = 0
            if m9:  # from the first m = 9 request to the last cold m = 9 answer (the build's end)
                b0, b1 = min(r["t_submit"] for r in m9), max(r["t_done"] for r in m9)
                overlap = sum(1 for r in res if r["cold"] == 0 and r["t_submit"] >= b0 and r["t_done"] <= b1)
            out["cold_leg"] = {"queries": len(res), "seconds": args.serve_cold_seconds,
                               "cold": _lat_stats(res, lambda r: r["cold"] == 1),
                               "warm": _lat_stats(res, lambda r: r["cold"] == 0),
                               "warm_answered_during_m9_build": overlap,
                               # answered while their ladder was still being built
                               "answered_from_building_ladders": S.stats()["early_answers"],
                               "m9_build_wait_s": round(max(r["t_done"] - r["t_submit"] for r in m9), 3) if m9 else None,
                               **_check(goldens, qs_cold, res)}
        build_s = {}
        for m in range(3, 10):  # every ladder resident before the warm leg
            t0 = time.perf_counter()
            r = S.query(m, 1000)
            build_s[m] = round(time.perf_counter() - t0, 3)
            assert r["status"] == 0
        _wait_built(S, 7)
        t0 = time.perf_counter()
        res = serve.run_open_loop(S, qs, timeout_s=seconds * 4 + 600)
        wall = time.perf_counter() - t0
        st0 = S.stats()
        out.update({"queries": len(qs), "achieved_qps": round(len(qs) / wall, 1),
                    "p50_ms": _lat_stats(res)["p50_ms"], "p99_ms": _lat_stats(res)["p99_ms"],
                    "warm": _lat_stats(res, lambda r: r["cold"] == 0), "ready_wait_s": build_s,
                    **_check(goldens, qs, res)})
        b0, sh0 = S.stats()["batches"], S.stats()["shared_reads"]
        res_b, sat = _closed_loop(serve, S, qs_burst, 600)
        sat.update(_check(goldens, qs_burst, res_b))
        sat["launches"] = S.stats()["batches"] - b0
        # queries whose giant power another query of their launch streamed
        sat["shared_reads"] = S.stats()["shared_reads"] - sh0
        sat["max_batch"] = S.stats()["max_batch_seen"]
        out["saturation"] = sat
        stats = S.stats()
        out.update({"batches": st0["batches"], "max_batch": stats["max_batch_seen"], "builds": stats["builds"],
                    "resident_gb": round(stats["resident_bytes"] / (1 << 30), 2), "evictions": stats["evictions"]})
    if args.serve_per_instance:
        with serve.Server(baby=32, max_n=1000, max_batch=1, slots=1, hbm_budget_bytes=budget) as S:
            for m in range(3, 10):
                assert S.query(m, 1000)["status"] == 0
            _wait_built(S, 7)
            res_p, per = _closed_loop(serve, S, qs_burst, 600)
            per.update(_check(goldens, qs_burst, res_p))
            per["same_answers_as_grouped"] = [r["gamma"] for r in res_p] == [r["gamma"] for r in res_b]
        out["per_instance"] = {"form": "one query per launch, one launch in flight (max_batch 1, slots 1)", **per}
        out["saturation"]["speedup_vs_per_instance"] = round(out["saturation"]["qps"] / per["qps"], 2)
    if args.serve_period:
        # Labelled fast mode: Proposition 8's shortcut, not the per-query path.
        with serve.Server(max_n=1000, hbm_budget_bytes=budget, period_mode=True) as S:
            build_s = {}
            for m in range(3, 10):
                t0 = time.perf_counter()
                r = S.query(m, 1000)
                build_s[m] = round(time.perf_counter() - t0, 3)
                assert r["status"] == 0
            res_t, tab = _closed_loop(serve, S, qs_burst, 600)
            tab.update(_check(goldens, qs_burst, res_t))
            tab["same_answers_as_grouped"] = [r["gamma"] for r in res_t] == [r["gamma"] for r in res_b]
            st = S.stats()
        out["period_mode"] = {"form": "labelled fast mode (Proposition 8): per m, one period search with "
                                      "compressed-K steps up to n = 1000, then a table read per query",
                              "build_s": build_s, "query_launches": st["batches"], **tab}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--cfg", type=int, default=-1, help="tile configuration (-1: tile table)")
    ap.add_argument("--workload", default="gemm",
                    choices=["gemm", "config2", "config3", "config4", "serve", "m10", "m11"])
    ap.add_argument("--m11-kmax", type=int, default=45)
    ap.add_argument("--m10-kmax", type=int, default=35)
    ap.add_argument("--with-m9", type=int, default=1, help="config3: also the m = 9 run")
    ap.add_argument("--m10-sparse", type=int, default=1)
    ap.add_argument("--sparse-form", default="auto", choices=["auto", "tiles", "entries"],
                    help="form of the compressed-K chain steps (library default: auto)")
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--f16-form", type=int, default=1, help="also time the step in the f16 form (labelled)")
    ap.add_argument("--slow-reps", type=int, default=3)
    ap.add_argument("--probe", type=int, default=1, help="measure the VALU rate of both instruction mixes")
    ap.add_argument("--probe-iters", type=int, default=20000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the Poisson query stream in the default run (0: none)")
    ap.add_argument("--serve-budget-gb", type=float, default=200.0)
    ap.add_argument("--serve-cold-seconds", type=float, default=12.0,
                    help="length of the cold leg (fresh engine, no ladder built)")
    ap.add_argument("--serve-burst", type=int, default=20000, help="queries of the saturation legs")
    ap.add_argument("--serve-period", type=int, default=1,
                    help="1: also run the labelled period-table mode of the server on the same burst")
    ap.add_argument("--serve-per-instance", type=int, default=1)
    ap.add_argument("--legs", type=int, default=1, help="default run: also the compact config 1-4 legs")
    ap.add_argument("--config2-rows", type=int, default=48)
    ap.add_argument("--config3-rows", type=int, default=128)
    ap.add_argument("--config4-rows", type=int, default=16)
    ap.add_argument("--batch-reps", type=int, default=1)
    ap.add_argument("--batch-cfg", type=int, default=-2,
                    help="config4: batched configuration (-2: time every one and keep the fastest, "
                         "-1: the library's schedule model)")
    ap.add_argument("--per-instance", type=int, default=1, help="config4: also time the per-instance path")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device copy first (scale for the HBM byte counters)")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "gemm_traffic.json"))
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one MI355X only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2409_17658_amd as mpr

    torch.cuda.set_device(0)
    mpr.init(0)
    mpr.set_sparse_form(args.sparse_form)
    if args.copy_calibration:
        copy_calibration(torch)
    if args.workload == "gemm":
        out = bench_gemm(args, mpr, torch)
        if args.legs:
            goldens = load_goldens()
            for name, fn in (("config1", lambda: leg_config1(mpr, torch)),
                             ("config2", lambda: leg_config2(mpr, torch, args)),
                             ("config3", lambda: leg_config3(mpr, torch, goldens, args)),
                             ("config4", lambda: leg_config4(mpr, torch, args))):
                t0 = time.perf_counter()
                out[name] = fn()
                out[name]["leg_s"] = round(time.perf_counter() - t0, 1)
                print("bench: %s done in %.1f s" % (name, out[name]["leg_s"]), file=sys.stderr, flush=True)
                torch.cuda.empty_cache()
        if args.serve_seconds > 0:
            out["serving"] = bench_serve(args, mpr, torch, args.serve_seconds)
        out["host"] = host_cpu()
    elif args.workload == "config2":
        out = bench_config2(args, mpr, torch)
    elif args.workload == "config3":
        out = bench_config3(args, mpr, torch)
    elif args.workload == "config4":
        out = bench_config4(args, mpr, torch)
    elif args.workload == "m10":
        out = bench_m10(args, mpr, torch)
    elif args.workload == "m11":
        out = bench_m11(args, mpr, torch)
    else:
        out = {"metric": "gamma_R query serving, Poisson 200 req/s, m in 3..9, n in 3..1000",
               "unit": "ms", "n_gpus": 1, "higher_is_better": False}
        out["serving"] = bench_serve(args, mpr, torch, args.serve_seconds if args.serve_seconds > 0 else 60.0)
        out["value"] = out["serving"]["p99_ms"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
