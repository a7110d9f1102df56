"""Autotuners of the (min,+) product's tile configuration and of the batched
kernel's configuration.

Products: for each size bucket it times every compiled configuration on an
N x N x N product (mpr_autotune_gemm, HIP events, inside libmpr) and keeps,
per arithmetic (packed uint16, and the f16 form), the fastest; the two size
-> configuration tables are persisted as JSON next to the library
(tile_table.json) and installed with mpr_set_tile_table by load_table().

Batched chains: tune_batch() times one launch of every batched
configuration on a uniform batch (many equal chains, so every
configuration fills the chip and the time measures its tile speed, not its
load balance) and stores each configuration's throughput relative to the
fastest (batch_table.json); load_batch_table() installs them with
mpr_set_batch_weights as the weights of the library's schedule model.

init() calls both loaders.

    python -m paper_2409_17658_amd.autotune [--out PATH] [N ...]   # product tables
    python -m paper_2409_17658_amd.autotune [--out PATH] batch     # batch weights
"""
from __future__ import annotations

import json
import os
import sys

from . import (autotune_gemm, batch_config_count, batch_config_info, gemm_config_count, gemm_config_info, init,
               set_batch_weights, set_tile_table)

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tile_table.json")
BATCH_TABLE = os.path.join(HERE, "batch_table.json")
DEFAULT_SIZES = (64, 256, 512, 848, 1024, 1536, 2048, 2507, 3072, 4096, 6144, 7411, 8192, 12288, 16384)


def tables_from_measurements(rows, configs) -> dict:
    """Per arithmetic, the size -> configuration table: the fastest
    configuration of that arithmetic at each tuned size, bucket bounds at the
    geometric midpoints between tuned sizes, equal neighbours merged."""
    out = {}
    for arith in ("u16", "f16"):
        mine = [c for c, info in enumerate(configs) if info["arith"] == arith]
        table = []
        for i, r in enumerate(rows):
            best = min(mine, key=lambda c: r["ms"][c])
            hi = int((r["n"] * rows[i + 1]["n"]) ** 0.5) if i + 1 < len(rows) else (1 << 62)
            if table and table[-1][1] == best:
                table[-1][0] = hi
            else:
                table.append([hi, best])
        out[arith] = table
    return out


def tune(sizes=DEFAULT_SIZES, reps: int = 3, path: str = TABLE) -> dict:
    init(0, tile_table=False)
    rows = []
    for n in sizes:
        best, ms = autotune_gemm(int(n), reps if n < 12000 else 1)
        rows.append({"n": int(n), "best": best, "ms": [round(x, 4) for x in ms]})
        print("n=%d best=%d %s" % (n, best, gemm_config_info(best)), file=sys.stderr, flush=True)
    configs = [gemm_config_info(c) for c in range(gemm_config_count())]
    out = {"configs": configs, "measurements": rows, "tables": tables_from_measurements(rows, configs)}
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    for t in out["tables"].values():
        set_tile_table([tuple(x) for x in t])
    return out


def load_table(path: str = TABLE) -> bool:
    """Installs the persisted tables if they exist and were tuned on the
    configurations the loaded library has (same count and shapes)."""
    if not os.path.exists(path):
        return False
    with open(path) as f:
        d = json.load(f)
    if len(d.get("configs", [])) != gemm_config_count():
        return False
    for c, info in enumerate(d["configs"]):
        if info != gemm_config_info(c):
            return False
    tables = d.get("tables")
    if not isinstance(tables, dict) or not tables:
        return False
    for t in tables.values():
        set_tile_table([tuple(x) for x in t])
    return True


def tune_batch(chains: int = 128, n: int = 1024, e: int = 9, reps: int = 2, path: str = BATCH_TABLE) -> dict:
    """Times every batched configuration on `chains` chains of an n x n
    matrix raised to e (entries 0..31, a quarter infinite; random bytes made
    on the device) and persists each configuration's throughput relative to
    the fastest."""
    import torch

    from . import alloc_matrix, batch_graph_create, batch_plan, batch_plan_info, batch_workspace_size, \
        graph_destroy, graph_launch, set_batch_config, workspace

    init(0)
    dev = torch.device("cuda")
    g = torch.Generator(device=dev)
    g.manual_seed(12345)
    descs = []
    for _ in range(chains):
        A = alloc_matrix(n, n, dev)
        vals = torch.randint(0, 32, (n, n), device=dev, generator=g, dtype=torch.int32)
        inf = torch.rand((n, n), device=dev, generator=g) < 0.25
        A.view(torch.int16).copy_(torch.where(inf, torch.full_like(vals, -1), vals).to(torch.int16))
        descs.append((A, e, alloc_matrix(n, n, dev), torch.empty(n, dtype=torch.int64, device=dev)))
    ws = workspace(batch_workspace_size(descs), dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.Stream()
    pairs = chains * (e - 1) * float(n) ** 3
    rates = []
    try:
        for cfg in range(batch_config_count()):
            set_batch_config(cfg)
            batch_plan(descs, ws, stream)
            assert batch_plan_info(ws)[0] == cfg
            graph = batch_graph_create(ws, st, stream)
            graph_launch(graph, stream)  # warm-up
            t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            t0.record(stream)
            for _ in range(reps):
                graph_launch(graph, stream)
            t1.record(stream)
            t1.synchronize()
            graph_destroy(graph)
            ms = t0.elapsed_time(t1) / reps
            rates.append(pairs / (ms * 1e-3) / 1e9)
            print("batch cfg %d %s: %.3f ms, %.1f G pairs/s" % (cfg, batch_config_info(cfg), ms, rates[-1]),
                  file=sys.stderr, flush=True)
    finally:
        set_batch_config(-1)
    if int(st.item()) != 0:
        raise RuntimeError("batch tuning run reported status %d" % int(st.item()))
    top = max(rates)
    out = {"configs": [batch_config_info(c) for c in range(batch_config_count())],
           "workload": {"chains": chains, "n": n, "e": e, "reps": reps},
           "gpairs": [round(r, 1) for r in rates], "weights": [round(r / top, 4) for r in rates]}
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    set_batch_weights(out["weights"])
    return out


def load_batch_table(path: str = BATCH_TABLE) -> bool:
    """Installs persisted batch weights if they were measured on the
    batched configurations the loaded library has."""
    if not os.path.exists(path):
        return False
    with open(path) as f:
        d = json.load(f)
    cfgs = d.get("configs", [])
    if len(cfgs) != batch_config_count() or any(info != batch_config_info(c) for c, info in enumerate(cfgs)):
        return False
    set_batch_weights(d["weights"])
    return True


if __name__ == "__main__":
    args = sys.argv[1:]
    out = None
    if "--out" in args:  # where to write the table (default: next to the library)
        k = args.index("--out")
        out = args[k + 1]
        del args[k:k + 2]
    if args[:1] == ["batch"]:
        print(json.dumps(tune_batch(path=out or BATCH_TABLE)["weights"]))
    else:
        sizes = [int(a) for a in args] or DEFAULT_SIZES
        print(json.dumps(tune(sizes, path=out or TABLE)["tables"]))
