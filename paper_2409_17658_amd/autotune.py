"""Autotuner of the (min,+) product's tile configuration.

For each size bucket it times every compiled configuration on an N x N x N
product (mpr_autotune_gemm, HIP events, inside libmpr) and keeps the
fastest; the size -> configuration table is persisted as JSON next to the
library and installed with mpr_set_tile_table by load_table() (called by
paper_2409_17658_amd.init).

    python -m paper_2409_17658_amd.autotune [N ...]
"""
from __future__ import annotations

import json
import os
import sys

from . import autotune_gemm, gemm_config_count, gemm_config_info, init, set_tile_table

HERE = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(HERE, "tile_table.json")
DEFAULT_SIZES = (64, 256, 512, 848, 1024, 1536, 2048, 2507, 3072, 4096, 6144, 7411, 8192, 12288, 16384)


def tune(sizes=DEFAULT_SIZES, reps: int = 3, path: str = TABLE) -> dict:
    init(0)
    rows = []
    for n in sizes:
        best, ms = autotune_gemm(int(n), reps if n < 12000 else 1)
        rows.append({"n": int(n), "best": best, "ms": [round(x, 4) for x in ms]})
        print("n=%d best=%d %s" % (n, best, gemm_config_info(best)), file=sys.stderr, flush=True)
    # bucket upper bounds: midpoints between tuned sizes (geometric)
    table = []
    for i, r in enumerate(rows):
        hi = int((r["n"] * rows[i + 1]["n"]) ** 0.5) if i + 1 < len(rows) else (1 << 62)
        if table and table[-1][1] == r["best"]:
            table[-1][0] = hi
        else:
            table.append([hi, r["best"]])
    out = {"configs": [gemm_config_info(c) for c in range(gemm_config_count())], "measurements": rows,
           "table": table}
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    set_tile_table([tuple(t) for t in table])
    return out


def load_table(path: str = TABLE) -> bool:
    """Installs a persisted table if one exists and was tuned on the
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
    set_tile_table([tuple(t) for t in d["table"]])
    return True


if __name__ == "__main__":
    sizes = [int(a) for a in sys.argv[1:]] or DEFAULT_SIZES
    print(json.dumps(tune(sizes)["table"]))
