"""Host-side checks of bench.py's contract (no GPU: each case exits before
the first device call)."""
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)


def test_more_than_one_gpu_is_refused_with_a_message():
    p = _bench("--gpus", "2")
    assert p.returncode == 2 and "one MI355X" in p.stderr and p.stdout == ""


def test_unknown_sparse_form_is_refused():
    p = _bench("--sparse-form", "dense")
    assert p.returncode == 2 and "--sparse-form" in p.stderr


def test_traffic_counters_match_the_product_sources():
    """The HBM traffic reported beside the headline comes from counter runs
    taken on these product sources; the stored digest must match them (a
    changed kernel reports no traffic until the counters are taken again)."""
    sys.path.insert(0, ROOT)
    import bench

    with open(os.path.join(ROOT, "profiles", "gemm_traffic.json")) as f:
        stored = json.load(f)
    assert stored["kernel_source_sha"] == bench.kernel_source_digest()
    assert bench.load_traffic(os.path.join(ROOT, "profiles", "gemm_traffic.json"), 0) == \
        stored["configs"]["0"]["bytes_per_launch"]
