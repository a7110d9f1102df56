"""Host code under AddressSanitizer + UndefinedBehaviorSanitizer: the C
oracle (gcc) and the host-only entry points of the C ABI (hipcc, sanitizers
on the host side only), each driven by a small C program."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")


def _run(cmd, cwd=None, env=None):
    p = subprocess.run(cmd, cwd=cwd, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=600)
    return p.returncode, p.stdout


def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    rc, out = _run(["gcc", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"), "-o", exe])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
    rc, out = _run([exe], env=env)
    assert rc == 0 and "ok" in out, out


@pytest.mark.skipif(not os.path.exists("/opt/rocm/bin/hipcc"), reason="hipcc not installed")
def test_abi_host_entry_points_under_asan_ubsan(tmp_path):
    hipcc = "/opt/rocm/bin/hipcc"
    csrc = os.path.join(ROOT, "paper_2409_17658_amd", "csrc")
    srcs = sorted(os.path.join(csrc, f) for f in os.listdir(csrc) if f.endswith(".hip"))
    objs = []
    for s in srcs:
        o = str(tmp_path / (os.path.basename(s) + ".o"))
        rc, out = _run([hipcc, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
                        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                        "-c", s, "-o", o])
        assert rc == 0, out
        objs.append(o)
    drv = str(tmp_path / "driver.o")
    rc, out = _run([hipcc, "-O1", "-g", "-x", "c++", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fsanitize=undefined", "-c", os.path.join(SAN, "abi_host_driver.c"), "-o", drv])
    assert rc == 0, out
    exe = str(tmp_path / "abi_san")
    rc, out = _run([hipcc, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
                    "-fsanitize=undefined", drv] + objs + ["-o", exe])
    assert rc == 0, out
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:protect_shadow_gap=0")
    rc, out = _run([exe], env=env)
    assert rc == 0 and "ok" in out, out
