"""The f16 arithmetic form is exact only because a uint16 value below 0x800
is its own f16 bit pattern, most of them subnormal: FP16 denormals must be
preserved, not flushed, in every kernel that runs the form.  This compiles
the sources that hold those kernels with the library's own flags and checks
the FP16/FP64 denormal mode of each kernel descriptor (no GPU needed)."""
import os
import re
import subprocess
import tempfile

import pytest

from paper_2409_17658_amd import build as B


@pytest.mark.parametrize("src", ["gemm.hip", "batch.hip", "sparse.hip"])
def test_f16_form_kernels_keep_fp16_denormals(src):
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "k.s")
        cmd = [B._hipcc()] + [f for f in B.CFLAGS if f != "-fPIC"] + [
            "--cuda-device-only", "-S", os.path.join(B.CSRC, src), "-o", out]
        p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        assert p.returncode == 0, p.stdout[-2000:]
        text = open(out).read()
    # one .amdhsa_kernel block per kernel; the f16-form instantiations carry
    # "Lb1E" (template argument true) in their mangled names
    blocks = re.findall(r"\.amdhsa_kernel (\S+)(.*?)\.end_amdhsa_kernel", text, re.S)
    f16 = [(name, body) for name, body in blocks if "Lb1E" in name]
    assert f16, "no f16-form kernels found in " + src
    for name, body in f16:
        m = re.search(r"\.amdhsa_float_denorm_mode_16_64\s+(\d+)", body)
        assert m and m.group(1) == "3", (name, m and m.group(1))
