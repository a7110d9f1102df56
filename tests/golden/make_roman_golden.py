"""Write tests/golden/roman_m{m}.json from the CPU oracle alone.

For each m: the least period (mu, lam, c) of A(G)^k, the trace of A(G)^k for
k = 1..KMAX (gamma_R(P_m x C_n) for n >= 3, Corollary 7) and SHA-256 digests
of the canonical form (N_k as little-endian uint16 row-major with 0xFFFF for
infinity, followed by R_k as little-endian int64) at selected k.

Usage: python tests/golden/make_roman_golden.py [m ...]   (default 1..8)
m = 8 takes several minutes on 8 cores.
"""
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402

KMAX = 300
DIGEST_K = sorted(set(range(1, 41)) | {50, 64, 100, 128, 200, 256, 299, 300})


def canonical_digest(N, R):
    return hashlib.sha256(O.to_u16(N).tobytes() + np.ascontiguousarray(R, dtype="<i8").tobytes()).hexdigest()


def main(ms):
    for m in ms:
        t0 = time.time()
        A = O.transfer(m)
        mu, lam, c, _ = O.find_period(A, 60)
        traces = {}
        digests = {}

        def on_step(k, N, R):
            traces[k] = O.trace(N, R)
            if k in DIGEST_K:
                digests[k] = canonical_digest(N, R)
            if k % 25 == 0:
                print("m=%d k=%d %.0fs" % (m, k, time.time() - t0), flush=True)

        O.power_chain(A, KMAX, on_step)
        out = {
            "_about": "Written by tests/golden/make_roman_golden.py from the CPU oracle only.",
            "m": m,
            "n_states": int(A.shape[0]),
            "period": [mu, lam, c],
            "trace": {str(k): int(v) for k, v in sorted(traces.items())},
            "digest_sha256": {str(k): v for k, v in sorted(digests.items())},
        }
        with open(os.path.join(HERE, "roman_m%d.json" % m), "w") as f:
            json.dump(out, f, indent=1)
        print("m=%d done in %.0fs period=%s" % (m, time.time() - t0, (mu, lam, c)), flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [1, 2, 3, 4, 5, 6, 7, 8])
