"""Write tests/golden/rowdp_m{m}.json: gamma_R(P_m x C_n) for small n by the
oracle's row-axis DP (independent of the transfer matrix), for the sizes the
transfer method cannot check with the oracle itself.

Usage: python tests/golden/make_rowdp_golden.py [m [nmax]]   (default 10 9)
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402


def main(m, nmax):
    out = {"_about": "Written by tests/golden/make_rowdp_golden.py from the oracle's row DP only.", "m": m,
           "gamma": {}}
    for n in range(3, nmax + 1):
        t0 = time.time()
        out["gamma"][str(n)] = O.rowdp_gamma(m, n)
        print("m=%d n=%d gamma=%d %.0fs" % (m, n, out["gamma"][str(n)], time.time() - t0), flush=True)
    with open(os.path.join(HERE, "rowdp_m%d.json" % m), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    a = [int(x) for x in sys.argv[1:]]
    main(a[0] if a else 10, a[1] if len(a) > 1 else 9)
