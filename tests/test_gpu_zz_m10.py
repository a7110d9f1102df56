"""m = 10 (64769 states, 8.4 GB per power; the paper could not hold two
such matrices): gamma_R(P_10 x C_n) by the transfer method (compressed-K
chain steps, a ring of 8 resident powers) against the oracle's row DP
(n <= 9, stored golden written by an oracle-only script), Remark 13 and
Theorem 11."""
import json
import os

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_m10_gamma(paper_values):
    import paper_2409_17658_amd as mpr

    mpr.init(0)
    A = mpr.build_transfer(10)
    assert A.shape[0] == paper_values["word_counts"]["values"]["10"]
    print("m10 transfer built", flush=True)
    mu, lam, c, tr = mpr.find_period(A, 35, traces=True, slots=8, sparse=True)
    print("m10 period", mu, lam, c, flush=True)
    with open(os.path.join(HERE, "rowdp_m10.json")) as f:
        rd = {int(k): v for k, v in json.load(f)["gamma"].items()}
    for n, v in rd.items():
        assert tr[n] == v, n
    assert mu is not None
    for n in range(5, 2001, 5):
        assert mpr.gamma_from_period(mu, lam, c, tr, n) == 22 * n // 5
    for n in range(10, 2001):
        assert mpr.gamma_from_period(mu, lam, c, tr, n) >= -(-22 * n // 5)
