"""The stored oracle goldens (tests/golden/roman_m*.json, written by
make_roman_golden.py from the oracle alone) pinned against the paper:
Table 2's periods, Section 4.3's closed forms (with the two printed values
that the independent row DP contradicts), Remark 13, and the row DP."""
import json
import math
import os

import pytest

import oracle as O

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(m):
    with open(os.path.join(HERE, "roman_m%d.json" % m)) as f:
        return json.load(f)


def closed_form(m, n):
    if m == 7:
        return math.ceil(16 * n / 5) + (0 if n % 5 == 0 else 1)
    if m == 8:
        c = math.ceil(18 * n / 5)
        if n % 5 == 0:
            return c
        if n % 5 in (2, 3, 4) or n == 6:
            return c + 1
        return c + 2
    raise ValueError


@pytest.mark.parametrize("m", [6, 7, 8])
def test_golden_period_matches_table2(paper_values, m):
    assert tuple(load(m)["period"]) == tuple(paper_values["periods"]["values"][str(m)])
    assert load(m)["n_states"] == paper_values["word_counts"]["values"][str(m)]


@pytest.mark.parametrize("m", [7, 8])
def test_golden_traces_match_closed_forms(m):
    g = load(m)["trace"]
    errata = {(7, 6): 20, (8, 3): 13}
    for n in range(3, 301):
        if (m, n) in errata:
            assert g[str(n)] == errata[(m, n)] == O.rowdp_gamma(m, n)
        else:
            assert g[str(n)] == closed_form(m, n), (m, n)


@pytest.mark.parametrize("m", [6, 7, 8])
def test_golden_remark13_and_period_consistency(m):
    d = load(m)
    g = {int(k): v for k, v in d["trace"].items()}
    mu, lam, c = d["period"]
    for n in range(5, 301, 5):
        assert g[n] == 2 * (m + 1) * n // 5
    for n in range(mu, 301 - lam):
        assert g[n + lam] - g[n] == c
    for n in range(3, 8):
        assert g[n] == O.rowdp_gamma(m, n)
