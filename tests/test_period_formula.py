"""The finite-difference solution after Proposition 8 (host functions of the
C ABI, no GPU): against the stored oracle goldens and the paper's closed
forms of Section 4.3 (m = 7, 8, 9; with the two printed values that differ)
and the m = 1 closed form."""
import json
import math
import os

import numpy as np
import pytest

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def mpr():
    import paper_2409_17658_amd as m

    if not os.path.exists(m.LIB_PATH):
        from paper_2409_17658_amd import build

        build.build()
    return m


def golden(m):
    with open(os.path.join(HERE, "roman_m%d.json" % m)) as f:
        d = json.load(f)
    tr = np.zeros(301, dtype=np.int64)
    for k, v in d["trace"].items():
        tr[int(k)] = v
    return tuple(d["period"]), tr


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 7, 8])
def test_extension_reproduces_the_chain(mpr, m):
    (mu, lam, c), tr = golden(m)
    short = tr[: mu + lam]  # only the traces up to the first repeat
    for n in range(1, 301):
        assert mpr.gamma_from_period(mu, lam, c, short, n) == tr[n], (m, n)


def test_formula_matches_section_4_3(mpr):
    for m, form in [(7, lambda n: math.ceil(16 * n / 5) + (n % 5 != 0)),
                    (8, lambda n: math.ceil(18 * n / 5) + (0 if n % 5 == 0 else 1 if n % 5 in (2, 3, 4) else 2)),
                    (1, lambda n: math.ceil(2 * n / 3))]:
        (mu, lam, c), tr = golden(m)
        numer = mpr.period_formula(mu, lam, c, tr[: mu + lam])
        for n in range(mu, 5000):
            v = c * n + numer[n % lam]
            assert v % lam == 0 and v // lam == form(n), (m, n)


def test_formula_m9_from_table2(mpr, paper_values):
    """m = 9: Table 2's (22, 5, 20) with the closed-form boundary values
    gives 4n / 4n + 2 for every n >= 22."""
    mu, lam, c = paper_values["periods"]["values"]["9"]
    tr = np.array([0] + [4 * n if n % 5 == 0 else 4 * n + 2 for n in range(1, mu + lam)], dtype=np.int64)
    numer = mpr.period_formula(mu, lam, c, tr)
    assert sorted(numer.tolist()) == [0, 10, 10, 10, 10]
    for n in range(mu, 3000):
        assert mpr.gamma_from_period(mu, lam, c, tr, n) == (4 * n if n % 5 == 0 else 4 * n + 2)


def test_bad_arguments(mpr):
    tr = np.zeros(10, dtype=np.int64)
    with pytest.raises(mpr.MprError):
        mpr.gamma_from_period(8, 5, 1, tr, 20)  # mu + lam - 1 > kmax
    with pytest.raises(mpr.MprError):
        mpr.gamma_from_period(0, 5, 1, tr, 20)


def test_empty_residue_class_stays_empty(mpr):
    """A directed 2-cycle with arc weights 1: closed walks exist only for
    even lengths, so the trace of A^k is +infinity (MPR_ROW_NONE) for odd k
    and k for even k; A^(k+2) = 2 (x) A^k from k = 1.  The extension and the
    closed form keep the odd class empty instead of adding to infinity."""
    mu, lam, c = 1, 2, 2
    none = mpr.ROW_NONE
    tr = np.array([none, none, 2], dtype=np.int64)  # traces of A^1, A^2 (index 0 unused)
    for n in range(1, 60):
        want = n if n % 2 == 0 else none
        assert mpr.gamma_from_period(mu, lam, c, tr, n) == want, n
    numer = mpr.period_formula(mu, lam, c, tr)
    assert numer[1] == none and numer[0] == 0  # gamma(n) = (2n + 0) / 2 for even n
