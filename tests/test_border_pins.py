"""The appendix's border ("loss") matrix in the oracle, pinned by the
definition itself (exhaustive almost Roman dominating functions, a DP over
pairs of column labellings that uses neither the word reduction nor
Algorithm 3) and by the paper's stated result for m = 4."""
import numpy as np
import pytest

import oracle as O


def traces(m, ns):
    A = O.border_transfer(m)
    mu, lam, c, g = O.find_period(A, 80)
    return {n: O.gamma_from_period(n, mu, lam, c, g) for n in ns}, (mu, lam, c)


@pytest.mark.parametrize("m,ns", [(2, range(3, 9)), (3, range(3, 6)), (4, range(3, 5))])
def test_border_matches_exhaustive_definition(m, ns):
    t, _ = traces(m, ns)
    for n in ns:
        assert t[n] == O.brute_border_loss(m, n), (m, n)


@pytest.mark.parametrize("m,nmax", [(2, 10), (3, 10), (4, 12)])
def test_border_matches_column_pair_dp(m, nmax):
    ns = list(range(3, nmax + 1))
    t, _ = traces(m, ns)
    cols = O.border_loss_columns(ns, m)
    assert [t[n] for n in ns] == [cols[n] for n in ns]


def test_border_m4_appendix_result(paper_values):
    """Appendix, last paragraph: Algorithm 2 on the border matrix for m = 4
    gives (n0, a, b) = (30, 1, 1), and 2 L_a(n) = n for 10 <= n <= 30.  The
    transfer method and the independent column DP both give 2 L_a(11) = 12
    (the bound 2 L_a(n) >= n that Lemma 10 needs holds there too)."""
    t, per = traces(4, range(3, 301))
    assert per == tuple(paper_values["loss_border_m4"]["period"])
    for n in range(10, 301):
        if n == 11:
            assert t[n] == 12
        else:
            assert t[n] == n, n
    assert min(t[n] - n for n in range(10, 301)) >= 0


def test_newly_dominated_counts_dominated_vertices():
    """Sum of Algorithm 3's counts over a closed walk equals |D(g)| of the
    function it encodes (checked by decoding random closed walks, m = 4)."""
    m, n = 4, 6
    W = O.words(m)
    A = O.border_transfer(m)
    rng = np.random.default_rng(1)
    seen = 0
    for _ in range(3000):
        walk = [int(rng.integers(len(W)))]
        for _ in range(n - 1):
            nxt = np.flatnonzero(A[walk[-1]] != O.INF)
            walk.append(int(rng.choice(nxt)))
        if A[walk[-1], walk[0]] == O.INF:
            continue
        f = np.array([[{0: 2, 1: 1, 2: 0, 3: 0}[int(W[walk[j], i])] for j in range(n)] for i in range(m)])
        two = f == 2
        nb2 = np.roll(two, 1, 1) | np.roll(two, -1, 1)
        nb2[1:] |= two[:-1]
        nb2[:-1] |= two[1:]
        D = int(((f > 0) | nb2).sum() + two[m - 1].sum())
        label = sum(A[walk[j], walk[(j + 1) % n]] for j in range(n))
        assert label == 5 * f.sum() - 2 * D
        seen += 1
    assert seen > 20
