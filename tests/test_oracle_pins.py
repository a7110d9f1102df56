"""Pins of the CPU oracle against facts fixed by the paper or by mathematics.

Nothing here compares the oracle with itself: every check reaches the same
number through something else -- a value the paper prints, a closed form,
exhaustive search, an independent dynamic programme along the other axis of
the cylinder, or brute force over walks / index triples.
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O
import synth

INF = O.INF


# ------------------------------------------------------------ words / matrix
def test_word_counts_table1(paper_values):
    """Table 1: C_m for m = 2..11."""
    for m, c in paper_values["word_counts"]["values"].items():
        assert len(O.words(int(m))) == c, m


def test_words_are_exactly_the_correct_words():
    """Definition 4 checked by an independent enumeration with itertools."""
    bad = {(0, 3), (3, 0), (0, 1), (1, 0), (1, 1)}
    for m in range(1, 6):
        ref = [w for w in itertools.product(range(4), repeat=m)
               if all((w[i], w[i + 1]) not in bad for i in range(m - 1))]
        got = [tuple(int(x) for x in w) for w in O.words(m)]
        assert got == ref


def test_transfer_entries_are_column_weights():
    """Corollary 7: finite entries equal 2 p(a) + p(b) of the column word p."""
    for m in (2, 3, 4):
        W = O.words(m)
        A = O.transfer(m)
        wt = 2 * (W == 0).sum(1) + (W == 1).sum(1)
        fin = A != INF
        assert np.all(A[fin] == np.broadcast_to(wt[None, :], A.shape)[fin])
        # every state has an arc in and an arc out (closed walks exist)
        assert fin.any(0).all() and fin.any(1).all()


def _rdf_ok(f, m, n):
    """Roman dominating function on P_m x C_n (rows cycles, columns paths)."""
    for i in range(m):
        for j in range(n):
            if f[i][j]:
                continue
            nb = [f[i][(j + 1) % n], f[i][(j - 1) % n]]
            if i > 0:
                nb.append(f[i - 1][j])
            if i + 1 < m:
                nb.append(f[i + 1][j])
            if 2 not in nb:
                return False
    return True


def test_closed_walks_are_roman_functions():
    """Proposition 6: a closed walk of n arcs in the word digraph decodes to a
    Roman dominating function whose weight is the walk's label.  Decode the
    letters of random closed walks (a -> 2, b -> 1, c/d -> 0) and check."""
    m, n = 3, 5
    W = O.words(m)
    A = O.transfer(m)
    rng = np.random.default_rng(0)
    checked = 0
    for _ in range(4000):
        walk = [int(rng.integers(len(W)))]
        for _ in range(n - 1):
            nxt = np.flatnonzero(A[walk[-1]] != INF)
            walk.append(int(rng.choice(nxt)))
        if A[walk[-1], walk[0]] == INF:
            continue
        f = [[{0: 2, 1: 1, 2: 0, 3: 0}[int(W[walk[j], i])] for j in range(n)] for i in range(m)]
        assert _rdf_ok(f, m, n)
        label = sum(A[walk[j], walk[(j + 1) % n]] for j in range(n))
        assert label == sum(map(sum, f))
        checked += 1
    assert checked > 50


# ------------------------------------------------------------ semiring
def _py_minplus(X, Y):
    """Triple loop straight from the definition, pure Python (tiny sizes)."""
    M, K = len(X), len(X[0])
    N = len(Y[0])
    C = [[INF] * N for _ in range(M)]
    for i in range(M):
        for j in range(N):
            best = INF
            for k in range(K):
                if X[i][k] != INF and Y[k][j] != INF:
                    best = min(best, X[i][k] + Y[k][j])
            C[i][j] = best
    return C


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 2), (7, 4, 9), (16, 16, 16), (5, 31, 3)])
def test_minplus_matches_triple_loop(shape):
    M, K, N = shape
    X = O.from_u16(synth.random_matrix(M, K, 11, 0, 9, 0.3))
    Y = O.from_u16(synth.random_matrix(K, N, 12, 0, 9, 0.4))
    assert O.minplus(X, Y).tolist() == _py_minplus(X.tolist(), Y.tolist())


def test_minplus_all_inf_and_identity():
    n = 9
    X = O.from_u16(synth.random_matrix(n, n, 3, 0, 20, 0.3))
    E = np.full((n, n), INF, dtype=np.int64)
    np.fill_diagonal(E, 0)
    assert np.array_equal(O.minplus(E, X), X)
    assert np.array_equal(O.minplus(X, E), X)
    Z = np.full((n, n), INF, dtype=np.int64)
    assert np.all(O.minplus(X, Z) == INF) and np.all(O.minplus(Z, X) == INF)


def test_scalar_rule_and_associativity():
    """Section 3: A (x) (alpha (x) B) = alpha (x) (A (x) B); (XY)Z = X(YZ)."""
    X = O.from_u16(synth.random_matrix(20, 13, 5, 0, 15, 0.3))
    Y = O.from_u16(synth.random_matrix(13, 17, 6, 0, 15, 0.3))
    Z = O.from_u16(synth.random_matrix(17, 11, 7, 0, 15, 0.3))
    alpha = 37
    Ya = np.where(Y == INF, INF, Y + alpha)
    P, Pa = O.minplus(X, Y), O.minplus(X, Ya)
    assert np.array_equal(np.where(P == INF, INF, P + alpha), Pa)
    assert np.array_equal(O.minplus(O.minplus(X, Y), Z), O.minplus(X, O.minplus(Y, Z)))


def test_carre_walks_theorem1():
    """Theorem 1: (A^k)_ij is the least label of a walk of exactly k arcs."""
    n, kmax = 5, 4
    A = O.from_u16(synth.random_matrix(n, n, 21, 0, 9, 0.45))
    for k in range(1, kmax + 1):
        N, R = O.power_chain(A, k)
        for i in range(n):
            for j in range(n):
                best = INF
                for mid in itertools.product(range(n), repeat=k - 1):
                    path = (i,) + mid + (j,)
                    w = 0
                    for a, b in zip(path, path[1:]):
                        if A[a, b] == INF:
                            w = INF
                            break
                        w += A[a, b]
                    best = min(best, w)
                got = INF if (R[i] == INF or N[i, j] == INF) else R[i] + N[i, j]
                assert got == best, (k, i, j)


def test_canonical_form_reconstructs_raw_power():
    """R_k[i] + N_k[i][j] equals the plain (unnormalised) power."""
    A = O.from_u16(synth.random_matrix(40, 40, 8, 0, 15, 0.3))
    P = A.copy()
    for k in range(2, 7):
        P = O.minplus(P, A)
        N, R = O.power_chain(A, k)
        rec = np.where((N == INF) | (R[:, None] == INF), INF, N + R[:, None])
        assert np.array_equal(rec, P)
        fin = N != INF
        assert np.all(N[fin] >= 0)
        assert all((N[i][N[i] != INF].min() == 0) for i in range(40) if R[i] != INF)


def test_chain_equals_squaring_and_associativity_of_powers():
    """A^a (x) A^b = A^(a+b) in canonical form; chain = binary powering."""
    A = O.transfer(4)
    pw = {e: O.power_chain(A, e) for e in (1, 2, 3, 5, 8, 13, 21)}
    for a, b in [(1, 1), (2, 3), (5, 8), (8, 13), (3, 5)]:
        Nc, Rc = O.product_of_powers(*pw[a], *pw[b])
        Ne, Re = O.power_chain(A, a + b)
        assert np.array_equal(Nc, Ne) and np.array_equal(Rc, Re)
    for e in (2, 7, 13, 21):
        Ns, Rs = O.power_square(A, e)
        Ne, Re = pw[e] if e in pw else O.power_chain(A, e)
        assert np.array_equal(Ns, Ne) and np.array_equal(Rs, Re)


def test_empty_rows_stay_empty():
    A = O.from_u16(synth.random_matrix(12, 12, 9, 0, 9, 0.2))
    A[3, :] = INF
    N, R = O.power_chain(A, 4)
    assert R[3] == INF and np.all(N[3] == INF)
    Ns, Rs = O.power_square(A, 4)
    assert np.array_equal(N, Ns) and np.array_equal(R, Rs)


# ------------------------------------------------------------ gamma_R
@pytest.mark.parametrize("m,ns", [(1, range(3, 8)), (2, range(3, 8)), (3, range(3, 6)), (4, range(3, 5))])
def test_gamma_matches_brute_force(m, ns):
    """Exhaustive 3^(mn) search (no word encoding) vs Algorithm 1."""
    for n in ns:
        assert O.gamma(m, n) == O.brute_gamma(m, n), (m, n)


def test_gamma_matches_row_dp():
    """Independent exact DP along the path axis vs Algorithm 1."""
    for m in range(1, 8):
        for n in range(3, 8):
            assert O.gamma(m, n) == O.rowdp_gamma(m, n), (m, n)


def test_cycle_closed_form():
    """m = 1 is the cycle C_n: gamma_R = ceil(2n/3)."""
    A = O.transfer(1)
    mu, lam, c, g = O.find_period(A, 40)
    for n in range(3, 41):
        assert O.gamma_from_period(n, mu, lam, c, g) == math.ceil(2 * n / 3), n
        assert O.gamma(1, n) == math.ceil(2 * n / 3)


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6])
def test_periods_table2(paper_values, m):
    """Table 2.  The search returns the least (mu, lam); the printed
    (n0, alpha, beta) must then satisfy n0 >= mu, lam | alpha and
    beta = c * alpha / lam (Lemma 2).  m = 4 prints (16, 5, 10) whose least
    form is (16, 1, 2)."""
    n0, alpha, beta = paper_values["periods"]["values"][str(m)]
    mu, lam, c, g = O.find_period(O.transfer(m), 60)
    assert mu is not None
    assert n0 >= mu and alpha % lam == 0 and beta == c * (alpha // lam)
    if m != 4:
        assert (mu, lam, c) == (n0, alpha, beta)
    else:
        assert (mu, lam, c) == (16, 1, 2)
    # the printed relation itself: A^(n0+alpha) = beta (x) A^(n0)
    A = O.transfer(m)
    N0, R0 = O.power_chain(A, n0)
    N1, R1 = O.power_chain(A, n0 + alpha)
    assert np.array_equal(N0, N1) and np.all(R1 - R0 == beta)


def test_gamma_small_tables_match_row_dp_m8_m9():
    """For m = 8, 9 and n <= 7 the row DP is cheap; compare with the paper's
    closed form for m = 9 (4n if 5 | n else 4n + 2)."""
    for n in range(3, 8):
        g9 = O.rowdp_gamma(9, n)
        assert g9 == (4 * n if n % 5 == 0 else 4 * n + 2), n


@pytest.mark.parametrize("m", [4, 5, 6, 7])
def test_remark13_multiples_of_five(m):
    """Corollary 12 / Remark 13: gamma_R = 2(m+1)n/5 for m, n >= 4, 5 | n."""
    A = O.transfer(m)
    mu, lam, c, g = O.find_period(A, 40)
    for n in (5, 10, 15, 20, 25, 50, 100, 300):
        assert O.gamma_from_period(n, mu, lam, c, g) == 2 * (m + 1) * n // 5, (m, n)


@pytest.mark.slow
def test_closed_form_m7_with_erratum(paper_values):
    """Section 4.3's formula for m = 7 holds for every n in 3..300 except
    n = 6, where the transfer method and the independent row DP both give
    20 (the formula prints ceil(96/5) + 1 = 21)."""
    A = O.transfer(7)
    mu, lam, c, g = O.find_period(A, 40)
    assert (mu, lam, c) == tuple(paper_values["periods"]["values"]["7"])
    for n in range(3, 301):
        got = O.gamma_from_period(n, mu, lam, c, g)
        ref = math.ceil(16 * n / 5) + (0 if n % 5 == 0 else 1)
        if n == 6:
            assert got == 20 and O.rowdp_gamma(7, 6) == 20
        else:
            assert got == ref, n


def test_row_dp_confirms_m8_n3_erratum():
    """Section 4.3's m = 8 formula gives 12 at n = 3; the row DP and the
    brute-force-checked transfer method give 13 (and 16, 18 at n = 4, 5)."""
    assert O.rowdp_gamma(8, 3) == 13
    assert O.rowdp_gamma(8, 4) == math.ceil(18 * 4 / 5) + 1
    assert O.rowdp_gamma(8, 5) == 18


# ------------------------------------------------------------ generators
def test_splitmix64_published_vector():
    """First outputs of SplitMix64 seeded with 1234567 (reference C code)."""
    assert [int(x) for x in synth.splitmix64(1234567, 0, 3)] == [
        6457827717110365317, 3203168211198807973, 9817491932198370423]


def test_random_matrix_law():
    A = synth.random_matrix(512, 512, 1, 0, 15, 0.30)
    inf = (A == 0xFFFF).mean()
    assert abs(inf - 0.30) < 0.01
    fin = A[A != 0xFFFF]
    assert fin.min() == 0 and fin.max() == 15
    # counter-based: a sub-block drawn alone equals the same rows of the whole
    B = synth.random_matrix(512, 512, 1, 0, 15, 0.30, chunk_rows=7)
    assert np.array_equal(A, B)


def test_entrywise_and_row_restricted_helpers():
    """minplus_at against the pure-Python triple loop; chain_rows and
    transfer_rows against whole-matrix computations."""
    X = O.from_u16(synth.random_matrix(23, 17, 41, 0, 9, 0.3))
    Y = O.from_u16(synth.random_matrix(17, 29, 42, 0, 9, 0.4))
    ref = _py_minplus(X.tolist(), Y.tolist())
    ii, jj = np.meshgrid(np.arange(23), np.arange(29), indexing="ij")
    got = O.minplus_at(X, Y, ii.ravel(), jj.ravel()).reshape(23, 29)
    assert got.tolist() == ref
    A = O.from_u16(synth.random_matrix(60, 60, 43, 0, 20, 0.5))
    N, R = O.power_chain(A, 7)
    rows = [0, 13, 59]
    Nr, Rr = O.chain_rows(A, rows, 7)
    assert np.array_equal(Nr, N[rows]) and np.array_equal(Rr, R[rows])
    T = O.transfer(5)
    assert np.array_equal(O.transfer_rows(5, [0, 7, 286]), T[[0, 7, 286]])


@pytest.mark.parametrize("shape", [(1, 1, 1), (3, 5, 2), (7, 4, 9), (16, 16, 16), (5, 31, 3)])
def test_listed_product_matches_triple_loop(shape):
    """The product over a right operand given by its finite entries, against
    the pure-Python triple loop (an all-infinite row and column included)."""
    M, K, N = shape
    X = O.from_u16(synth.random_matrix(M, K, 51, 0, 9, 0.3))
    Y = O.from_u16(synth.random_matrix(K, N, 52, 0, 9, 0.4))
    Y[K // 2, :] = INF
    Y[:, N // 2] = INF
    assert O.minplus_rows(X, O.finite_rows(Y)).tolist() == _py_minplus(X.tolist(), Y.tolist())


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 7])
def test_transfer_arcs_are_the_finite_entries(m):
    """The arc lists equal the finite entries of the whole matrix (whose
    entries are pinned by exhaustive search and the row DP)."""
    start, col, val, n = O.transfer_arcs(m)
    fs, fc, fv, fn = O.finite_rows(O.transfer(m))
    assert n == fn and np.array_equal(start, fs) and np.array_equal(col, fc) and np.array_equal(val, fv)


def test_transfer_arc_counts():
    """Arc counts nnz(A) for m = 1..9 (counted from the rule lists; m = 8
    and 9 without the dense matrix), and every state has an arc out."""
    want = [7, 33, 167, 836, 4195, 21043, 105566, 529584, 2656733]
    for m, nnz in enumerate(want, start=1):
        start, _, _, n = O.transfer_arcs(m)
        assert start[-1] == nnz and n == len(O.words(m)) and np.all(np.diff(start) >= 1), m


def test_sparse_chain_rows_equal_the_dense_chain():
    """Rows of A^k followed through the arc lists equal the rows of the
    whole-matrix chain, for every k."""
    m, e, rows = 6, 25, [0, 1, 400, 847]
    A = O.transfer(m)
    seen = {}
    O.chain_rows_sparse(O.transfer_rows(m, rows), O.transfer_arcs(m), e,
                        on_step=lambda k, N, R: seen.__setitem__(k, (N.copy(), R.copy())))

    def check(k, N, R):
        assert np.array_equal(seen[k][0], N[rows]) and np.array_equal(seen[k][1], R[rows]), k

    O.power_chain(A, e, on_step=check)


def _raw_period_brute(A, K=12):
    """Least (mu, lam) and a c with A^(mu+lam) = c (x) A^mu, from raw powers
    (the definition, no canonical forms); c = 0 when A^mu has no finite entry."""
    P = {1: O.from_u16(O.to_u16(A)) if A.dtype == np.uint16 else A.astype(np.int64)}
    for k in range(2, K + 1):
        P[k] = O.minplus(P[k - 1], P[1])
    for mu in range(1, K):
        for lam in range(1, K - mu + 1):
            X, Y = P[mu], P[mu + lam]
            if not np.array_equal(X == O.INF, Y == O.INF):
                continue
            fin = X != O.INF
            d = np.unique(Y[fin] - X[fin])
            if len(d) == 0:
                return mu, lam, 0
            if len(d) == 1:
                return mu, lam, int(d[0])
    return None


def test_find_period_degenerate_matrices():
    """Pins the period search on tiny and degenerate matrices against the
    definition on raw powers: a single finite entry, all infinite, a
    nilpotent pattern (powers become all infinite: any c fits, 0 reported),
    a weighted 2-cycle (period 2), a self-loop beside a 2-cycle of another
    mean weight (no periodic regime), and small random ones."""
    I = O.INF
    cases = [np.array([[3]]), np.array([[I]]), np.array([[I, 1], [I, I]]), np.array([[I, 0], [5, I]]),
             np.array([[2, I, I], [I, I, 1], [I, 4, I]])]
    rng = np.random.default_rng(5)
    for _ in range(6):
        M = rng.integers(0, 6, (4, 4)).astype(np.int64)
        M[rng.random((4, 4)) < 0.5] = I
        cases.append(M)
    for A in cases:
        A = A.astype(np.int64)
        want = _raw_period_brute(A) or (None, None, None)  # none: components with different cycle means
        mu, lam, c, _ = O.find_period(A, 12)
        assert (mu, lam, c) == want, (A.tolist(), (mu, lam, c), want)
