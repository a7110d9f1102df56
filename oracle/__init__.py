"""Exact CPU oracle for the (min,+) power method (arXiv 2409.17658).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline are the only callers.  The product path (the HIP library and its
Python binding) never imports this package, and this package never imports
the product path.

All arithmetic is exact int64 (C in ``oracle.c``; period search and the
closed forms in this file).  Infinity is ``INF`` (= int64 max) and is never
added.  Conversions to and from the uint16 storage format of the GPU path
(0xFFFF = infinity) happen only at this module's boundary.

Functions and the passages they follow:
  words(m)                    Definition 4 (correct words)
  transfer(m)                 rule lists of Section 4.1 + the labelling of
                              Corollary 7 (arc q->p weighs 2 p(a) + p(b))
  minplus(X, Y)               the (min,+) product of Section 3
  minplus_at(X, Y, ii, jj)    single entries of the same product
  transfer_rows(m, rows)      rows of A(G) alone
  normalise(C)                canonical (N, R) form: row minima pulled out
                              with the scalar rule of Section 3
  product_of_powers(...)      same rule applied to both operands
  chain(A, e)                 A^k = A^(k-1) (x) A  (Algorithm 2, step 3)
  trace(N, R)                 Corollary 7
  find_period(A, kmax)        Lemma 2 / Proposition 8 / Algorithm 2
  gamma_from_period(...)      the finite-difference solution after Prop. 8
  border_transfer(m)          the appendix's border matrix: modified last-row
                              rule, Algorithm 3 (newly dominated vertices),
                              label 10 p(a) + 5 p(b) - 2 nd(q, p)
  border_loss_columns(n, m)   the same minimum by a DP over pairs of column
                              labellings (no word reduction, no Algorithm 3)
  brute_border_loss(m, n)     Definition 14 + the loss, exhaustively
  brute_gamma(m, n)           definition of a Roman dominating function
  rowdp_gamma(m, n)           exact DP along the path axis (independent)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

INF = np.iinfo(np.int64).max
U16_INF = 0xFFFF

_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        i64, p = ctypes.c_int64, ctypes.c_void_p
        L.oracle_words.restype = i64
        L.oracle_words.argtypes = [ctypes.c_int, p]
        L.oracle_follows.restype = ctypes.c_int
        L.oracle_follows.argtypes = [p, p, ctypes.c_int]
        L.oracle_transfer.restype = ctypes.c_int
        L.oracle_transfer.argtypes = [ctypes.c_int, p]
        L.oracle_minplus.restype = ctypes.c_int
        L.oracle_minplus.argtypes = [i64, i64, i64, p, p, p]
        L.oracle_normalise.restype = None
        L.oracle_normalise.argtypes = [i64, i64, p, p]
        L.oracle_product_of_powers.restype = ctypes.c_int
        L.oracle_product_of_powers.argtypes = [i64, p, p, p, p, p, p]
        L.oracle_trace.restype = i64
        L.oracle_trace.argtypes = [i64, p, p]
        L.oracle_brute_gamma.restype = i64
        L.oracle_brute_gamma.argtypes = [ctypes.c_int, ctypes.c_int]
        L.oracle_minplus_at.restype = None
        L.oracle_minplus_at.argtypes = [i64, i64, p, p, p, p, i64, p]
        L.oracle_transfer_rows.restype = ctypes.c_int
        L.oracle_transfer_rows.argtypes = [ctypes.c_int, p, i64, p]
        L.oracle_border_transfer.restype = ctypes.c_int
        L.oracle_border_transfer.argtypes = [ctypes.c_int, p]
        L.oracle_brute_border_loss.restype = i64
        L.oracle_brute_border_loss.argtypes = [ctypes.c_int, ctypes.c_int]
        L.oracle_threads.restype = ctypes.c_int
        L.oracle_threads.argtypes = []
        L.oracle_minplus_rows.restype = ctypes.c_int
        L.oracle_minplus_rows.argtypes = [i64, i64, i64, p, p, p, p, p]
        L.oracle_transfer_arcs.restype = ctypes.c_int
        L.oracle_transfer_arcs.argtypes = [ctypes.c_int, p, p, p, p]
        L.oracle_rowdp_gamma.restype = i64
        L.oracle_rowdp_gamma.argtypes = [ctypes.c_int, ctypes.c_int]
        _lib = L
    return _lib


def threads() -> int:
    """OpenMP threads the oracle's loops run on."""
    return int(lib().oracle_threads())


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int64)


# ---------------------------------------------------------------- storage
def from_u16(a) -> np.ndarray:
    """uint16 storage (0xFFFF = infinity) -> exact int64 with INF."""
    a = np.asarray(a)
    out = a.astype(np.int64)
    out[a == U16_INF] = INF
    return out


def to_u16(a) -> np.ndarray:
    """int64 with INF -> uint16 storage; finite values must be < 0xFFFF."""
    a = np.asarray(a, dtype=np.int64)
    fin = a != INF
    if np.any(a[fin] < 0) or np.any(a[fin] >= U16_INF):
        raise OverflowError("finite value outside [0, 0xFFFE]")
    out = np.full(a.shape, U16_INF, dtype=np.uint16)
    out[fin] = a[fin].astype(np.uint16)
    return out


# ---------------------------------------------------------------- words / matrix
def words(m: int) -> np.ndarray:
    """Correct words of length m (Definition 4) in increasing base-4 order,
    row 1 most significant; letters a=0, b=1, c=2, d=3.  Shape (C_m, m)."""
    L = lib()
    n = L.oracle_words(m, None)
    if n < 0:
        raise ValueError("m out of range")
    out = np.zeros((n, m), dtype=np.uint8)
    L.oracle_words(m, _ptr(out))
    return out


def follows(q, p) -> bool:
    """True when word p can follow word q (rule lists of Section 4.1)."""
    q = np.ascontiguousarray(q, dtype=np.uint8)
    p = np.ascontiguousarray(p, dtype=np.uint8)
    return bool(lib().oracle_follows(_ptr(q), _ptr(p), len(q)))


def transfer(m: int) -> np.ndarray:
    """A(G) of Corollary 7 for P_m x C_n as exact int64 with INF."""
    n = len(words(m))
    A = np.empty((n, n), dtype=np.int64)
    if lib().oracle_transfer(m, _ptr(A)) != 0:
        raise RuntimeError("oracle_transfer failed")
    return A


# ---------------------------------------------------------------- products
def minplus(X, Y) -> np.ndarray:
    """C = X (x) Y in the (min,+) semiring (Section 3), exact int64."""
    X, Y = _c64(X), _c64(Y)
    M, K = X.shape
    K2, N = Y.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    C = np.empty((M, N), dtype=np.int64)
    if lib().oracle_minplus(M, K, N, _ptr(X), _ptr(Y), _ptr(C)) != 0:
        raise MemoryError("oracle_minplus failed")
    return C


def finite_rows(Y):
    """The finite entries of Y row by row: (start, col, val) with row k's
    columns col[start[k]:start[k+1]] (ascending) and values val[...]; the
    shape's column count rides along as the fourth element."""
    Y = _c64(Y)
    fin = Y != INF
    start = np.concatenate([[0], np.cumsum(fin.sum(axis=1))]).astype(np.int64)
    rr, cc = np.nonzero(fin)
    return start, cc.astype(np.int32), Y[rr, cc].astype(np.int64), Y.shape[1]


def minplus_rows(X, Yrows) -> np.ndarray:
    """X (x) Y (Section 3) with Y given by finite_rows() / transfer_arcs():
    the same definition, the infinite entries of Y never visited."""
    X = _c64(X)
    start, col, val, N = Yrows
    M, K = X.shape
    if len(start) != K + 1:
        raise ValueError("inner dimensions differ")
    C = np.empty((M, N), dtype=np.int64)
    lib().oracle_minplus_rows(M, K, N, _ptr(X), _ptr(start), _ptr(col), _ptr(val), _ptr(C))
    return C


def transfer_arcs(m: int):
    """A(G) of Corollary 7 by its finite entries (finite_rows() layout),
    for m whose dense matrix is too large (m = 10: 64769 states)."""
    n = len(words(m))
    count = np.empty(n, dtype=np.int64)
    if lib().oracle_transfer_arcs(m, _ptr(count), None, None, None) != 0:
        raise RuntimeError("oracle_transfer_arcs failed")
    start = np.concatenate([[0], np.cumsum(count)]).astype(np.int64)
    col = np.empty(int(start[-1]), dtype=np.int32)
    val = np.empty(int(start[-1]), dtype=np.int64)
    if lib().oracle_transfer_arcs(m, None, _ptr(start), _ptr(col), _ptr(val)) != 0:
        raise RuntimeError("oracle_transfer_arcs failed")
    return start, col, val, n


def minplus_at(X, Y, ii, jj) -> np.ndarray:
    """Entries (ii[t], jj[t]) of X (x) Y, each from the definition alone."""
    X, Y = _c64(X), _c64(Y)
    ii, jj = _c64(ii), _c64(jj)
    out = np.empty(len(ii), dtype=np.int64)
    lib().oracle_minplus_at(X.shape[1], Y.shape[1], _ptr(X), _ptr(Y), _ptr(ii), _ptr(jj), len(ii), _ptr(out))
    return out


def transfer_rows(m: int, rows) -> np.ndarray:
    """Rows `rows` of A(G) without building the whole matrix."""
    rows = _c64(rows)
    n = len(words(m))
    out = np.empty((len(rows), n), dtype=np.int64)
    if lib().oracle_transfer_rows(m, _ptr(rows), len(rows), _ptr(out)) != 0:
        raise RuntimeError("oracle_transfer_rows failed")
    return out


def normalise(C):
    """(N, r): r_i = min finite entry of row i (INF if none), N = C - r."""
    N = _c64(C).copy()
    M, n = N.shape
    r = np.empty(M, dtype=np.int64)
    lib().oracle_normalise(M, n, _ptr(N), _ptr(r))
    return N, r


def add_offsets(R, r) -> np.ndarray:
    """R + r with INF ("no finite entry") absorbing."""
    R, r = _c64(R), _c64(r)
    out = np.full(R.shape, INF, dtype=np.int64)
    ok = (R != INF) & (r != INF)
    out[ok] = R[ok] + r[ok]
    return out


def product_of_powers(Na, Ra, Nb, Rb):
    """Canonical form of (Ra (+) Na) (x) (Rb (+) Nb)."""
    Na, Ra, Nb, Rb = _c64(Na), _c64(Ra), _c64(Nb), _c64(Rb)
    n = Na.shape[0]
    Nc = np.empty((n, n), dtype=np.int64)
    Rc = np.empty(n, dtype=np.int64)
    if lib().oracle_product_of_powers(n, _ptr(Na), _ptr(Ra), _ptr(Nb), _ptr(Rb), _ptr(Nc), _ptr(Rc)) != 0:
        raise MemoryError("oracle_product_of_powers failed")
    return Nc, Rc


def power_chain(A, e: int, on_step=None):
    """Canonical form of A^e by the chain A^k = A^(k-1) (x) A, k = 2..e.
    on_step(k, N_k, R_k) is called for every k = 1..e when given."""
    A = _c64(A)
    N, R = normalise(A)
    if on_step:
        on_step(1, N, R)
    for k in range(2, e + 1):
        N, r = normalise(minplus(N, A))
        R = add_offsets(R, r)
        if on_step:
            on_step(k, N, R)
    return N, R


def chain_rows(A, rows, e: int):
    """Rows `rows` of the canonical A^e by the same chain, computed alone:
    row i of A^k depends only on row i of A^(k-1) and on A."""
    A = _c64(A)
    N, R = normalise(A[np.asarray(rows)])
    for _ in range(2, e + 1):
        N, r = normalise(minplus(N, A))
        R = add_offsets(R, r)
    return N, R


def chain_rows_sparse(first_rows, Arows, e: int, on_step=None):
    """chain_rows with A given by its finite entries (transfer_arcs() or
    finite_rows()) and its rows `rows` given as first_rows (e.g. from
    transfer_rows()); on_step(k, N_k, R_k) for every k = 1..e when given."""
    N, R = normalise(first_rows)
    if on_step:
        on_step(1, N, R)
    for k in range(2, e + 1):
        N, r = normalise(minplus_rows(N, Arows))
        R = add_offsets(R, r)
        if on_step:
            on_step(k, N, R)
    return N, R


def power_square(A, e: int):
    """Canonical form of A^e by binary powering (squares A^(2^j) and the
    products of the powers picked by the bits of e)."""
    A = _c64(A)
    P = normalise(A)
    acc = None
    while True:
        if e & 1:
            acc = P if acc is None else product_of_powers(acc[0], acc[1], P[0], P[1])
        e >>= 1
        if not e:
            break
        P = product_of_powers(P[0], P[1], P[0], P[1])
    return acc


def trace(N, R) -> int:
    """Corollary 7: min_i (R_i + N_ii); INF when every term is infinite."""
    N, R = _c64(N), _c64(R)
    return int(lib().oracle_trace(N.shape[0], _ptr(N), _ptr(R)))


def gamma(m: int, n: int) -> int:
    """gamma_R(P_m x C_n) by Algorithm 1 (words, A(G), A^n, min diagonal)."""
    if n < 3:
        raise ValueError("C_n is a simple cycle only for n >= 3")
    return trace(*power_chain(transfer(m), n))


# ---------------------------------------------------------------- periodicity
def _class_key(N, R):
    """A power up to a scalar shift: (N, R - min R, which rows are empty)."""
    fin = R != INF
    base = int(R[fin].min()) if fin.any() else 0
    rel = np.where(fin, R - base, INF)
    return to_u16(N).tobytes() + rel.astype(np.int64).tobytes()


def find_period(A, kmax: int, keep_gamma: bool = True):
    """Smallest (mu, lam, c) with A^(mu+lam) = c (x) A^mu, k <= kmax.

    The classes [A^k] up to a scalar shift satisfy [A^(k+1)] = [A (x) A^k]
    (Section 3's scalar rule), so the class sequence is eventually periodic
    and its first repeat gives the least pre-period mu and the least period
    lam; every pair (n0, alpha) with A^(n0+alpha) = beta (x) A^(n0) has
    n0 >= mu and lam | alpha (Lemma 2).  Returns (mu, lam, c, gammas) where
    gammas[k] = trace of A^k for k = 1..K run, or (None, None, None, gammas)
    when no repeat occurs up to kmax.
    """
    A = _c64(A)
    seen = {}
    gam = {}
    N, R = normalise(A)
    k = 1
    while True:
        gam[k] = trace(N, R)
        key = _class_key(N, R)
        if key in seen:
            k0, R0 = seen[key]
            fin = R != INF
            if not fin.any():  # no finite entry: A^(k0+lam) = c (x) A^k0 for every c; report 0
                return k0, k - k0, 0, gam
            diffs = np.unique(R[fin] - R0[fin])
            if len(diffs) != 1:
                raise AssertionError("class keys equal but offsets disagree")
            return k0, k - k0, int(diffs[0]), gam
        seen[key] = (k, R.copy())
        if k >= kmax:
            return None, None, None, gam
        N, r = normalise(minplus(N, A))
        R = add_offsets(R, r)
        k += 1


def gamma_from_period(n: int, mu: int, lam: int, c: int, gam: dict) -> int:
    """Finite-difference solution after Proposition 8: for n >= mu,
    gamma(n) = gamma(mu + (n - mu) mod lam) + c * floor((n - mu) / lam)."""
    if n < mu:
        return gam[n]
    q, r = divmod(n - mu, lam)
    return gam[mu + r] + c * q


# ---------------------------------------------------------------- independent checks
def brute_gamma(m: int, n: int) -> int:
    """Minimum weight over all 3^(mn) labellings that are Roman dominating."""
    v = lib().oracle_brute_gamma(m, n)
    if v < 0:
        raise ValueError("too large for brute force")
    return int(v)


def rowdp_gamma(m: int, n: int) -> int:
    """gamma_R(P_m x C_n) by a DP over the rows (cycles C_n), n <= 9."""
    v = lib().oracle_rowdp_gamma(m, n)
    if v < 0:
        raise ValueError("n out of range for the row DP")
    return int(v)


# ---------------------------------------------------------------- border (loss) matrix
def border_transfer(m: int) -> np.ndarray:
    """The appendix's border matrix for a strip of m rows (signed int64, INF)."""
    n = len(words(m))
    A = np.empty((n, n), dtype=np.int64)
    if lib().oracle_border_transfer(m, _ptr(A)) != 0:
        raise RuntimeError("oracle_border_transfer failed")
    return A


def brute_border_loss(m: int, n: int) -> int:
    """min over almost Roman dominating functions g of 5 g - 2 |D(g)|."""
    v = lib().oracle_brute_border_loss(m, n)
    if v == np.iinfo(np.int64).min:
        raise ValueError("too large for brute force")
    return int(v)


def border_loss_columns(ns, m: int = 4):
    """min of 5 g - 2 |D(g)| over almost Roman dominating functions of the
    m-row strip, for each n in ns, by a transfer matrix over PAIRS of
    consecutive column labellings (3^m each): the arc (a, b) -> (b, c) is
    allowed when every zero of b outside row m has a 2 next to it (in b, or
    in a or c on its row) and costs 5 w(b) - 2 (dominated vertices of b +
    2s in b's row m, which dominate the vertex below the strip).  The trace
    of its n-th power is the minimum over cyclic sequences of n columns."""
    L = 3 ** m
    cols = np.array(list(np.ndindex(*([3] * m))), dtype=np.int64)  # (L, m)
    two = cols == 2
    vert2 = np.zeros_like(two)
    vert2[:, 1:] |= two[:, :-1]
    vert2[:, :-1] |= two[:, 1:]
    S = L * L
    M = np.full((S, S), INF, dtype=np.int64)
    w = cols.sum(1)
    for a in range(L):
        for b in range(L):
            nb = vert2[b][None, :] | two[a][None, :] | two  # b's rows next to a 2, for every c
            ok = ~np.any((cols[b][None, :m - 1] == 0) & ~nb[:, :m - 1], axis=1)
            dom = ((cols[b][None, :] > 0) | nb).sum(1) + int(two[b][m - 1])
            cost = 5 * w[b] - 2 * dom
            cs = np.flatnonzero(ok)
            M[a * L + b, b * L + cs] = cost[cs]
    out = {}
    ns = sorted(ns)
    N, R = normalise(M)
    k = 1
    for target in ns:
        while k < target:
            N, r = normalise(minplus(N, M))
            R = add_offsets(R, r)
            k += 1
        out[target] = trace(N, R)
    return out
