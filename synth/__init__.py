"""Seeded synthetic inputs, shared by the tests, the benchmark and the smoke check.

This module holds none of the method's arithmetic: it only draws the input
matrices, instance lists and query streams that both the HIP path and the
oracle then consume (the same bytes go to both sides).

Random numbers come from the SplitMix64 stream (Steele, Lea and Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014): the t-th
output (t = 0, 1, ...) of the stream seeded with s is
    mix(s + (t + 1) * 0x9E3779B97F4A7C15 mod 2^64)
with the published finaliser
    z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31.
Being counter-based, any element can be drawn on its own, so matrices are
generated in row chunks.

Entry law of a random matrix (storage uint16, 0xFFFF = infinity): element t
(row-major index) is infinite when the high 32 bits of z_t are below
inf_frac * 2^32, otherwise lo + (low 32 bits of z_t) mod (hi - lo + 1).
"""
from __future__ import annotations

import math

import numpy as np

U16_INF = 0xFFFF
_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * _M1
    z = z ^ (z >> np.uint64(27))
    z = z * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, t0: int, count: int) -> np.ndarray:
    """Outputs t0 .. t0+count-1 of the SplitMix64 stream seeded with `seed`."""
    with np.errstate(over="ignore"):
        t = np.arange(t0 + 1, t0 + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + t * _GOLDEN
        return _mix(z)


def uniform01(seed: int, count: int, t0: int = 0) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of the stream."""
    return (splitmix64(seed, t0, count) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def random_matrix(rows: int, cols: int, seed: int, lo: int = 0, hi: int = 15,
                  inf_frac: float = 0.30, ld: int | None = None, chunk_rows: int = 1024) -> np.ndarray:
    """rows x cols uint16 matrix (row stride ld >= cols; padding columns are
    infinite) with the entry law in the module docstring."""
    ld = cols if ld is None else ld
    if ld < cols:
        raise ValueError("ld < cols")
    out = np.full((rows, ld), U16_INF, dtype=np.uint16)
    thr = np.uint64(int(round(inf_frac * 4294967296.0)))
    span = np.uint64(hi - lo + 1)
    for r0 in range(0, rows, chunk_rows):
        r1 = min(rows, r0 + chunk_rows)
        z = splitmix64(seed, r0 * cols, (r1 - r0) * cols).reshape(r1 - r0, cols)
        vals = (np.uint64(lo) + (z & np.uint64(0xFFFFFFFF)) % span).astype(np.uint16)
        vals[(z >> np.uint64(32)) < thr] = U16_INF
        out[r0:r1, :cols] = vals
    return out


def banded_matrix(n: int, w: int = 64, ld: int | None = None) -> np.ndarray:
    """Structured family whose powers keep spreading out:
    A_ij = |i-j| + ((7 i + 13 j) mod 4) when |i-j| <= w, else infinite."""
    ld = n if ld is None else ld
    i = np.arange(n, dtype=np.int64)[:, None]
    j = np.arange(n, dtype=np.int64)[None, :]
    d = np.abs(i - j)
    vals = d + (7 * i + 13 * j) % 4
    out = np.full((n, ld), U16_INF, dtype=np.uint16)
    out[:, :n] = np.where(d <= w, vals, U16_INF).astype(np.uint16)
    return out


def batch_instances(count: int = 256, seed: int = 4, nmin: int = 256, nmax: int = 4096,
                    emin: int = 8, emax: int = 128):
    """Instance list of the batched workload: sizes log-uniform in
    [nmin, nmax] (rounded to integers), exponents uniform in [emin, emax],
    and the seed each instance's matrix is drawn from."""
    u = uniform01(seed, 2 * count)
    out = []
    for i in range(count):
        n = int(round(math.exp(math.log(nmin) + u[2 * i] * (math.log(nmax) - math.log(nmin)))))
        e = emin + int(u[2 * i + 1] * (emax - emin + 1))
        out.append({"n": max(nmin, min(nmax, n)), "e": min(emax, e), "seed": seed * 100003 + i})
    return out


def poisson_queries(rate: float, count: int, seed: int = 5, m_range=(3, 9), n_range=(3, 1000)):
    """Open-loop query stream: exponential gaps of mean 1/rate seconds,
    m and n uniform over their inclusive ranges.  Returns a list of
    (arrival_time_s, m, n)."""
    u = uniform01(seed, 3 * count)
    t = 0.0
    out = []
    for i in range(count):
        t += -math.log(1.0 - u[3 * i]) / rate
        m = m_range[0] + int(u[3 * i + 1] * (m_range[1] - m_range[0] + 1))
        n = n_range[0] + int(u[3 * i + 2] * (n_range[1] - n_range[0] + 1))
        out.append((t, min(m, m_range[1]), min(n, n_range[1])))
    return out
