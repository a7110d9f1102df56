"""The query server: answers equal the oracle's gamma_R, and every answer is
the same when the query runs alone and when it runs inside a Poisson mix
(tolerance 0); a tiny HBM budget forces admission waits and evictions."""
import json
import math
import os
import time

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

_CACHE = {}


def oracle_gamma(m, n):
    if m not in _CACHE:
        A = O.transfer(m)
        _CACHE[m] = O.find_period(A, 60)
    mu, lam, c, g = _CACHE[m]
    return O.gamma_from_period(n, mu, lam, c, g)


def golden_gamma(m, n):
    """Stored gamma_R table (written from the oracle by
    tests/golden/make_roman_golden.py) extended by its period (Proposition 8)."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "roman_m%d.json" % m)) as f:
        d = json.load(f)
    mu, lam, c = d["period"]
    return O.gamma_from_period(n, mu, lam, c, {int(k): v for k, v in d["trace"].items()})


@pytest.fixture(scope="module")
def serve():
    import paper_2409_17658_amd as m
    from paper_2409_17658_amd import serve as s

    m.lib()
    m.init(0)
    return s


def test_server_alone_and_in_mix(serve):
    qs = synth.poisson_queries(400.0, 300, seed=5, m_range=(2, 6), n_range=(3, 200))
    with serve.Server(baby=16, max_n=200, max_batch=64, slots=4, hbm_budget_bytes=8 << 30) as S:
        mixed = serve.run_open_loop(S, qs, timeout_s=240)
        st = S.stats()
        alone = [S.query(m, n)["gamma"] for (_, m, n) in qs[:60]]
    for (t, m, n), r in zip(qs, mixed):
        assert r["status"] == 0
        assert r["gamma"] == oracle_gamma(m, n), (m, n)
    assert alone == [r["gamma"] for r in mixed[:60]]
    assert st["completed"] == len(qs) and st["builds"] == 5
    assert st["batches"] >= 1 and st["max_batch_seen"] >= 1


def test_server_budget_forces_eviction(serve):
    """Budget below two ladders: requests alternate between m = 5 and 6."""
    b5, b6 = serve.ladder_bytes(5, 8, 64), serve.ladder_bytes(6, 8, 64)
    with serve.Server(baby=8, max_n=64, max_batch=16, slots=2, hbm_budget_bytes=max(b5, b6) + 1024) as S:
        out = [S.query(m, n) for m, n in [(5, 40), (6, 41), (5, 63), (6, 9), (5, 3)]]
        st = S.stats()
    for r in out:
        assert r["status"] == 0 and r["gamma"] == oracle_gamma(r["m"], r["n"])
    assert st["evictions"] >= 3 and st["builds"] >= 4


def test_server_rejects_bad_queries(serve):
    with serve.Server(baby=8, max_n=50, max_batch=8, slots=1, hbm_budget_bytes=1 << 30) as S:
        assert S.query(3, 2)["status"] == 1
        assert S.query(3, 51)["status"] == 1
        assert S.query(0, 10)["status"] == 1
        r = S.query(1, 50)
        assert r["status"] == 0 and r["gamma"] == math.ceil(2 * 50 / 3)
        assert S.query(9, 10)["status"] == 2  # its ladder exceeds the 1 GiB budget


def test_server_ladder_boundaries(serve):
    """Queries on the seams of the ladder: n <= B read off the baby traces,
    n = B (the first giant), B + 1, 2B, 2B + 1 and n = max_n, for m = 1..4."""
    B, max_n = 8, 41
    ns = [3, 4, B - 1, B, B + 1, 2 * B, 2 * B + 1, max_n - 1, max_n]
    with serve.Server(baby=B, max_n=max_n, max_batch=16, slots=2, hbm_budget_bytes=1 << 30) as S:
        for m in (1, 2, 3, 4):
            for n in ns:
                r = S.query(m, n)
                assert r["status"] == 0 and r["gamma"] == oracle_gamma(m, n), (m, n, r)


@pytest.mark.parametrize("B,max_n", [(1, 12), (5, 23), (16, 16)])
def test_server_ladder_shapes(serve, B, max_n):
    """B = 1 (the first giant is A itself), an odd B (the chain to A^B starts
    on the other buffer), and max_n <= B (no giant at all): every n."""
    with serve.Server(baby=B, max_n=max_n, max_batch=16, slots=2, hbm_budget_bytes=1 << 30) as S:
        for m in (2, 3, 5):
            for n in range(3, max_n + 1):
                r = S.query(m, n)
                assert r["status"] == 0 and r["gamma"] == oracle_gamma(m, n), (m, n, r)


def test_query_keeps_other_results(serve):
    """A result that arrives while query() waits for its own is handed to
    the next poll(), not dropped."""
    with serve.Server(baby=8, max_n=40, max_batch=8, slots=2, hbm_budget_bytes=1 << 30) as S:
        S.submit(3, 17, 4242)
        time.sleep(0.2)  # let it complete first
        r = S.query(3, 18)
        assert r["gamma"] == oracle_gamma(3, 18)
        held = S.poll(1000)
        assert [h["tag"] for h in held] == [4242] and held[0]["gamma"] == oracle_gamma(3, 17)


@pytest.mark.parametrize("wide_only", [False, True])
def test_server_large_ladders_mixed_batches(serve, wide_only):
    """m = 7 (N = 2507) and m = 8 (N = 7411) queries, alone and mixed in the
    same launches, from the byte copies of the ladders and from the uint16
    powers, against the stored gamma_R tables."""
    ns = [3, 31, 32, 33, 64, 65, 97, 150, 299, 300, 301, 517, 999, 1000]
    qs = [(m, n) for n in ns for m in (7, 8)]
    with serve.Server(baby=32, max_n=1000, max_batch=64, slots=2, hbm_budget_bytes=32 << 30,
                      wide_only=wide_only) as S:
        alone = {q: S.query(*q)["gamma"] for q in qs}
        for k, (m, n) in enumerate(qs):  # one burst: later queries wait for a slot and share launches
            S.submit(m, n, k)
        got, t_end = {}, time.monotonic() + 240
        while len(got) < len(qs) and time.monotonic() < t_end:
            for r in S.poll(20):
                got[r["tag"]] = r
        st = S.stats()
    assert len(got) == len(qs)
    for k, (m, n) in enumerate(qs):
        assert got[k]["status"] == 0
        assert got[k]["gamma"] == alone[(m, n)] == golden_gamma(m, n), (m, n)
    assert st["max_batch_seen"] >= 2
    assert st["narrow_builds"] == (0 if wide_only else 2)


def test_server_shared_giant_groups(serve):
    """Queries of one launch that share a giant power A^(32 i) are answered in
    groups of up to 8 that read it once.  A burst submitted while the ladders
    of m = 7 and m = 8 (N = 2507, 7411) are still being built, so the queries
    on one giant become answerable together (when the build has written it)
    and go in one launch: 20 queries on A^160 of m = 8 (groups of 8, 8, 4),
    10 on A^288 of m = 7 (8, 2) and four alone; every answer equal to its
    answer alone and to the stored tables."""
    qs = [(8, 160 + j) for j in range(1, 21)] + [(7, 288 + j) for j in range(3, 31, 3)]
    qs += [(8, 999), (7, 40), (8, 100), (7, 641)]
    rng = np.random.default_rng(23)
    qs = [qs[k] for k in rng.permutation(len(qs))]
    with serve.Server(baby=32, max_n=1000, max_batch=256, slots=1, hbm_budget_bytes=32 << 30) as S:
        for k, (m, n) in enumerate(qs):
            S.submit(m, n, k)
        got, t_end = {}, time.monotonic() + 240
        while len(got) < len(qs) and time.monotonic() < t_end:
            for r in S.poll(50):
                got[r["tag"]] = r
        # the last answers may come from a ladder whose build is still ending
        while S.stats()["narrow_builds"] < 2 and time.monotonic() < t_end:
            time.sleep(0.01)
        st = S.stats()
        alone = {q: S.query(*q)["gamma"] for q in set(qs)}
        st1 = S.stats()
    assert len(got) == len(qs)
    for k, (m, n) in enumerate(qs):
        assert got[k]["status"] == 0 and got[k]["cold"] == 1
        assert got[k]["gamma"] == alone[(m, n)] == golden_gamma(m, n), (m, n)
    assert st["narrow_builds"] == 2
    assert st["shared_reads"] == (7 + 7 + 3) + (7 + 1)
    assert st1["shared_reads"] == st["shared_reads"]  # one query per launch


def test_server_large_batches(serve):
    """One launch slot and a burst of 200 queries: batches grow past 16
    queries; every answer against the oracle."""
    rng = np.random.default_rng(17)
    qs = [(int(m), int(n)) for m, n in zip(rng.integers(3, 7, 200), rng.integers(3, 201, 200))]
    with serve.Server(baby=16, max_n=200, max_batch=256, slots=1, hbm_budget_bytes=8 << 30) as S:
        for m in range(3, 7):
            S.query(m, 200)  # build the ladders first
        for k, (m, n) in enumerate(qs):
            S.submit(m, n, k)
        got, t_end = {}, time.monotonic() + 120
        while len(got) < len(qs) and time.monotonic() < t_end:
            for r in S.poll(20):
                got[r["tag"]] = r
        st = S.stats()
    assert len(got) == len(qs)
    for k, (m, n) in enumerate(qs):
        assert got[k]["status"] == 0 and got[k]["gamma"] == oracle_gamma(m, n), (m, n)
    assert st["max_batch_seen"] > 16


@pytest.mark.parametrize("wide_only", [False, True])
def test_server_resident_bytes(serve, wide_only):
    """The bytes a ladder holds, as the server accounts them, are the ones
    mpr_server_ladder_bytes states (with and without the byte copies)."""
    with serve.Server(baby=8, max_n=64, max_batch=8, slots=1, hbm_budget_bytes=4 << 30, wide_only=wide_only) as S:
        S.query(6, 40)
        b6 = S.stats()["resident_bytes"]
        S.query(5, 40)
        b56 = S.stats()["resident_bytes"]
    assert b6 == serve.ladder_bytes(6, 8, 64, wide_only)
    assert b56 - b6 == serve.ladder_bytes(5, 8, 64, wide_only)
    assert serve.ladder_bytes(6, 8, 64, False) > serve.ladder_bytes(6, 8, 64, True)


def test_server_busy_poll(serve):
    """The busy-polling worker answers the same as the sleeping one."""
    qs = synth.poisson_queries(400.0, 120, seed=9, m_range=(2, 6), n_range=(3, 120))
    with serve.Server(baby=16, max_n=120, max_batch=64, slots=2, hbm_budget_bytes=4 << 30, busy_poll=True) as S:
        res = serve.run_open_loop(S, qs, timeout_s=120)
    for (_, m, n), r in zip(qs, res):
        assert r["status"] == 0 and r["gamma"] == oracle_gamma(m, n), (m, n)


def test_warm_queries_overlap_a_cold_build(serve):
    """Continuous batching with overlap: an m = 9 request arrives first and
    waits seconds for its ladder (built on the build stream); warm requests
    for m = 3..8 submitted after it are all answered before it, each equal
    to the stored gamma_R table (m = 9: Section 4.3's closed form)."""
    rng = np.random.default_rng(23)
    warm = [(int(m), int(n)) for m, n in zip(rng.integers(3, 9, 150), rng.integers(3, 1001, 150))]
    with serve.Server(baby=32, max_n=1000, max_batch=64, slots=4, hbm_budget_bytes=200 << 30) as S:
        for m in range(3, 9):
            assert S.query(m, 1000)["status"] == 0  # ladders of m = 3..8 resident
        builds0 = S.stats()["builds"]
        S.submit(9, 997, 10 ** 6)
        got, t_end = {}, time.monotonic() + 300
        for k, (m, n) in enumerate(warm):
            S.submit(m, n, k)
            time.sleep(0.004)
        while 10 ** 6 not in got and time.monotonic() < t_end:
            for r in S.poll(20):
                got[r["tag"]] = r
        st = S.stats()
    big = got[10 ** 6]
    assert big["status"] == 0 and big["cold"] == 1 and big["gamma"] == 4 * 997 + 2
    assert st["builds"] == builds0 + 1
    assert len(got) == len(warm) + 1  # every warm answer came before the cold one
    for k, (m, n) in enumerate(warm):
        r = got[k]
        assert r["status"] == 0 and r["cold"] == 0 and r["gamma"] == golden_gamma(m, n), (m, n)
        assert r["t_done"] < big["t_done"] and r["t_submit"] > big["t_submit"]


def test_cold_ladder_answers_progressively(serve):
    """A ladder still being built answers the queries whose giant power is
    already written (the build announces each giant by an event): on a fresh
    engine, m = 8 queries n = 3 (a baby trace), 40 (giant 1), 70 (giant 2),
    500 (giant 15) and 999 (giant 31) submitted at once are answered in giant
    order, the first ones while the later giants are still being computed,
    each equal to the stored gamma_R table."""
    ns = [999, 500, 70, 40, 3]
    with serve.Server(baby=32, max_n=1000, max_batch=64, slots=4, hbm_budget_bytes=200 << 30) as S:
        for k, n in enumerate(ns):
            S.submit(8, n, k)
        got, t_end = {}, time.monotonic() + 120
        while len(got) < len(ns) and time.monotonic() < t_end:
            for r in S.poll(20):
                got[r["tag"]] = r
        st = S.stats()
        assert S.query(8, 999)["gamma"] == golden_gamma(8, 999)  # and from the finished ladder
    t = {n: got[k]["t_done"] for k, n in enumerate(ns)}
    for k, n in enumerate(ns):
        r = got[k]
        assert r["status"] == 0 and r["cold"] == 1 and r["gamma"] == golden_gamma(8, n), n
    assert t[3] <= t[40] < t[500] < t[999]
    assert t[70] < t[999]
    assert st["early_answers"] >= 3 and st["builds"] == 1


def test_small_ladder_not_stuck_behind_large_build(serve):
    """Ladder builds are scheduled shortest first: an m = 8 ladder (N = 7411,
    30 products of about 12 ms) started while the m = 9 ladder (30 products
    of about 0.28 s) is in its giant products is built between them, so an
    m = 8 query needing its last giant is answered within about a second,
    long before the m = 9 build ends (alternating products of the two would
    take about 9 s)."""
    with serve.Server(baby=32, max_n=1000, max_batch=64, slots=4, hbm_budget_bytes=200 << 30) as S:
        S.submit(9, 997, 1)
        time.sleep(2.0)  # m = 9: past its babies, into its giant products
        S.submit(8, 999, 2)
        got, t_end = {}, time.monotonic() + 120
        while len(got) < 2 and time.monotonic() < t_end:
            for r in S.poll(20):
                got[r["tag"]] = r
    big, small = got[1], got[2]
    assert big["status"] == 0 and big["gamma"] == 4 * 997 + 2
    assert small["status"] == 0 and small["gamma"] == golden_gamma(8, 999)
    assert small["t_done"] - small["t_submit"] < 3.0
    assert small["t_done"] < big["t_done"]


def test_server_request_deadline(serve):
    """Requests not launched within request_timeout_s complete with
    MPR_ETIMEDOUT (7): a cold m = 8 query for n = 999 needs the ladder's last
    giant, which takes longer than 20 ms to build; once the ladder is
    resident the same query is answered within the deadline."""
    with serve.Server(baby=32, max_n=1000, max_batch=64, slots=4, hbm_budget_bytes=200 << 30,
                      request_timeout_s=0.02) as S:
        r = S.query(8, 999)
        assert r["status"] == 7 and r["t_done"] - r["t_submit"] >= 0.02
        t_end = time.monotonic() + 60
        while S.stats()["narrow_builds"] < 1 and time.monotonic() < t_end:
            time.sleep(0.01)
        r2 = S.query(8, 999)
        st = S.stats()
    assert r2["status"] == 0 and r2["gamma"] == golden_gamma(8, 999)
    assert st["builds"] == 1


def test_server_cancel(serve):
    """mpr_server_cancel completes a waiting request with MPR_ECANCELED (8);
    requests of other tags, and a cancel of an unknown tag, are unaffected."""
    with serve.Server(baby=32, max_n=1000, max_batch=64, slots=4, hbm_budget_bytes=200 << 30) as S:
        S.submit(8, 999, 1)
        S.submit(8, 998, 2)
        S.cancel(1)
        S.cancel(12345)
        got, t_end = {}, time.monotonic() + 60
        while len(got) < 2 and time.monotonic() < t_end:
            for r in S.poll(20):
                got[r["tag"]] = r
        r3 = S.query(8, 997)
        S.cancel(2)  # already answered: nothing happens
        time.sleep(0.05)
        late = S.poll(0)
    assert got[1]["status"] == 8
    assert got[2]["status"] == 0 and got[2]["gamma"] == golden_gamma(8, 998)
    assert r3["status"] == 0 and r3["gamma"] == golden_gamma(8, 997)
    assert late == []


def test_build_refused_without_free_memory_then_retried(serve):
    """Admission is by the device's free memory as well as the byte budget:
    with almost all of the device's memory held elsewhere (a host-side
    allocation, no fault involved) a ladder that fits the budget is refused
    with MPR_ENOMEM (the idle ladder is evicted first); the failure is not
    kept, so once the memory is back the next request builds and answers."""
    import torch

    with serve.Server(baby=8, max_n=40, max_batch=8, slots=1, hbm_budget_bytes=8 << 30) as S:
        assert S.query(3, 10)["status"] == 0
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        hog = []  # take the device's free memory down to at most 128 MiB
        try:
            for _ in range(64):
                free, _ = torch.cuda.mem_get_info()
                if free <= (128 << 20):
                    break
                hog.append(torch.empty(min(free - (64 << 20), 32 << 30), dtype=torch.uint8, device="cuda"))
            assert torch.cuda.mem_get_info()[0] <= (128 << 20)
            r1 = S.query(4, 20)
        finally:
            del hog
            torch.cuda.empty_cache()
        r2 = S.query(4, 21)
        r3 = S.query(3, 11)
        st = S.stats()
    assert r1["status"] == 2  # MPR_ENOMEM
    assert r2["status"] == 0 and r2["gamma"] == oracle_gamma(4, 21)
    assert r3["status"] == 0 and r3["gamma"] == oracle_gamma(3, 11)
    assert st["evictions"] >= 1


def test_server_period_mode(serve):
    """The labelled fast mode (Proposition 8): each build searches the period
    of A up to max_n and keeps the traces, so a query is a table read (no
    query launch, no resident device memory); every answer equals the
    stored tables (m = 9: Section 4.3's closed form), including n past the
    confirmed period, whose traces come from the period."""
    ns = (3, 4, 5, 17, 31, 32, 33, 100, 299, 641, 999, 1000)
    qs = [(m, n) for m in range(3, 10) for n in ns]
    with serve.Server(max_n=1000, hbm_budget_bytes=64 << 30, period_mode=True) as S:
        for k, (m, n) in enumerate(qs):
            S.submit(m, n, k)
        got, t_end = {}, time.monotonic() + 240
        while len(got) < len(qs) and time.monotonic() < t_end:
            for r in S.poll(50):
                got[r["tag"]] = r
        again = S.query(8, 777)
        bad = S.query(8, 1001)  # past max_n
        st = S.stats()
    assert len(got) == len(qs)
    for k, (m, n) in enumerate(qs):
        exp = (4 * n if n % 5 == 0 else 4 * n + 2) if m == 9 else golden_gamma(m, n)
        assert got[k]["status"] == 0 and got[k]["gamma"] == exp, (m, n)
    assert again["status"] == 0 and again["cold"] == 0 and again["gamma"] == golden_gamma(8, 777)
    assert bad["status"] == 1  # MPR_EINVAL
    assert st["builds"] == 7 and st["batches"] == 0 and st["resident_bytes"] == 0
    assert st["period_answers"] == len(qs) + 1


def test_server_period_mode_budget(serve):
    """Period mode admits a build by its transient bytes: a budget below
    them answers MPR_ENOMEM; one above, after which the bytes are released."""
    need = serve.period_build_bytes(7)
    assert need > 0
    with serve.Server(max_n=300, hbm_budget_bytes=need - 1, period_mode=True) as S:
        r = S.query(7, 100)
    assert r["status"] == 2  # MPR_ENOMEM: could never be admitted
    with serve.Server(max_n=300, hbm_budget_bytes=need, period_mode=True) as S:
        r = S.query(7, 100)
        st = S.stats()
    assert r["status"] == 0 and r["gamma"] == golden_gamma(7, 100)
    assert st["resident_bytes"] == 0 and st["builds"] == 1
