"""m = 9 (21909 states, 0.96 GB per power): the period of Table 2 and the
closed form of Section 4.3 (4n if 5 | n else 4n + 2), through the period
search and through the query server's ladders (n up to 1000)."""
import pytest

pytestmark = pytest.mark.gpu


def closed_form_m9(n):
    return 4 * n if n % 5 == 0 else 4 * n + 2


@pytest.fixture(scope="module")
def mpr():
    import paper_2409_17658_amd as m

    m.lib()
    m.init(0)
    return m


def test_m9_period_table2(mpr, paper_values):
    A = mpr.build_transfer(9)
    mu, lam, c, tr = mpr.find_period(A, 40, traces=True, slots=30)
    assert (mu, lam, c) == tuple(paper_values["periods"]["values"]["9"])
    for n in range(3, 41):
        assert tr[n] == closed_form_m9(n), n


def test_m9_server_ladder(mpr):
    from paper_2409_17658_amd import serve

    ns = [3, 4, 5, 31, 32, 33, 64, 65, 97, 300, 511, 512, 513, 777, 998, 999, 1000]
    with serve.Server(baby=32, max_n=1000, max_batch=64, slots=2, hbm_budget_bytes=100 << 30) as S:
        first = S.query(9, 1000)
        assert first["status"] == 0 and first["cold"] == 1
        for k, n in enumerate(ns):
            S.submit(9, n, k)
        got = {}
        while len(got) < len(ns):
            for r in S.poll(100):
                got[r["tag"]] = r
    assert first["gamma"] == closed_form_m9(1000)
    for k, n in enumerate(ns):
        assert got[k]["status"] == 0 and got[k]["gamma"] == closed_form_m9(n), n
