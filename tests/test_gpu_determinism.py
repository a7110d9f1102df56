"""Determinism: the same call twice gives the same bits.  The kernels' only
atomics are minima (order-independent) and work-list counters (which decide
who computes an item, not what it is), so the product, the batched launch,
the period search and the server must repeat exactly."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpr():
    import paper_2409_17658_amd as m

    m.lib()
    m.init(0)
    return m


def test_product_and_grid_form_repeat(mpr):
    X = synth.random_matrix(3001, 2049, 131, 0, 15, 0.3)
    Y = synth.random_matrix(2049, 3003, 132, 0, 15, 0.3)
    A, B = mpr.to_device(X), mpr.to_device(Y)
    C1 = mpr.minplus_gemm(A, B)
    C2 = mpr.minplus_gemm(A, B)
    C3 = mpr.minplus_gemm(A, B, spare=True)
    assert torch.equal(C1, C2) and torch.equal(C1, C3)


def test_batch_repeats(mpr):
    inst = synth.batch_instances(12, seed=9, nmin=64, nmax=700, emin=2, emax=20)
    chains = []
    for d in inst:
        A = mpr.to_device(synth.random_matrix(d["n"], d["n"], d["seed"], 0, 31, 0.25))
        chains.append((A, d["e"], mpr.alloc_matrix(d["n"], d["n"]), torch.empty(d["n"], dtype=torch.int64,
                                                                                  device="cuda")))
    mpr.batch_power(chains)
    first = [(mpr.to_host(N).copy(), R.cpu().numpy().copy()) for (_, _, N, R) in chains]
    for (_, _, N, R) in chains:
        N.view(torch.int16).fill_(0)
        R.fill_(0)
    mpr.batch_power(chains)
    for (_, _, N, R), (N1, R1) in zip(chains, first):
        assert np.array_equal(mpr.to_host(N), N1) and np.array_equal(R.cpu().numpy(), R1)


def test_period_search_repeats(mpr):
    A = mpr.build_transfer(7)
    r1 = mpr.find_period(A, 60, sparse=True)
    r2 = mpr.find_period(A, 60, sparse=True)
    assert r1[:3] == r2[:3] and list(r1[3]) == list(r2[3])


def test_server_repeats(mpr):
    from paper_2409_17658_amd import serve

    qs = [(m, n) for m in (3, 5, 7) for n in (3, 40, 333, 1000)]
    with serve.Server(baby=32, max_n=1000, max_batch=64, slots=2, hbm_budget_bytes=32 << 30) as S:
        a = [S.query(m, n)["gamma"] for m, n in qs]
        b = [S.query(m, n)["gamma"] for m, n in qs]
    assert a == b
