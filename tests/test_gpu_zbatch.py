"""Batched power chains (one launch) against the oracle, against
the same chains run one at a time, and across HIP graph replays."""
import numpy as np
import pytest
import torch

import oracle as O
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mpr():
    import paper_2409_17658_amd as m

    m.lib()
    m.init(0)
    return m


def _small_batch(mpr):
    sizes = [(40, 2), (700, 5), (129, 17), (64, 1), (333, 9), (1, 4), (257, 3), (95, 12), (512, 6), (200, 20)]
    chains, mats = [], []
    for i, (n, e) in enumerate(sizes):
        X = synth.random_matrix(n, n, 500 + i, 0, 31, 0.25)
        mats.append((X, e))
        A = mpr.to_device(X)
        chains.append((A, e, mpr.alloc_matrix(n, n), torch.empty(n, dtype=torch.int64, device="cuda")))
    return chains, mats


@pytest.mark.parametrize("cfg", list(range(12)))
def test_batch_matches_oracle_and_solo(mpr, cfg):
    print("batch cfg", cfg, flush=True)
    mpr.set_batch_config(cfg)
    try:
        chains, mats = _small_batch(mpr)
        mpr.batch_power(chains)
        for (A, e, N, R), (X, _) in zip(chains, mats):
            Nr, Rr = O.power_chain(O.from_u16(X), e)
            assert np.array_equal(N.cpu().numpy(), O.to_u16(Nr)), (X.shape, e)
            assert np.array_equal(R.cpu().numpy(), Rr)
            Ns, Rs = mpr.minplus_power(A, e, mpr.CHAIN)
            assert np.array_equal(Ns.cpu().numpy(), N.cpu().numpy()) and torch.equal(Rs, R)
    finally:
        mpr.set_batch_config(-1)


@pytest.mark.parametrize("cfg", [0, 6, 11])
def test_batch_large_entries(mpr, cfg):
    """Entries 2100..3000 (every finite product entry >= 2100, so the f16
    form recomputes every block in uint16) beside a small-entry chain."""
    print("batch large", cfg, flush=True)
    mpr.set_batch_config(cfg)
    try:
        mats, chains = [], []
        for i, (n, e) in enumerate([(150, 4), (300, 3), (77, 6)]):
            X = synth.random_matrix(n, n, 900 + i, 0 if i == 0 else 2100, 31 if i == 0 else 3000, 0.2)
            mats.append((X, e))
            chains.append((mpr.to_device(X), e, mpr.alloc_matrix(n, n), torch.empty(n, dtype=torch.int64,
                                                                                    device="cuda")))
        mpr.batch_power(chains)
        for (A, e, N, R), (X, _) in zip(chains, mats):
            Nr, Rr = O.power_chain(O.from_u16(X), e)
            assert np.array_equal(N.cpu().numpy(), O.to_u16(Nr)) and np.array_equal(R.cpu().numpy(), Rr)
    finally:
        mpr.set_batch_config(-1)


def test_batch_roman_and_banded(mpr):
    chains, refs = [], []
    for m, e in [(3, 30), (5, 20), (6, 7)]:
        A = mpr.build_transfer(m)
        n = A.shape[0]
        chains.append((A, e, mpr.alloc_matrix(n, n), torch.empty(n, dtype=torch.int64, device="cuda")))
        refs.append(O.power_chain(O.transfer(m), e))
    X = synth.banded_matrix(450, 64)
    chains.append((mpr.to_device(X), 6, mpr.alloc_matrix(450, 450), torch.empty(450, dtype=torch.int64, device="cuda")))
    refs.append(O.power_chain(O.from_u16(X), 6))
    mpr.batch_power(chains)
    for (A, e, N, R), (Nr, Rr) in zip(chains, refs):
        assert np.array_equal(N.cpu().numpy(), O.to_u16(Nr)) and np.array_equal(R.cpu().numpy(), Rr)


def test_batch_graph_replays(mpr):
    """Captured launch replayed several times with eager work in between;
    every replay must reproduce the eager result."""
    chains, mats = _small_batch(mpr)
    ws = mpr.workspace(mpr.batch_workspace_size(chains))
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    mpr.batch_plan(chains, ws)
    mpr.batch_launch(ws, st)
    torch.cuda.synchronize()
    eager = [(N.clone(), R.clone()) for (_, _, N, R) in chains]
    stream = torch.cuda.Stream()
    g = mpr.batch_graph_create(ws, st, stream)
    try:
        for rep in range(3):
            for (_, _, N, R) in chains:
                N.view(torch.int16).fill_(7)
                R.fill_(-1)
            torch.cuda.synchronize()
            mpr.graph_launch(g, stream)
            stream.synchronize()
            x = torch.randn(1000, device="cuda").sum()  # unrelated eager work
            torch.cuda.synchronize()
            for (_, _, N, R), (Ne, Re) in zip(chains, eager):
                assert np.array_equal(N.cpu().numpy(), Ne.cpu().numpy()) and torch.equal(R, Re), rep
        assert int(st.item()) == 0
        del x
    finally:
        mpr.graph_destroy(g)


@pytest.mark.parametrize("cfg", [0, 6, 9])
def test_batch_persistent_form(mpr, cfg):
    """The persistent grid (resident workgroups looping over the work list)
    against the one-workgroup-per-panel form and the oracle: 64 chains of
    N = 2048 give 2048 to 4096 panels, more than the resident workgroups,
    so persistent workgroups take several panels each; also captured in a
    graph and replayed."""
    print("persistent batch cfg", cfg, flush=True)
    mpr.set_batch_config(cfg)
    try:
        n, e, count = 2048, 3, 64
        chains, mats = [], []
        for i in range(count):
            X = synth.random_matrix(n, n, 700 + i, 0, 31, 0.25)
            mats.append(X)
            chains.append((mpr.to_device(X), e, mpr.alloc_matrix(n, n), torch.empty(n, dtype=torch.int64, device="cuda")))
        ws = mpr.workspace(mpr.batch_workspace_size(chains))
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        mpr.batch_plan(chains, ws)
        mpr.batch_launch(ws, st)
        torch.cuda.synchronize()
        per_panel = [(N.clone(), R.clone()) for (_, _, N, R) in chains]
        mpr.set_batch_persistent(True)
        mpr.batch_plan(chains, ws)
        _, grid, panels = mpr.batch_plan_info(ws)
        assert 1 <= grid < panels
        stream = torch.cuda.Stream()
        g = mpr.batch_graph_create(ws, st, stream)
        try:
            for rep in range(2):
                for (_, _, N, R) in chains:
                    N.view(torch.int16).fill_(7)
                    R.fill_(-1)
                torch.cuda.synchronize()
                mpr.graph_launch(g, stream)
                stream.synchronize()
                for (_, _, N, R), (Np, Rp) in zip(chains, per_panel):
                    assert torch.equal(N.view(torch.int16), Np.view(torch.int16)) and torch.equal(R, Rp), rep
        finally:
            mpr.graph_destroy(g)
        assert int(st.item()) == 0
        rows = [0, 1029, n - 1]
        for k in (0, count - 1):
            Nr, Rr = O.chain_rows(O.from_u16(mats[k]), rows, e)
            N, R = chains[k][2], chains[k][3]
            assert np.array_equal(N.cpu().numpy()[rows], O.to_u16(Nr)) and np.array_equal(R.cpu().numpy()[rows], Rr)
    finally:
        mpr.set_batch_persistent(False)
        mpr.set_batch_config(-1)


def test_batch_full_config4_sampled_rows(mpr):
    """The full batched workload (256 chains, N log-uniform in [256, 4096],
    e in [8, 128], entries U[0,31] with 25% infinity) in the benchmark's
    launch; rows of three chains checked against the oracle's
    row-restricted chain, every chain against its solo GPU run."""
    inst = synth.batch_instances(256, seed=4)
    chains, mats = [], []
    for d in inst:
        X = synth.random_matrix(d["n"], d["n"], d["seed"], 0, 31, 0.25)
        mats.append(X)
        chains.append((mpr.to_device(X), d["e"], mpr.alloc_matrix(d["n"], d["n"]),
                       torch.empty(d["n"], dtype=torch.int64, device="cuda")))
    print("batch generated", flush=True)
    mpr.batch_power(chains)
    torch.cuda.synchronize()
    print("batch done", flush=True)
    order = sorted(range(256), key=lambda i: -inst[i]["n"])
    picks = [order[0], order[128], order[-1]]
    for i in picks:
        A, e, N, R = chains[i]
        n = A.shape[0]
        rows = [0, n // 2, n - 1]
        Nr, Rr = O.chain_rows(O.from_u16(mats[i]), rows, e)
        assert np.array_equal(N.cpu().numpy()[rows], O.to_u16(Nr)), (n, e)
        assert np.array_equal(R.cpu().numpy()[rows], Rr)
    ws = mpr.workspace(max(mpr.power_workspace_size(d["n"], d["e"]) for d in inst))
    for (A, e, N, R) in chains[::8]:
        Ns, Rs = mpr.minplus_power(A, e, mpr.CHAIN, ws=ws)
        assert torch.equal(Ns.view(torch.int16), N.view(torch.int16)) and torch.equal(Rs, R)


@pytest.mark.parametrize("arith", ["u16", "f16"])
def test_batch_weights_route_the_plan(mpr, arith):
    """An installed weight table (the form the batch autotuner persists)
    steers the library's configuration model: with one configuration of the
    process-wide arithmetic weighted far above the others the plan takes
    it, and its results equal the oracle's."""
    chains, mats = _small_batch(mpr)
    cnt = mpr.batch_config_count()
    prior = mpr.get_batch_weights()
    mine = [c for c in range(cnt) if mpr.batch_config_info(c)["arith"] == arith]
    ws = mpr.workspace(mpr.batch_workspace_size(chains))
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    try:
        with mpr.arith_scope(arith):
            for target in (mine[0], mine[2], mine[-1]):
                print("batch weights", arith, target, flush=True)
                w = [1e-3] * cnt
                w[target] = 1.0
                mpr.set_batch_weights(w)
                mpr.batch_plan(chains, ws)
                assert mpr.batch_plan_info(ws)[0] == target
                for (_, _, N, R) in chains:
                    N.view(torch.int16).fill_(7)
                mpr.batch_launch(ws, st)
                torch.cuda.synchronize()
                assert int(st.item()) == 0
                for (A, e, N, R), (X, _) in zip(chains, mats):
                    Nr, Rr = O.power_chain(O.from_u16(X), e)
                    assert np.array_equal(N.cpu().numpy(), O.to_u16(Nr)) and np.array_equal(R.cpu().numpy(), Rr)
    finally:
        mpr.set_batch_weights(prior)


def test_batch_autotuner_persists_and_installs(mpr, tmp_path):
    """The batch autotuner times every batched configuration, persists the
    relative throughputs (fastest = 1) and load_batch_table installs them;
    the plan then follows the model with those weights."""
    from paper_2409_17658_amd import autotune

    prior = mpr.get_batch_weights()
    p = tmp_path / "batch.json"
    try:
        out = autotune.tune_batch(chains=16, n=256, e=3, reps=1, path=str(p))
        w = out["weights"]
        assert len(w) == mpr.batch_config_count() and max(w) == 1.0 and min(w) > 0
        mpr.set_batch_weights(None)
        assert autotune.load_batch_table(str(p))
        assert mpr.get_batch_weights() == pytest.approx(w)
        bad = dict(out, configs=out["configs"][:-1])
        p.write_text(__import__("json").dumps(bad))
        assert not autotune.load_batch_table(str(p))
    finally:
        mpr.set_batch_weights(prior)
