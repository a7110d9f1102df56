"""Roman transfer matrices for m = 6, 7, 8 (the paper's new cases): powers
to n = 300 by the chain and by binary powering, the least period, and
gamma_R for n = 3..300, against the stored oracle goldens (bit-exact
canonical-form digests at selected k)."""
import hashlib
import json
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(m):
    with open(os.path.join(HERE, "roman_m%d.json" % m)) as f:
        return json.load(f)


@pytest.fixture(scope="module")
def mpr():
    import paper_2409_17658_amd as m

    m.lib()
    m.init(0)
    return m


def digest(N, R):
    n = N.shape[0]
    h = np.ascontiguousarray(N.cpu().numpy()[:, :n]).astype("<u2").tobytes()
    return hashlib.sha256(h + np.ascontiguousarray(R.cpu().numpy(), dtype="<i8").tobytes()).hexdigest()


@pytest.mark.parametrize("m", [6, 7, 8])
def test_period_and_gamma_to_300(mpr, m):
    print("roman m", m, flush=True)
    g = load(m)
    A = mpr.build_transfer(m)
    mu, lam, c, tr = mpr.find_period(A, 300, traces=True, slots=40)
    assert [mu, lam, c] == g["period"]
    for k in range(1, 301):
        assert tr[k] == g["trace"][str(k)], k


@pytest.mark.parametrize("arith", ["u16", "f16"])
@pytest.mark.parametrize("m", [6, 7, 8])
def test_chain_and_squaring_digests(mpr, m, arith):
    """Both arithmetic forms (the packed uint16 default and the f16 form)
    give the oracle's canonical powers bit for bit."""
    g = load(m)
    A = mpr.build_transfer(m)
    with mpr.arith_scope(arith):
        for k in (1, 2, 3, 21, 26, 64, 128, 299, 300):
            for sched in (mpr.CHAIN, mpr.SQUARE):
                if sched == mpr.CHAIN and k not in (1, 3, 26, 300):
                    continue
                N, R = mpr.minplus_power(A, k, sched)
                assert digest(N, R) == g["digest_sha256"][str(k)], (k, sched)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 7])
def test_border_transfer_bit_exact(mpr, m):
    import oracle as O

    A, shift = mpr.build_border_transfer(m)
    ref = O.border_transfer(m)
    got = A.cpu().numpy().astype(np.int64)
    fin = ref != O.INF
    assert np.array_equal(got == 0xFFFF, ~fin)
    assert np.array_equal(got[fin] - shift, ref[fin])


def test_border_m4_period_and_loss(mpr, paper_values):
    """Appendix: Algorithm 2 on the border matrix, m = 4: (30, 1, 1); the
    traces minus n * shift are 2 L_a(n) = n for 10 <= n <= 300 except
    2 L_a(11) = 12 (as the oracle and its column DP give)."""
    A, shift = mpr.build_border_transfer(4)
    mu, lam, c, tr = mpr.find_period(A, 300, traces=True, slots=40)
    assert (mu, lam, c - lam * shift) == tuple(paper_values["loss_border_m4"]["period"])
    for n in range(10, 301):
        assert tr[n] - n * shift == (12 if n == 11 else n), n


@pytest.mark.parametrize("form", ["tiles", "entries"])
@pytest.mark.parametrize("m", [1, 3, 5, 6, 7, 8])
def test_sparse_chain_digests(mpr, m, form):
    """The compressed-K chain (only rows of A reaching each column block)
    gives the same canonical powers, bit for bit, as the oracle goldens, in
    both forms of its step (dense rows of A per block, or A's finite
    entries only)."""
    print("sparse chain", m, form, flush=True)
    g = load(m)
    A = mpr.build_transfer(m)
    mpr.set_sparse_form(form)
    try:
        for k in (1, 2, 3, 26, 64, 300):
            N, R = mpr.minplus_power(A, k, mpr.CHAIN_SPARSE)
            assert digest(N, R) == g["digest_sha256"][str(k)], k
    finally:
        mpr.set_sparse_form("auto")


def test_sparse_period_matches(mpr):
    for m in (6, 7, 8):
        g = load(m)
        A = mpr.build_transfer(m)
        mu, lam, c, tr = mpr.find_period(A, 300, traces=True, slots=8, sparse=True)
        assert [mu, lam, c] == g["period"]
        assert all(tr[k] == g["trace"][str(k)] for k in range(1, 301))


@pytest.mark.parametrize("arith,form", [("f16", "tiles"), ("u16", "tiles"), ("u16", "entries")])
def test_sparse_chain_random_and_edge_blocks(mpr, arith, form):
    """Both arithmetic forms of the compressed-K step and both forms of the
    uint16 step (dense rows of A per block, or its finite entries only);
    the cases with entries up to 3000 and 0x3FFF are large enough that the
    f16 form recomputes blocks (their normalised powers stay <= 0x7FFF, so
    no step overflows).  Sizes cover partial row blocks of 256 and of 64, a
    single short block, and a nearly dense last case."""
    import oracle as O
    import synth

    mpr.set_sparse_arith(arith)
    mpr.set_sparse_form(form)
    try:
        for n, frac, e, hi in [(700, 0.95, 6, 40), (333, 0.99, 9, 40), (129, 0.5, 5, 40), (64, 0.9, 4, 40),
                               (300, 0.9, 4, 3000), (200, 0.97, 2, 0x3FFF), (37, 0.8, 3, 40), (530, 0.1, 3, 60)]:
            print("sparse random", arith, form, n, flush=True)
            X = synth.random_matrix(n, n, 77 + n, 0, hi, frac)
            X[:, 64:128] = 0xFFFF  # an empty column block
            N, R = mpr.minplus_power(mpr.to_device(X), e, mpr.CHAIN_SPARSE)
            Nr, Rr = O.power_chain(O.from_u16(X), e)
            assert np.array_equal(N.cpu().numpy(), O.to_u16(Nr)) and np.array_equal(R.cpu().numpy(), Rr), n
    finally:
        mpr.set_sparse_arith("u16")
        mpr.set_sparse_form("auto")


def test_sparse_chain_u16_digests(mpr):
    mpr.set_sparse_arith("u16")
    try:
        g = load(7)
        A = mpr.build_transfer(7)
        for k in (2, 26, 300):
            N, R = mpr.minplus_power(A, k, mpr.CHAIN_SPARSE)
            assert digest(N, R) == g["digest_sha256"][str(k)], k
    finally:
        mpr.set_sparse_arith("u16")


def test_sparse_plan_sized_for_the_matrix(mpr):
    """The compressed-K plan sized for the transfer matrix (a few per cent
    of the dense worst case) gives the same powers; a plan share too small
    for it is reported on the device (MPR_ENOMEM, nothing computed), and
    refused on the host when no status word could report it."""
    import torch

    g = load(7)
    A = mpr.build_transfer(7)
    n = A.shape[0]
    exact = mpr.sparse_plan_bytes(A)
    worst = mpr.power_workspace_size(n, 26, mpr.CHAIN_SPARSE) - mpr.power_workspace_size(n, 26, mpr.CHAIN)
    assert exact * 4 < worst  # m = 7: 2.4 MB against 13.3 MB (m = 10: about 30x)
    base = mpr.power_workspace_size(n, 26, mpr.CHAIN) + 256
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    N, R = mpr.minplus_power(A, 26, mpr.CHAIN_SPARSE, ws=mpr.workspace(base + exact), d_status=st, check=False)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and digest(N, R) == g["digest_sha256"]["26"]
    small = mpr.workspace(base + exact - 4096)
    mpr.minplus_power(A, 26, mpr.CHAIN_SPARSE, N, R, ws=small, d_status=st, check=False)
    torch.cuda.synchronize()
    assert int(st.item()) == 2  # MPR_ENOMEM
    with pytest.raises(mpr.MprError) as e:
        mpr.minplus_power(A, 26, mpr.CHAIN_SPARSE, N, R, ws=small, check=False)
    assert e.value.status == 1  # no status word: refused before any launch


@pytest.mark.parametrize("form", ["auto", "entries"])
@pytest.mark.parametrize("m", [4, 6, 7])
def test_period_with_a_reused_buffer(mpr, m, form):
    """A ring of two powers plus A's own buffer (for matrices too large for
    a longer ring): a period the ring can not confirm (lam >= 2) is
    confirmed exactly one period after the class repeat, so mu comes out
    lam above the least pre-period; lam, c and every trace equal the
    goldens (m = 4 has lam = 1, confirmed in the ring).  Both forms of the
    compressed-K step (these sizes take the tile form by default)."""
    print("reuse_a", m, form, flush=True)
    g = load(m)
    mu0, lam0, c0 = g["period"]
    A = mpr.build_transfer(m)
    mpr.set_sparse_form(form)
    try:
        mu, lam, c, tr = mpr.find_period(A, 300, traces=True, slots=2, sparse=True, extend=True, reuse_a=True)
    finally:
        mpr.set_sparse_form("auto")
    assert (mu, lam, c) == ((mu0 if lam0 < 2 else mu0 + lam0), lam0, c0)
    for k in range(1, 301):
        assert tr[k] == g["trace"][str(k)], k
    with pytest.raises(mpr.MprError):  # needs the compressed-K steps (A is read by dense ones)
        mpr.find_period(mpr.build_transfer(m), 40, slots=2, reuse_a=True)
