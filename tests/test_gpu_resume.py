"""Checkpoint and resume of a chain.  Row i of A^(k+1) = A^k (x) A needs
row i of A^k and A only (Algorithm 2's chain in canonical form), so the
whole state of a chain is (N_k, R_k, k): a chain stopped at k, saved to a
file, reloaded and resumed for the remaining steps gives the same bits as
the chain run in one go (mpr_minplus_power), and its rows equal the
oracle's row chain."""
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


@pytest.mark.parametrize("schedule", ["CHAIN", "CHAIN_SPARSE"])
def test_resume_from_checkpoint_equals_one_chain(mpr, tmp_path, schedule):
    sched = getattr(mpr, schedule)
    m, k0, e = 7, 17, 40
    print("resume", schedule, flush=True)
    A = mpr.build_transfer(m)
    n = A.shape[0]
    Ne, Re = mpr.minplus_power(A, e, sched)
    Nk, Rk = mpr.minplus_power(A, k0, sched)
    path = tmp_path / "chain_k17.npz"
    mpr.save_power(path, Nk, Rk, k0)
    del Nk, Rk
    Nk, Rk, k = mpr.load_power(path)
    assert k == k0
    N, R = mpr.chain_resume(A, Nk, Rk, e - k, sched)
    assert torch.equal(N, Ne) and torch.equal(R, Re)
    # in place, in two legs
    mpr.chain_resume(A, Nk, Rk, 10, sched, N_out=Nk, R_out=Rk)
    mpr.chain_resume(A, Nk, Rk, e - k - 10, sched, N_out=Nk, R_out=Rk)
    assert torch.equal(Nk, Ne) and torch.equal(Rk, Re)
    # zero steps: a copy
    N0, R0 = mpr.chain_resume(A, Ne, Re, 0, sched)
    assert torch.equal(N0, Ne) and torch.equal(R0, Re)
    rows = [0, 1, 999, n - 1]
    want = {}
    O.chain_rows_sparse(O.transfer_rows(m, rows), O.transfer_arcs(m), e,
                        on_step=lambda j, Nj, Rj: want.__setitem__(j, (O.to_u16(Nj), Rj.copy())) if j == e else None)
    assert np.array_equal(mpr.to_host(N)[rows], want[e][0])
    assert np.array_equal(R.cpu().numpy()[rows], want[e][1])


def test_resume_banded_matches_oracle(mpr):
    """A banded matrix (values keep spreading, nothing collapses): resuming
    at k = 5 for 6 steps gives A^11, equal to the oracle's chain."""
    Ah = synth.banded_matrix(300, 16)
    A = mpr.to_device(Ah)
    N5, R5 = mpr.minplus_power(A, 5, mpr.CHAIN)
    N, R = mpr.chain_resume(A, N5, R5, 6, mpr.CHAIN)
    Nr, Rr = O.power_chain(O.from_u16(Ah), 11)
    assert np.array_equal(mpr.to_host(N), O.to_u16(Nr))
    assert np.array_equal(R.cpu().numpy(), Rr)
