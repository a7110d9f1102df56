"""The allocation-free power entry point (mpr_minplus_power_noalloc, for
callers that cannot allocate device memory) against the workspace entry
point it shares its kernels with, and against the oracle: two calls in a row
per schedule, the second on a smaller input (the fixed scratch keeps the
first call's contents), and the size limit refused before any launch."""
import ctypes

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


def _call_noalloc(mpr, A, e, schedule, N, R, st):
    """Straight through the C ABI (no Python-side buffers)."""
    L = mpr.lib()
    n = A.shape[0]
    return L.mpr_minplus_power_noalloc(ctypes.c_void_p(A.data_ptr()), n, mpr._ld(A), e, schedule,
                                       ctypes.c_void_p(N.data_ptr()), mpr._ld(N), ctypes.c_void_p(R.data_ptr()),
                                       ctypes.c_void_p(st.data_ptr()), mpr._stream(None))


@pytest.mark.parametrize("schedule", [0, 1, 2])
def test_noalloc_matches_workspace_path_twice(mpr, schedule):
    cases = [(1100, 7, 31, 0.25), (333, 5, 200, 0.4)]  # second call smaller
    for n, e, hi, frac in cases:
        print("noalloc schedule", schedule, "n", n, "e", e, flush=True)
        X = synth.random_matrix(n, n, 1300 + n + schedule, 0, hi, frac)
        A = mpr.to_device(X)
        N = mpr.alloc_matrix(n, n)
        R = torch.empty(n, dtype=torch.int64, device="cuda")
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        assert _call_noalloc(mpr, A, e, schedule, N, R, st) == 0
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        Nw, Rw = mpr.minplus_power(A, e, schedule)
        assert torch.equal(N.view(torch.int16), Nw.view(torch.int16)) and torch.equal(R, Rw), (n, schedule)
        if n <= 400:
            Nr, Rr = O.power_chain(O.from_u16(X), e)
            assert np.array_equal(N.cpu().numpy(), O.to_u16(Nr)) and np.array_equal(R.cpu().numpy(), Rr)
        else:
            rows = [0, 511, n - 1]
            Nr, Rr = O.chain_rows(O.from_u16(X), rows, e)
            assert np.array_equal(N.cpu().numpy()[rows], O.to_u16(Nr)) and np.array_equal(R.cpu().numpy()[rows], Rr)


def test_noalloc_roman_and_limits(mpr):
    """m = 7 (2507 states) by the chain fits the scratch; a chain on
    n = 5793 does not and is refused with MPR_ENOMEM, outputs untouched."""
    A = mpr.build_transfer(7)
    n = A.shape[0]
    N = mpr.alloc_matrix(n, n)
    R = torch.empty(n, dtype=torch.int64, device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert _call_noalloc(mpr, A, 26, 0, N, R, st) == 0
    Nw, Rw = mpr.minplus_power(A, 26, 0)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert torch.equal(N.view(torch.int16), Nw.view(torch.int16)) and torch.equal(R, Rw)
    big = 5793
    Ab = mpr.alloc_matrix(big, big, fill=0)
    Nb = mpr.alloc_matrix(big, big, fill=7)
    Rb = torch.full((big,), -5, dtype=torch.int64, device="cuda")
    assert _call_noalloc(mpr, Ab, 3, 0, Nb, Rb, st) == 2  # MPR_ENOMEM
    torch.cuda.synchronize()
    assert int((Nb.view(torch.int16) != 7).sum().item()) == 0 and int((Rb != -5).sum().item()) == 0
    assert mpr.power_workspace_size(5792, 3, 0) <= mpr.NOALLOC_SCRATCH_BYTES < mpr.power_workspace_size(big, 3, 0)
