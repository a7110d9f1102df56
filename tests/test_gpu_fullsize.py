"""Full-size parity (the benchmark's sizes, in its launch configuration):
whole rows of the N = 16384 product, including the tile seams, in both
arithmetic forms; and a full-size chain whose normalised entries cross
2048 in some blocks (so the f16 form's uint16 recomputation runs at the
benchmark tile's full size), checked row by row against the oracle's
row-restricted chain.  Tolerance 0 throughout."""
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


def _rows(t, rows):
    """Rows of a device uint16 matrix as a host array (indexing through an
    int16 view: torch does not index uint16 device tensors)."""
    idx = torch.as_tensor(np.asarray(rows), device=t.device)
    return t.view(torch.int16)[idx].cpu().numpy().view(np.uint16)


SEAM_ROWS = [0, 1, 63, 64, 127, 128, 255, 256, 511, 512, 8191, 8192, 16255, 16256, 16383]


def test_gemm_n16384_full_rows_both_forms(mpr):
    n = 16384
    X = synth.random_matrix(n, n, 1, 0, 15, 0.30)
    Y = synth.random_matrix(n, n, 2, 0, 15, 0.30)
    rng = np.random.default_rng(7)
    rows = np.unique(np.concatenate([SEAM_ROWS, rng.integers(0, n, 260)]))[:272]
    assert len(rows) >= 256
    ref = O.to_u16(O.minplus(O.from_u16(X)[rows], O.from_u16(Y)))
    A, B = mpr.to_device(X), mpr.to_device(Y)
    C = mpr.alloc_matrix(n, n)
    for arith in ("u16", "f16"):
        with mpr.arith_scope(arith):
            cfg = mpr.gemm_pick_config(n, n, n)
            print("n16384 rows", arith, "cfg", cfg, flush=True)
            C.view(torch.int16).fill_(7)
            mpr.minplus_gemm(A, B, C, check=True)
            got = _rows(C, rows)
            assert np.array_equal(got, ref), arith


@pytest.mark.parametrize("arith", ["u16", "f16"])
def test_banded_chain_n8192_crosses_2048(mpr, arith):
    """A^40 of the banded family at N = 8192: the band widens by 64 per
    step, so far-off-diagonal normalised entries pass 2048 while entries
    near the diagonal stay small, and the product's tiles are mixed."""
    n, e = 8192, 40
    X = synth.banded_matrix(n, 64)
    rng = np.random.default_rng(11)
    rows = np.unique(np.concatenate([[0, 1, 127, 128, 4095, 4096, 8190, 8191], rng.integers(0, n, 8)]))
    Nr, Rr = O.chain_rows(O.from_u16(X), rows, e)
    fin = Nr[Nr != O.INF]
    assert fin.max() >= 2048 and (fin < 2048).any()  # both sides of the f16 form's exact range
    with mpr.arith_scope(arith):
        print("banded chain", arith, "cfg", mpr.gemm_pick_config(n, n, n), flush=True)
        N, R = mpr.minplus_power(mpr.to_device(X), e, mpr.CHAIN, check=True)
    assert np.array_equal(_rows(N, rows), O.to_u16(Nr))
    assert np.array_equal(R.cpu().numpy()[rows], Rr)
