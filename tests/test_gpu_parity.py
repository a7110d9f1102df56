"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every comparison is exact (integers; tolerance 0).  Inputs come from the
seeded generators in `synth`, the same bytes for both sides.
"""
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


def _u16(a):
    return O.to_u16(a)


def _dev(mpr, a):
    return mpr.to_device(a)


def _host(t):
    return t.cpu().numpy()


# ------------------------------------------------------------------ products
SHAPES = [(1, 1, 1), (7, 9, 5), (31, 33, 17), (64, 64, 64), (127, 129, 255), (300, 257, 511), (513, 200, 130)]


@pytest.mark.parametrize("shape", SHAPES)
def test_gemm_random_all_configs(mpr, shape):
    M, N, K = shape
    print("gemm", shape, flush=True)
    X = synth.random_matrix(M, K, 101, 0, 15, 0.30)
    Y = synth.random_matrix(K, N, 102, 0, 15, 0.30)
    ref = _u16(O.minplus(O.from_u16(X), O.from_u16(Y)))
    A, B = _dev(mpr, X), _dev(mpr, Y)
    for cfg in range(mpr.gemm_config_count()):
        C = mpr.minplus_gemm(A, B, cfg=cfg)
        assert np.array_equal(_host(C), ref), cfg


@pytest.mark.parametrize("law", [(0, 15, 0.30), (1024, 1039, 0.30)])
def test_gemm_spare_grid_form_all_configs(mpr, law):
    """The launch that leaves a workgroup slot per CU free
    (mpr_minplus_gemm_spare: extra LDS per workgroup; configurations of
    fewer than 3 workgroups per CU run as the 128 x 128 tile) at a ragged
    size with more tiles than the device holds at once, for every
    configuration: the whole product equals the plain launch bit for bit,
    and sampled rows (tile seams, the last row) equal the oracle's.  The
    second entry law sends every tile of the f16 configurations through
    their uint16 recomputation."""
    M, N, K = 4001, 4103, 999
    lo, hi, inf = law
    print("gemm spare", law, flush=True)
    X = synth.random_matrix(M, K, 111 + lo, lo, hi, inf)
    Y = synth.random_matrix(K, N, 112 + lo, lo, hi, inf)
    rows = [0, 1, 63, 64, 127, 128, 255, 256, 1999, 2048, M - 2, M - 1]
    ref = _u16(O.minplus(O.from_u16(X[rows]), O.from_u16(Y)))
    A, B = _dev(mpr, X), _dev(mpr, Y)
    for cfg in range(mpr.gemm_config_count()):
        C0 = mpr.minplus_gemm(A, B, cfg=cfg)
        C1 = mpr.minplus_gemm(A, B, cfg=cfg, spare=True)
        assert torch.equal(C0, C1), cfg
        assert np.array_equal(_host(C1)[rows], ref), cfg


def test_gemm_spare_small(mpr):
    """A small product in the same launch form, same bits as the oracle."""
    X = synth.random_matrix(130, 77, 121, 0, 15, 0.3)
    Y = synth.random_matrix(77, 201, 122, 0, 15, 0.3)
    ref = _u16(O.minplus(O.from_u16(X), O.from_u16(Y)))
    A, B = _dev(mpr, X), _dev(mpr, Y)
    for cfg in range(mpr.gemm_config_count()):
        assert np.array_equal(_host(mpr.minplus_gemm(A, B, cfg=cfg, spare=True)), ref), cfg


def test_gemm_unaligned_leading_dimensions(mpr):
    """Row strides that are not multiples of 8 take the element-wise path."""
    M, N, K = 45, 37, 29
    X = synth.random_matrix(M, K, 7, 0, 15, 0.3)
    Y = synth.random_matrix(K, N, 8, 0, 15, 0.3)
    ref = _u16(O.minplus(O.from_u16(X), O.from_u16(Y)))
    Ap = np.full((M, K + 2), 0xFFFF, dtype=np.uint16)  # row stride 31
    Ap[:, :K] = X
    Bp = np.pad(Y, ((0, 0), (0, 5)))  # row stride 42
    A = torch.from_numpy(Ap).cuda()[:, :K]
    B = torch.from_numpy(Bp).cuda()[:, :N]
    assert A.stride(0) % 8 and B.stride(0) % 8
    Cbuf = torch.zeros((M, N + 1), dtype=torch.uint16, device="cuda")  # row stride 38
    for cfg in range(mpr.gemm_config_count()):
        mpr.minplus_gemm(A, B, C=Cbuf[:, :N], cfg=cfg)
        assert np.array_equal(_host(Cbuf[:, :N]), ref), cfg


def test_gemm_extremes(mpr):
    """All-infinite rows/columns, entries at the 0x7FFF bound, empty K."""
    n = 70
    X = synth.random_matrix(n, n, 3, 0, 0x7FFF, 0.3)
    Y = synth.random_matrix(n, n, 4, 0x7000, 0x7FFF, 0.2)
    X[:, 0] = 0x7FFF
    X[5, :] = 0xFFFF
    Y[:, 9] = 0xFFFF
    ref = _u16(O.minplus(O.from_u16(X), O.from_u16(Y)))
    C = mpr.minplus_gemm(_dev(mpr, X), _dev(mpr, Y))
    got = _host(C)
    assert np.array_equal(got, ref)
    assert np.all(got[5] == 0xFFFF) and np.all(got[:, 9] == 0xFFFF)
    # empty inner dimension: every entry infinite
    A0 = mpr.alloc_matrix(4, 0)
    B0 = mpr.alloc_matrix(0, 6)
    C0 = mpr.minplus_gemm(A0, B0)
    assert np.all(_host(C0) == 0xFFFF)


def _all_cfg_equal(mpr, X, Y, what):
    ref = _u16(O.minplus(O.from_u16(X), O.from_u16(Y)))
    A, B = _dev(mpr, X), _dev(mpr, Y)
    for cfg in range(mpr.gemm_config_count()):
        C = mpr.minplus_gemm(A, B, cfg=cfg)
        assert np.array_equal(_host(C), ref), (what, cfg, mpr.gemm_config_info(cfg))
    return ref


def test_gemm_f16_form_boundaries(mpr):
    """Cases aimed at the f16 form of the product configurations: sums on
    both sides of 2048 (exact below, recomputed in uint16 from there), the
    clamp of finite values >= 0x800, finite values 0x7C00..0x7FFF (f16
    infinity / NaN patterns), and sums up to 0xFFFE that must stay finite."""
    print("f16 boundaries", flush=True)
    M, N, K = 200, 190, 5
    rng = np.random.default_rng(11)
    # around 2048: entries 1000..1050, sums 2000..2100, minima of few terms
    X = rng.integers(1000, 1051, (M, K)).astype(np.uint16)
    Y = rng.integers(1000, 1051, (K, N)).astype(np.uint16)
    X[rng.random((M, K)) < 0.3] = 0xFFFF
    ref = _all_cfg_equal(mpr, X, Y, "around 2048")
    assert (ref < 2048).any() and ((ref >= 2048) & (ref != 0xFFFF)).any()
    # exact 2047 / 2048 minima
    X = np.full((70, 40), 0xFFFF, np.uint16)
    Y = np.full((40, 66), 0xFFFF, np.uint16)
    X[:, 3] = 1023
    Y[3, :] = 1024          # 2047 everywhere ...
    Y[3, ::2] = 1025        # ... or 2048 in even columns
    ref = _all_cfg_equal(mpr, X, Y, "2047/2048")
    assert (ref[:, 1::2] == 2047).all() and (ref[:, ::2] == 2048).all()
    # f16 infinity / NaN bit patterns as finite values, sums up to 0xFFFE
    X = rng.integers(0x7C00, 0x8000, (90, 70)).astype(np.uint16)
    Y = rng.integers(0x7C00, 0x8000, (70, 80)).astype(np.uint16)
    X[rng.random(X.shape) < 0.4] = 0xFFFF
    Y[:, 5] = 0xFFFF
    X[0, :] = 0x7FFF
    Y[:, 0] = 0x7FFF
    ref = _all_cfg_equal(mpr, X, Y, "0x7C00..0x7FFF")
    assert ref[0, 0] == 0xFFFE and (ref[:, 5] == 0xFFFF).all()


def test_gemm_f16_form_mixed_blocks(mpr):
    """Small entries except for a band of rows of A and a band of columns of
    B with large ones: only the blocks that meet the bands hold minima
    >= 2048, so some blocks keep their f16 results and others recompute."""
    print("f16 mixed blocks", flush=True)
    M, N, K = 700, 650, 333
    X = synth.random_matrix(M, K, 21, 0, 15, 0.3)
    Y = synth.random_matrix(K, N, 22, 0, 15, 0.3)
    X[300:340, :] = synth.random_matrix(40, K, 23, 3000, 9000, 0.2)
    Y[:, 500:520] = synth.random_matrix(K, 20, 24, 0x7800, 0x7FFF, 0.2)
    ref = _all_cfg_equal(mpr, X, Y, "mixed")
    assert (ref[300:340] >= 2048).all() and (ref[:300, :500] < 64).all()


def test_gemm_overflow_is_reported(mpr):
    X = synth.random_matrix(40, 40, 5, 0, 15, 0.3)
    X[3, 4] = 0x8000
    A = _dev(mpr, X)
    with pytest.raises(mpr.MprError) as e:
        mpr.minplus_gemm(A, A)
    assert e.value.status == 3


def test_gemm_full_size_sampled(mpr):
    """N = 16384 (the benchmark size) in the benchmark's launch: sampled
    entries, each recomputed by the oracle from the definition."""
    n = 16384
    X = synth.random_matrix(n, n, 1, 0, 15, 0.30)
    Y = synth.random_matrix(n, n, 2, 0, 15, 0.30)
    C = mpr.minplus_gemm(_dev(mpr, X), _dev(mpr, Y), check=False)
    rng = np.random.default_rng(0)
    ii = np.concatenate([rng.integers(0, n, 1500), [0, n - 1, n - 1, 0]])
    jj = np.concatenate([rng.integers(0, n, 1500), [0, n - 1, 0, n - 1]])
    got = _host(C)[ii, jj]
    ref = _u16(O.minplus_at(O.from_u16(X), O.from_u16(Y), ii, jj))
    assert np.array_equal(got, ref)


# ------------------------------------------------------------------ normalisation / offsets
def test_autotune_and_tile_table(mpr):
    """mpr_autotune_gemm times every configuration and names the fastest;
    a table installed from it routes products to that configuration, whose
    results still equal the oracle's; the installed table is then restored."""
    n = 200
    best, ms = mpr.autotune_gemm(n, reps=2)
    assert len(ms) == mpr.gemm_config_count() and 0 <= best < len(ms)
    assert all(t > 0 for t in ms) and ms[best] == min(ms)
    prev = [mpr.gemm_pick_config(k, k, k) for k in (100, 300, 5000)]
    X = synth.random_matrix(n, n, 61, 0, 40, 0.3)
    Y = synth.random_matrix(n, n, 62, 0, 40, 0.3)
    ref = _u16(O.minplus(O.from_u16(X), O.from_u16(Y)))
    try:
        for arith in ("u16", "f16"):
            mine = [c for c in range(len(ms)) if mpr.gemm_config_info(c)["arith"] == arith]
            fast = min(mine, key=lambda c: ms[c])
            other = mine[(mine.index(fast) + 1) % len(mine)]
            mpr.set_tile_table([(250, fast), (1 << 40, other)])
            with mpr.arith_scope(arith):
                assert mpr.gemm_pick_config(n, n, n) == fast
                assert mpr.gemm_pick_config(300, 300, 300) == other
                C = mpr.minplus_gemm(_dev(mpr, X), _dev(mpr, Y))
                assert np.array_equal(_host(C), ref), arith
    finally:
        mpr.init(0)  # reinstalls the persisted tables
    assert [mpr.gemm_pick_config(k, k, k) for k in (100, 300, 5000)] == prev


def test_normalise_matches_oracle(mpr):
    X = synth.random_matrix(123, 301, 9, 3, 40, 0.3)
    X[7, :] = 0xFFFF
    C = _dev(mpr, X)
    Rin = torch.arange(123, dtype=torch.int64, device="cuda") * 5
    Rin[11] = mpr.ROW_NONE
    X[11, :] = 0xFFFF
    C = _dev(mpr, X)
    Rout = mpr.normalise(C, Rin)
    N, r = O.normalise(O.from_u16(X))
    assert np.array_equal(_host(C), _u16(N))
    R = O.add_offsets(Rin.cpu().numpy(), r)
    assert np.array_equal(Rout.cpu().numpy(), R)


@pytest.mark.parametrize("rows,cols,pad", [(5, 16384, 0), (3, 24583, 0), (2, 30001, 7), (4, 1000, 1), (3, 7, 0)])
def test_normalise_row_lengths(mpr, rows, cols, pad):
    """Register-resident rows (<= 24576 entries), two-pass rows, odd strides."""
    X = synth.random_matrix(rows, cols, 31 + cols, 2, 700, 0.3)
    X[0, :] = 0xFFFF
    buf = np.full((rows, cols + pad), 0xFFFF, dtype=np.uint16)
    buf[:, :cols] = X
    C = torch.from_numpy(buf).cuda()[:, :cols] if pad else _dev(mpr, X)
    Rout = mpr.normalise(C)
    N, r = O.normalise(O.from_u16(X))
    assert np.array_equal(_host(C), _u16(N)) and np.array_equal(Rout.cpu().numpy(), r)


def test_gemm_norm_product_of_powers(mpr):
    A = O.transfer(4)
    Pa = O.power_chain(A, 5)
    Pb = O.power_chain(A, 7)
    Nc, Rc = O.product_of_powers(*Pa, *Pb)
    C, R = mpr.minplus_gemm_norm(_dev(mpr, _u16(Pa[0])), _dev(mpr, _u16(Pb[0])),
                                 torch.from_numpy(Pa[1]).cuda(), torch.from_numpy(Pb[1]).cuda())
    assert np.array_equal(_host(C), _u16(Nc)) and np.array_equal(R.cpu().numpy(), Rc)


# ------------------------------------------------------------------ transfer matrix
@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6, 7, 8])
def test_build_transfer_bit_exact(mpr, m):
    A = mpr.build_transfer(m)
    assert np.array_equal(_host(A), _u16(O.transfer(m)))


def test_build_transfer_m9_sampled_rows(mpr):
    A = mpr.build_transfer(9)
    rows = [0, 1, 777, 12345, 21908]
    assert np.array_equal(_host(A)[rows], _u16(O.transfer_rows(9, rows)))


@pytest.mark.parametrize("m", [10, 11])
def test_build_transfer_largest_sampled_rows(mpr, m):
    """The largest builds the API accepts (C_10 = 64769, C_11 = 191476
    states: a 73 GB matrix at m = 11): sampled rows, including the first and
    the last, against the oracle's row-restricted builder."""
    print("transfer m", m, flush=True)
    n = mpr.transfer_size(m)
    A = mpr.build_transfer(m)
    rows = [0, 1, n // 3, n // 2 + 7, n - 2, n - 1]
    got = np.stack([A[r].cpu().numpy() for r in rows])
    del A
    torch.cuda.empty_cache()
    assert np.array_equal(got, _u16(O.transfer_rows(m, rows)))


# ------------------------------------------------------------------ powers
@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("m,e", [(3, 1), (3, 2), (3, 17), (4, 23), (5, 12), (6, 9)])
def test_power_transfer(mpr, m, e, schedule):
    A = mpr.build_transfer(m)
    N, R = mpr.minplus_power(A, e, schedule)
    Nr, Rr = O.power_chain(O.transfer(m), e)
    assert np.array_equal(_host(N), _u16(Nr)) and np.array_equal(R.cpu().numpy(), Rr)


@pytest.mark.parametrize("schedule", [0, 1])
def test_power_random_and_banded(mpr, schedule):
    for X, e in [(synth.random_matrix(257, 257, 11, 0, 31, 0.25), 9), (synth.banded_matrix(600, 64), 8)]:
        N, R = mpr.minplus_power(_dev(mpr, X), e, schedule)
        Nr, Rr = O.power_chain(O.from_u16(X), e)
        assert np.array_equal(_host(N), _u16(Nr)) and np.array_equal(R.cpu().numpy(), Rr)


@pytest.mark.parametrize("arith", ["u16", "f16"])
def test_power_split_k_steps(mpr, arith):
    """Chains of matrices too small to fill the device split each step's k
    into ranges (a minimum over k taken in parts, then the minimum of the
    parts): n = 300 (2 ranges, the last 140 deep), 520 and 848 (several
    ranges, ragged tails), 200 (k too short to split).  Every power equals
    the oracle's chain, and equals the unsplit chain that a workspace of
    only the layout's size gives."""
    prev = mpr.get_arith()
    mpr.set_arith(arith)
    try:
        for n, e, seed in [(300, 6, 21), (520, 5, 22), (848, 4, 23), (200, 5, 24)]:
            print("split-k", arith, n, e, flush=True)
            X = synth.random_matrix(n, n, seed, 0, 40, 0.35)
            A = _dev(mpr, X)
            N, R = mpr.minplus_power(A, e, 0)
            Nr, Rr = O.power_chain(O.from_u16(X), e)
            assert np.array_equal(_host(N), _u16(Nr)) and np.array_equal(R.cpu().numpy(), Rr)
            ld = (n + 7) // 8 * 8
            N1, R1 = mpr.minplus_power(A, e, 0, ws=mpr.workspace(n * ld * 2 + 256))
            assert torch.equal(N1, N) and torch.equal(R1, R)
    finally:
        mpr.set_arith(prev)


def test_power_empty_rows_stay_empty(mpr):
    X = synth.random_matrix(90, 90, 12, 0, 9, 0.2)
    X[3, :] = 0xFFFF
    for sched in (0, 1):
        N, R = mpr.minplus_power(_dev(mpr, X), 6, sched)
        Nr, Rr = O.power_chain(O.from_u16(X), 6)
        assert np.array_equal(_host(N), _u16(Nr)) and np.array_equal(R.cpu().numpy(), Rr)
        assert int(R[3].item()) == mpr.ROW_NONE


def test_chain_full_size_rows_config2(mpr):
    """N = 8192, 64-step chain (A^64), entries U[0,15] with 30% infinity:
    sampled rows against the oracle's row-restricted chain."""
    n, e = 8192, 64
    X = synth.random_matrix(n, n, 3, 0, 15, 0.30)
    N, R = mpr.minplus_power(_dev(mpr, X), e, mpr.CHAIN, check=True)
    rows = [0, 4097, n - 1]
    Nr, Rr = O.chain_rows(O.from_u16(X), rows, e)
    assert np.array_equal(_host(N)[rows], _u16(Nr))
    assert np.array_equal(R.cpu().numpy()[rows], Rr)


# ------------------------------------------------------------------ traces
def test_traces(mpr):
    A = O.transfer(5)
    Pa, Pb = O.power_chain(A, 6), O.power_chain(A, 9)
    Xd, Yd = _dev(mpr, _u16(Pa[0])), _dev(mpr, _u16(Pb[0]))
    RX, RY = torch.from_numpy(Pa[1]).cuda(), torch.from_numpy(Pb[1]).cuda()
    assert int(mpr.trace_min(Xd, RX).item()) == O.trace(*Pa)
    g = int(mpr.trace_of_product(Xd, RX, Yd, RY).item())
    assert g == O.trace(*O.product_of_powers(*Pa, *Pb)) == O.gamma(5, 15)
    # ragged size, random offsets, empty row
    n = 203
    X = synth.random_matrix(n, n, 21, 0, 30, 0.4)
    Y = synth.random_matrix(n, n, 22, 0, 30, 0.4)
    rx = (np.arange(n) * 7 % 13).astype(np.int64)
    ry = (np.arange(n) * 5 % 11).astype(np.int64)
    rx[4] = O.INF
    X[4, :] = 0xFFFF
    ref = O.trace(*O.product_of_powers(O.from_u16(X), rx, O.from_u16(Y), ry))
    got = int(mpr.trace_of_product(_dev(mpr, X), torch.from_numpy(rx).cuda(), _dev(mpr, Y),
                                   torch.from_numpy(ry).cuda()).item())
    assert got == ref


def _trace_ref(X, rx, Y, ry):
    return O.trace(*O.product_of_powers(O.from_u16(X), rx, O.from_u16(Y), ry))


def test_trace_of_product_offsets_and_layouts(mpr):
    """Tiles whose offsets spread past 2^28 (int64 path) beside tiles that
    do not (32-bit path), huge offsets with a small spread, empty rows and
    whole empty tiles, NULL offsets, and a row stride that is not a
    multiple of 8 (element-wise loads)."""
    n = 300
    X = synth.random_matrix(n, n, 31, 0, 40, 0.3)
    Y = synth.random_matrix(n, n, 32, 0, 40, 0.3)
    base = np.arange(n, dtype=np.int64) % 9
    cases = []
    wide = base.copy()
    wide[:64] += (np.arange(64, dtype=np.int64) * 37 % 5) << 40  # only the first row tile is wide ...
    wide[64:] += 1000  # ... and it holds the minimum
    cases.append(("wide rows", wide, base))
    cases.append(("wide inner", base, wide))
    cases.append(("huge base", base + (1 << 50), base + 123456789012))
    emp = base.copy()
    emp[64:128] = O.INF  # a whole empty row tile
    emp[7] = O.INF
    cases.append(("empty rows", emp, base))
    for name, rx, ry in cases:
        print("trace", name, flush=True)
        got = int(mpr.trace_of_product(_dev(mpr, X), torch.from_numpy(rx).cuda(), _dev(mpr, Y),
                                       torch.from_numpy(ry).cuda()).item())
        assert got == _trace_ref(X, rx, Y, ry), name
    zero = np.zeros(n, dtype=np.int64)
    got = int(mpr.trace_of_product(_dev(mpr, X), None, _dev(mpr, Y), None).item())
    assert got == _trace_ref(X, zero, Y, zero)
    # row stride n + 3 for both operands
    Xp = np.full((n, n + 3), 0xFFFF, np.uint16)
    Yp = np.full((n, n + 3), 0xFFFF, np.uint16)
    Xp[:, :n], Yp[:, :n] = X, Y
    Xd, Yd = torch.from_numpy(Xp).cuda()[:, :n], torch.from_numpy(Yp).cuda()[:, :n]
    assert Xd.stride(0) % 8
    got = int(mpr.trace_of_product(Xd, torch.from_numpy(base).cuda(), Yd, torch.from_numpy(base).cuda()).item())
    assert got == _trace_ref(X, base, Y, base)


def test_trace_of_product_large_chunked(mpr):
    """n = 5900: 93^2 = 8649 tiles, above the size from which the trace
    launch gives each block several tiles (the last block holds one).  The
    reference is the diagonal of (RX (+) X) (x) (RY (+) Y), entry by entry
    from the definition (Corollary 7), then its minimum."""
    n = 5900
    X = synth.random_matrix(n, n, 41, 0, 2000, 0.25)
    Y = synth.random_matrix(n, n, 42, 0, 2000, 0.25)
    rx = (np.arange(n, dtype=np.int64) * 7919 % 61)
    ry = (np.arange(n, dtype=np.int64) * 104729 % 53)
    Xo, Yo = O.from_u16(X), O.from_u16(Y)
    Xr = np.where(Xo == O.INF, O.INF, Xo + rx[:, None])
    Yr = np.where(Yo == O.INF, O.INF, Yo + ry[:, None])
    idx = np.arange(n, dtype=np.int64)
    ref = int(O.minplus_at(Xr, Yr, idx, idx).min())
    got = int(mpr.trace_of_product(_dev(mpr, X), torch.from_numpy(rx).cuda(), _dev(mpr, Y),
                                   torch.from_numpy(ry).cuda()).item())
    assert got == ref
    # the minimum planted in the very last tile (the one-tile last block)
    X2, Y2 = X.copy(), Y.copy()
    X2[n - 1, n - 2] = 0
    Y2[n - 2, n - 1] = 0
    rx2, ry2 = rx + 100, ry + 100
    rx2[n - 1], ry2[n - 2] = 0, 0
    got2 = int(mpr.trace_of_product(_dev(mpr, X2), torch.from_numpy(rx2).cuda(), _dev(mpr, Y2),
                                    torch.from_numpy(ry2).cuda()).item())
    assert got2 == 0


def _trace_t_ref(X, rx, YT, cy):
    """min of the diagonal of (RX (+) X) (x) Y with Y[l][i] = CY[i] + YT[i][l],
    every diagonal entry from the definition of the product (Corollary 7)."""
    Xo, Yo = O.from_u16(X), O.from_u16(YT)
    Xr = np.where((Xo == O.INF) | (rx[:, None] == O.INF), O.INF, Xo + np.where(rx == O.INF, 0, rx)[:, None])
    Yr = np.where((Yo == O.INF) | (cy[:, None] == O.INF), O.INF, Yo + np.where(cy == O.INF, 0, cy)[:, None])
    idx = np.arange(X.shape[0], dtype=np.int64)
    return int(O.minplus_at(Xr, np.ascontiguousarray(Yr.T), idx, idx).min())


@pytest.mark.parametrize("n", [1, 7, 203, 520, 1100])
def test_trace_of_product_t(mpr, n):
    """Right operand given through the canonical form of its transpose:
    row lengths below one 8-value chunk, ragged tails, one and two chunks
    per lane; empty rows on either side, an all-infinite row."""
    X = synth.random_matrix(n, n, 51, 0, 900, 0.4)
    YT = synth.random_matrix(n, n, 52, 0, 900, 0.4)
    rx = (np.arange(n, dtype=np.int64) * 13 % 17)
    cy = (np.arange(n, dtype=np.int64) * 7 % 19)
    if n > 8:
        rx[3] = O.INF
        cy[5] = O.INF
        X[6, :] = 0xFFFF
    ref = _trace_t_ref(X, rx, YT, cy)
    got = int(mpr.trace_of_product_t(_dev(mpr, X), torch.from_numpy(rx).cuda(), _dev(mpr, YT),
                                     torch.from_numpy(cy).cuda()).item())
    assert got == ref


def test_trace_of_product_t_offsets_and_layouts(mpr):
    """Huge offsets, NULL offsets, an all-infinite operand, a row stride that
    is not a multiple of 8 (element-wise loads), and n = 5900 (large)."""
    n = 300
    X = synth.random_matrix(n, n, 53, 0, 40, 0.3)
    YT = synth.random_matrix(n, n, 54, 0, 40, 0.3)
    base = np.arange(n, dtype=np.int64) % 9
    got = int(mpr.trace_of_product_t(_dev(mpr, X), torch.from_numpy(base + (1 << 50)).cuda(), _dev(mpr, YT),
                                     torch.from_numpy(base + 123456789012).cuda()).item())
    assert got == _trace_t_ref(X, base + (1 << 50), YT, base + 123456789012)
    zero = np.zeros(n, dtype=np.int64)
    got = int(mpr.trace_of_product_t(_dev(mpr, X), None, _dev(mpr, YT), None).item())
    assert got == _trace_t_ref(X, zero, YT, zero)
    inf = np.full((n, n), 0xFFFF, np.uint16)
    got = int(mpr.trace_of_product_t(_dev(mpr, inf), None, _dev(mpr, YT), None).item())
    assert got == O.INF
    Xp = np.full((n, n + 3), 0xFFFF, np.uint16)
    Yp = np.full((n, n + 3), 0xFFFF, np.uint16)
    Xp[:, :n], Yp[:, :n] = X, YT
    Xd, Yd = torch.from_numpy(Xp).cuda()[:, :n], torch.from_numpy(Yp).cuda()[:, :n]
    assert Xd.stride(0) % 8
    got = int(mpr.trace_of_product_t(Xd, torch.from_numpy(base).cuda(), Yd, torch.from_numpy(base).cuda()).item())
    assert got == _trace_t_ref(X, base, YT, base)
    n = 5900
    X = synth.random_matrix(n, n, 55, 0, 2000, 0.25)
    YT = synth.random_matrix(n, n, 56, 0, 2000, 0.25)
    rx = (np.arange(n, dtype=np.int64) * 7919 % 61)
    cy = (np.arange(n, dtype=np.int64) * 104729 % 53)
    got = int(mpr.trace_of_product_t(_dev(mpr, X), torch.from_numpy(rx).cuda(), _dev(mpr, YT),
                                     torch.from_numpy(cy).cuda()).item())
    assert got == _trace_t_ref(X, rx, YT, cy)


# ------------------------------------------------------------------ gamma_R and periods
def test_config1_gamma_m3(mpr):
    """P_3 x C_n for n = 3..40 from one GPU chain, vs oracle and brute force."""
    A = mpr.build_transfer(3)
    mu, lam, c, tr = mpr.find_period(A, 40, traces=True)
    assert (mu, lam, c) == (11, 4, 6)
    for n in range(3, 41):
        assert tr[n] == O.gamma(3, n), n
    for n in range(3, 6):
        assert tr[n] == O.brute_gamma(3, n)


@pytest.mark.parametrize("m", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("extend", [False, True])
@pytest.mark.parametrize("pipeline", [False, True])
def test_find_period_small_m(mpr, m, extend, pipeline):
    """Every trace to k = 60 against the oracle, computed power by power or,
    with extend, computed up to the confirming power and extended by the
    period after it; with pipeline, each power computed while the host reads
    the previous one's class hash."""
    A = mpr.build_transfer(m)
    mu, lam, c, tr = mpr.find_period(A, 60, traces=True, extend=extend, pipeline=pipeline)
    omu, olam, oc, og = O.find_period(O.transfer(m), 60)
    assert (mu, lam, c) == (omu, olam, oc)
    for k in range(1, 61):
        ref = O.gamma_from_period(k, omu, olam, oc, og) if k > max(og) else og[k]
        assert tr[k] == ref, k


def test_find_period_stops_early_without_traces(mpr):
    A = mpr.build_transfer(5)
    mu, lam, c, tr = mpr.find_period(A, 300, traces=False)
    assert (mu, lam, c) == (16, 5, 12) and tr is None


def _tiny_cases():
    I = O.INF
    cases = [np.array([[3]]), np.array([[I]]), np.array([[I, 1], [I, I]]), np.array([[I, 0], [5, I]]),
             np.array([[2, I, I], [I, I, 1], [I, 4, I]])]
    rng = np.random.default_rng(5)
    for _ in range(4):
        M = rng.integers(0, 6, (5, 5)).astype(np.int64)
        M[rng.random((5, 5)) < 0.5] = I
        cases.append(M)
    return [c.astype(np.int64) for c in cases]


def test_tiny_and_degenerate_powers_and_periods(mpr):
    """1 x 1 up to 5 x 5 matrices: a single finite entry, all infinite, a
    nilpotent pattern, a weighted 2-cycle, a self-loop beside a 2-cycle of
    another mean (no periodic regime), random sparse ones: every power
    schedule and both period searches against the oracle."""
    for A in _tiny_cases():
        print("tiny", A.shape, flush=True)
        Ad = _dev(mpr, _u16(A))
        for e in (1, 2, 3, 7):
            Nr, Rr = O.power_chain(A, e)
            for schedule in (mpr.CHAIN, mpr.SQUARE, mpr.CHAIN_SPARSE):
                N, R = mpr.minplus_power(Ad, e, schedule)
                assert np.array_equal(_host(N), _u16(Nr)) and np.array_equal(R.cpu().numpy(), Rr), (A, e, schedule)
        mu, lam, c, tr = O.find_period(A, 12)
        for sparse in (False, True):
            for extend in (False, True):
                for pipeline in (False, True):
                    got = mpr.find_period(Ad, 12, traces=True, slots=8, sparse=sparse, extend=extend,
                                          pipeline=pipeline)
                    key = (A.tolist(), sparse, extend, pipeline)
                    assert got[:3] == (mu, lam, c), (key, got[:3], (mu, lam, c))
                    assert all(got[3][k] == tr[k] for k in tr), key
                    if mu is not None:  # every k <= 12, beyond the oracle's own powers by the period
                        for k in range(1, 13):
                            ref = tr[k] if k in tr else tr[mu + (k - mu) % lam]
                            if k not in tr and ref != O.INF:
                                ref += c * ((k - mu) // lam)
                            assert got[3][k] == ref, (key, k)


def test_find_period_pipeline_ring_bound(mpr):
    """A weighted 5-cycle repeats with period 5 from the first power.  A ring
    of 6 powers confirms it, computed power by power and with the next power
    computed ahead (the workspace sized with the pipeline flag holds the
    extra buffer); a pipelined search given only the 6 buffers of the plain
    ring confirms periods up to 4 and reports none."""
    I = O.INF
    L = 5
    A = np.full((L, L), I, dtype=np.int64)
    for i in range(L):
        A[i, (i + 1) % L] = 1 + (i % 2)
    mu, lam, c, tr = O.find_period(A, 30)
    assert lam == L
    Ad = _dev(mpr, _u16(A))
    for pipeline in (False, True):
        got = mpr.find_period(Ad, 30, slots=6, pipeline=pipeline)
        assert got[:3] == (mu, lam, c), pipeline
        assert all(got[3][k] == tr[k] for k in tr), pipeline
    ws = mpr.workspace(mpr.period_workspace_size(L, 6, 0))
    assert mpr.find_period(Ad, 30, ws=ws, pipeline=True)[0] is None
    assert mpr.period_workspace_size(L, 6, mpr.PERIOD_PIPELINE) > mpr.period_workspace_size(L, 6, 0)


def test_find_period_not_found(mpr):
    A = mpr.build_transfer(6)
    mu, lam, c, tr = mpr.find_period(A, 10, traces=True)
    assert mu is None
    assert tr[10] == O.gamma(6, 10)


def test_valu_probe_confirms_the_peak(mpr):
    """The register-only probe of each form's instruction mix runs at or
    below the nominal VALU peak the kernels are priced against (CUs x 64
    lanes x 2.4 GHz x pairs per lane-instruction) and near it; the clock it
    reports is a plausible shader clock."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    for arith, per_lane_clk in (("u16", 1.0), ("f16", 4.0 / 3.0)):
        rate, ghz = mpr.valu_probe(arith, 20000)
        nominal = cus * 64 * per_lane_clk * 2.4e9
        print("probe", arith, rate / 1e9, ghz, flush=True)
        assert 0.7 * nominal < rate < 1.02 * nominal, (arith, rate, nominal)
        assert 1.0 < ghz < 2.6
    with pytest.raises(mpr.MprError):
        mpr.valu_probe("u16", 0)
