"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/mpr.h declares, and its host-only entry points and
argument checks behave as documented."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def mpr():
    import paper_2409_17658_amd as m

    if not os.path.exists(m.LIB_PATH):
        from paper_2409_17658_amd import build

        build.build()
    m.lib()
    return m


def _declared():
    src = open(os.path.join(ROOT, "include", "mpr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mpr_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(mpr):
    names = _declared()
    assert len(names) >= 25
    L = mpr.lib()
    for n in names:
        assert hasattr(L, n), n
    # and the binding declares a signature for each of them
    assert set(names) == set(mpr.exported_symbols())


def test_transfer_size_matches_table1(mpr, paper_values):
    for m, c in paper_values["word_counts"]["values"].items():
        assert mpr.transfer_size(int(m)) == c


def test_transfer_words_match_oracle_order(mpr):
    for m in range(1, 12):  # up to the largest m the builder accepts
        assert np.array_equal(mpr.transfer_words(m), O.words(m)), m


def test_argument_errors_are_synchronous(mpr):
    L = mpr.lib()
    n = ctypes.c_int64()
    assert L.mpr_transfer_size(0, ctypes.byref(n)) == 1
    assert L.mpr_transfer_size(13, ctypes.byref(n)) == 1
    assert L.mpr_transfer_size(3, None) == 1
    # negative sizes, missing pointers, short leading dimensions
    assert L.mpr_minplus_gemm(-1, 4, 4, None, 4, None, 4, None, 4, None, None) == 1
    assert L.mpr_minplus_gemm(4, 4, 4, None, 4, None, 4, None, 4, None, None) == 1
    p = ctypes.c_void_p(16)
    assert L.mpr_minplus_gemm(4, 8, 4, p, 3, p, 8, p, 8, None, None) == 1
    assert L.mpr_minplus_gemm_spare(-1, 4, 8, 4, p, 3, p, 8, p, 8, None, None) == 1
    assert L.mpr_minplus_gemm_spare(99, 4, 8, 4, p, 4, p, 8, p, 8, None, None) == 1  # no such configuration
    assert L.mpr_minplus_power(p, 4, 4, 0, 0, p, 4, p, p, 1 << 20, None, None) == 1
    assert L.mpr_minplus_power(p, 4, 4, 3, 7, p, 4, p, p, 1 << 20, None, None) == 1
    assert L.mpr_minplus_power(p, 4, 4, 3, 0, p, 4, p, p, 16, None, None) == 2  # workspace too small
    assert L.mpr_build_transfer(12, p, 1 << 20, None) == 1
    nb = ctypes.c_size_t()
    assert L.mpr_period_workspace_size_ex(8, 4, 4 | 8, ctypes.byref(nb)) == 1  # pipeline with reuse_a
    assert L.mpr_period_workspace_size_ex(8, 4, 16, ctypes.byref(nb)) == 1    # no such flag
    # chain_resume: squaring is not a chain, negative steps, in place with another stride
    assert L.mpr_chain_resume(p, 4, 8, p, 8, p, 3, 1, p, 8, p, p, 1 << 20, None, None) == 1
    assert L.mpr_chain_resume(p, 4, 8, p, 8, p, -1, 0, p, 8, p, p, 1 << 20, None, None) == 1
    assert L.mpr_chain_resume(p, 4, 8, p, 8, p, 3, 0, p, 16, p, p, 1 << 20, None, None) == 1
    assert L.mpr_chain_resume(p, 4, 8, p, 8, p, 3, 0, ctypes.c_void_p(32), 8, p, p, 16, None, None) == 2
    assert L.mpr_batch_launch(ctypes.c_void_p(12345), None, None) == 1  # never planned
    assert L.mpr_graph_launch(None, None) == 1
    assert mpr.lib().mpr_status_string(3).decode().startswith("finite value")
    assert mpr.lib().mpr_status_string(7).decode().startswith("request waited")
    assert mpr.lib().mpr_status_string(8).decode() == "request cancelled"


def test_workspace_sizes(mpr):
    ws_chain = mpr.power_workspace_size(1000, 10, mpr.CHAIN)
    ws_sq = mpr.power_workspace_size(1000, 10, mpr.SQUARE)
    assert ws_chain >= 1000 * 1000 * 2 and ws_sq >= 4 * 1000 * 1000 * 2
    assert mpr.period_workspace_size(100, 10) >= 10 * 100 * 104 * 2
    with pytest.raises(mpr.MprError):
        mpr.period_workspace_size(100, 1)


def test_chain_workspace_holds_split_k_parts(mpr):
    """The chain of a matrix too small to fill the device with 64 x 64 tiles
    gets room for the partial products of split-k steps (each range of k
    at least 128 deep, at most 8 ranges); a large one gets the layout only
    (its ping-pong buffer plus 256 bytes).  Sizes as on a 256-CU device."""
    layout = lambda n: n * ((n + 7) // 8 * 8) * 2 + 256
    assert mpr.power_workspace_size(8192, 5, mpr.CHAIN) == layout(8192)
    assert mpr.power_workspace_size(2000, 5, mpr.CHAIN) == layout(2000)  # 1024 tiles
    assert mpr.power_workspace_size(200, 5, mpr.CHAIN) == layout(200)  # k = 200 is too short to split
    # n = 300: 25 tiles, k = 300 gives 2 ranges, so one partial product
    assert mpr.power_workspace_size(300, 5, mpr.CHAIN) == layout(300) + 300 * 304 * 2 + 256
    # n = 848: 196 tiles, 6 ranges of k (ceil(1024 / 196) = 6 <= 848 // 128)
    assert mpr.power_workspace_size(848, 5, mpr.CHAIN) == layout(848) + 5 * 848 * 848 * 2 + 256


def test_configs_describe_themselves(mpr):
    for c in range(mpr.gemm_config_count()):
        info = mpr.gemm_config_info(c)
        assert info["bm"] % info["tm"] == 0 and info["bn"] % info["tn"] == 0
        assert info["threads"] == (info["bm"] // info["tm"]) * (info["bn"] // info["tn"])
    for c in range(mpr.batch_config_count()):
        assert mpr.batch_config_info(c)["panel_rows"] in (32, 64, 128)
    with pytest.raises(mpr.MprError):
        mpr.set_tile_table([(100, 0), (50, 1)])  # not ascending
    with pytest.raises(mpr.MprError):
        mpr.set_tile_table([(100, 3), (1 << 62, 6)])  # two arithmetics in one table
    from paper_2409_17658_amd import autotune

    try:
        mpr.set_tile_table([(96, 3), (1024, 0), (1 << 62, 1)])
        mpr.set_tile_table([(96, 9), (1 << 62, 13)])
        assert mpr.get_arith() == "u16"  # the default arithmetic
        assert [mpr.gemm_pick_config(k, k, k) for k in (50, 500, 5000)] == [3, 0, 1]
        with mpr.arith_scope("f16"):
            assert [mpr.gemm_pick_config(k, k, k) for k in (50, 500, 5000)] == [9, 13, 13]
        assert mpr.get_arith() == "u16"
        with pytest.raises(ValueError):
            mpr.set_arith("f32")
    finally:
        autotune.load_table()


def test_sparse_form_setting(mpr):
    """The form of the compressed-K step is a process-wide setting with three
    values; anything else is refused by the binding and by the library."""
    for f in ("tiles", "entries", "auto"):
        mpr.set_sparse_form(f)
    with pytest.raises(ValueError):
        mpr.set_sparse_form("dense")
    assert mpr.lib().mpr_set_sparse_form(3) == 1 and mpr.lib().mpr_set_sparse_form(-1) == 1  # MPR_EINVAL
    assert mpr.lib().mpr_set_sparse_form(0) == 0


def test_batch_weights_install_and_reset(mpr):
    """Weights of the batched-configuration model: one per configuration,
    non-negative, each arithmetic keeping one; None restores the prior."""
    cnt = mpr.batch_config_count()
    prior = mpr.get_batch_weights()
    try:
        mpr.set_batch_weights(None)
        base = mpr.get_batch_weights()
        assert len(base) == cnt and all(w > 0 for w in base)
        w = [0.0] * cnt
        w[2], w[9] = 1.0, 0.5
        mpr.set_batch_weights(w)
        assert mpr.get_batch_weights() == w
        for bad in ([1.0] * (cnt - 1), [0.0] * cnt, [-1.0] + [1.0] * (cnt - 1),
                    [1.0] * 6 + [0.0] * (cnt - 6)):
            with pytest.raises((mpr.MprError, ValueError)):
                mpr.set_batch_weights(bad)
        assert mpr.get_batch_weights() == w  # a refused table leaves the installed one
    finally:
        mpr.set_batch_weights(prior)


def test_product_path_has_no_oracle_import():
    """The product package never imports the oracle (or any CPU fallback)."""
    pkg = os.path.join(ROOT, "paper_2409_17658_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "liboracle" not in txt, f


def test_binding_rejects_mistyped_buffers(mpr):
    """Offset vectors must be contiguous int64 of the right length and
    matrices 2-D uint16 with unit column stride; anything else is refused on
    the host before a pointer reaches the library."""
    import torch

    for bad in (torch.zeros(8, dtype=torch.int32), torch.zeros(4, dtype=torch.int64),
                torch.zeros(16, dtype=torch.int64)[::2], torch.zeros((2, 4), dtype=torch.int64)):
        with pytest.raises(ValueError):
            mpr._vptr(bad, 8)
    assert mpr._vptr(None, 8) is None
    for bad in (torch.zeros((4, 4), dtype=torch.int16), torch.zeros((4, 8), dtype=torch.uint16)[:, ::2],
                torch.zeros(16, dtype=torch.uint16)):
        with pytest.raises(ValueError):
            mpr._ld(bad)
    assert mpr._ld(torch.zeros((4, 8), dtype=torch.uint16)[:, :5]) == 8


def test_trace_t_binding_checks(mpr):
    """trace_of_product_t refuses operands with different row strides and
    mistyped offset vectors on the host, before any library call."""
    import torch

    X = torch.zeros((8, 8), dtype=torch.uint16)
    Y = torch.zeros((8, 16), dtype=torch.uint16)[:, :8]
    with pytest.raises(ValueError):
        mpr.trace_of_product_t(X, None, Y, None)
    with pytest.raises(ValueError):
        mpr.trace_of_product_t(X, torch.zeros(8, dtype=torch.int32), X, None)
    with pytest.raises(ValueError):
        mpr.trace_of_product_t(X, None, X, torch.zeros(4, dtype=torch.int64))


def test_tile_table_loader_checks_configurations(mpr, tmp_path):
    """A persisted table is installed only when it was tuned on the
    configurations the loaded library has."""
    import json

    from paper_2409_17658_amd import autotune

    cfgs = [mpr.gemm_config_info(c) for c in range(mpr.gemm_config_count())]
    good = {"configs": cfgs, "measurements": [], "tables": {"u16": [[500, 3], [1 << 62, 1]],
                                                             "f16": [[500, 9], [1 << 62, 7]]}}
    p = tmp_path / "t.json"
    p.write_text(json.dumps(good))
    try:
        assert autotune.load_table(str(p))
        assert mpr.gemm_pick_config(400, 400, 400) == 3 and mpr.gemm_pick_config(600, 600, 600) == 1
        with mpr.arith_scope("f16"):
            assert mpr.gemm_pick_config(400, 400, 400) == 9 and mpr.gemm_pick_config(600, 600, 600) == 7
        for bad in ({**good, "configs": cfgs[:-1]},
                    {**good, "configs": [dict(cfgs[0], bm=cfgs[0]["bm"] * 2)] + cfgs[1:]},
                    {"configs": cfgs, "measurements": [], "table": [[500, 3], [1 << 62, 1]]}):
            p.write_text(json.dumps(bad))
            assert not autotune.load_table(str(p))
            assert mpr.gemm_pick_config(400, 400, 400) == 3  # the installed table stays
        assert not autotune.load_table(str(tmp_path / "missing.json"))
    finally:
        autotune.load_table()  # the persisted table again
