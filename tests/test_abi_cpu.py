"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every function include/lpa.h declares; argument errors that are
caught before any device work return their documented codes."""
import ctypes
import os

import pytest

from paper_2411_19901_amd import lpa


def test_library_exports_every_header_function():
    L = lpa.load()
    names = lpa.header_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(L, name), name


def test_error_strings():
    L = lpa.load()
    for code in range(0, 7):
        assert L.lpa_error_string(code)
    assert L.lpa_error_string(99) == b"unknown status"


def test_config_default():
    cfg = lpa.lpa_config_default()
    assert cfg.flags == lpa.LPA_MODE_DET | lpa.LPA_VALIDATE
    assert cfg.rho == 8 and not cfg.stream and cfg.lane_max_degree == 0
    assert cfg.check_every == 0 and not cfg.workspace and cfg.workspace_bytes == 0
    assert cfg.stream_chunk_kib == 0 and list(cfg.reserved) == [0] * 2
    assert cfg.move_blocks_per_cu == 0


def _init(**kw):
    L = lpa.load()
    g = lpa.LpaGraph(kw.get("n", 4), kw.get("nnz", 0), kw.get("rp", 0), kw.get("col", 0),
                     kw.get("rp64", 0))
    cfg = lpa.lpa_config_default()
    for k, v in kw.get("cfg", {}).items():
        setattr(cfg, k, v)
    h = ctypes.c_void_p(123)
    rc = L.lpa_init(ctypes.byref(g) if kw.get("g", True) else None, None, kw.get("k", 8),
                    kw.get("tol", 0.05), kw.get("max_iter", 20), 0, ctypes.byref(cfg),
                    ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("kw,code", [
    (dict(g=False), lpa.LPA_ERR_ARG),
    (dict(n=-1), lpa.LPA_ERR_ARG),
    (dict(n=4, rp=0), lpa.LPA_ERR_ARG),              # null row_ptr with n > 0
    (dict(n=0, nnz=3), lpa.LPA_ERR_ARG),
    (dict(n=4, rp=8, nnz=2**31), lpa.LPA_ERR_ARG),   # nnz beyond int32 offsets
    (dict(n=4, rp=8, rp64=16), lpa.LPA_ERR_ARG),     # both offset widths given
    (dict(n=4, rp64=16, nnz=2**62), lpa.LPA_ERR_ARG),  # beyond the largest graph
    (dict(n=4, rp=8, tol=-0.1), lpa.LPA_ERR_ARG),
    (dict(n=4, rp=8, tol=float("nan")), lpa.LPA_ERR_ARG),
    (dict(n=4, rp=8, max_iter=-1), lpa.LPA_ERR_ARG),
    (dict(n=4, rp=8, cfg=dict(rho=-2)), lpa.LPA_ERR_ARG),
    (dict(n=4, rp=8, k=3), lpa.LPA_ERR_UNSUPPORTED),
    (dict(n=4, rp=8, k=64), lpa.LPA_ERR_UNSUPPORTED),
    (dict(n=4, rp=8, cfg=dict(flags=7)), lpa.LPA_ERR_UNSUPPORTED),
])
def test_init_argument_errors(kw, code):
    rc, h = _init(**kw)
    assert rc == code
    assert not h.value  # *out is cleared on failure


def test_null_handle_calls():
    L = lpa.load()
    assert L.lpa_free(None) == lpa.LPA_OK
    assert L.lpa_step(None, None, None) == lpa.LPA_ERR_ARG
    assert L.lpa_run(None, None) == lpa.LPA_ERR_ARG
    assert L.lpa_last_error(None) == b""


def test_workspace_bytes_host_only():
    det = lpa.workspace_bytes(1000, 20000, k=8, mode="det")
    asy = lpa.workspace_bytes(1000, 20000, k=8, mode="async")
    assert det > 1000 * 14 and asy > 1000 * 9
    assert lpa.workspace_bytes(0, 0) > 0
    L = lpa.load()
    out = ctypes.c_size_t(0)
    assert L.lpa_workspace_bytes(10, 20, 3, 20, None, ctypes.byref(out)) == lpa.LPA_ERR_UNSUPPORTED
    assert L.lpa_workspace_bytes(-1, 20, 8, 20, None, ctypes.byref(out)) == lpa.LPA_ERR_ARG


def test_batch_arguments():
    L = lpa.load()
    b = ctypes.c_void_p(7)
    assert L.lpa_batch_create(0, 8, None, ctypes.byref(b)) == lpa.LPA_ERR_ARG
    assert not b.value
    assert L.lpa_batch_create(4, 5, None, ctypes.byref(b)) == lpa.LPA_ERR_UNSUPPORTED
    assert L.lpa_batch_free(None) == lpa.LPA_OK
    assert L.lpa_batch_run(None, None, 0, None) == lpa.LPA_ERR_ARG


def test_bm_paper_rule_flag():
    # the vote of Algorithm 3 needs k = 1; unknown flag bits are refused
    for mode in ("det", "async"):
        one = lpa.workspace_bytes(5000, 80000, k=1, mode=mode, rule="bm_paper")
        assert one == lpa.workspace_bytes(5000, 80000, k=1, mode=mode)
    L = lpa.load()
    out = ctypes.c_size_t(0)
    cfg = lpa.lpa_config_default()
    cfg.flags = lpa.LPA_MODE_DET | lpa.LPA_RULE_BM_PAPER
    assert L.lpa_workspace_bytes(10, 20, 8, 20, ctypes.byref(cfg), ctypes.byref(out)) == lpa.LPA_ERR_ARG
    assert L.lpa_workspace_bytes(10, 20, 1, 20, ctypes.byref(cfg), ctypes.byref(out)) == lpa.LPA_OK
    cfg.flags = lpa.LPA_MODE_DET | 0x10000
    assert L.lpa_workspace_bytes(10, 20, 1, 20, ctypes.byref(cfg), ctypes.byref(out)) == \
        lpa.LPA_ERR_UNSUPPORTED
    # shared variables instead of votes: det sketch rule without double scan only
    for bad in (lpa.LPA_MODE_ASYNC | lpa.LPA_SHARED_VARS,
                lpa.LPA_MODE_DET | lpa.LPA_SHARED_VARS | lpa.LPA_RESCAN,
                lpa.LPA_MODE_DET | lpa.LPA_SHARED_VARS | lpa.LPA_RULE_BM_PAPER):
        cfg.flags = bad
        assert L.lpa_workspace_bytes(10, 20, 1, 20, ctypes.byref(cfg), ctypes.byref(out)) == \
            lpa.LPA_ERR_ARG
    cfg.flags = lpa.LPA_MODE_DET | lpa.LPA_SHARED_VARS
    assert L.lpa_workspace_bytes(10, 20, 8, 20, ctypes.byref(cfg), ctypes.byref(out)) == lpa.LPA_OK
    # one shared sketch per hub: async sketch rule without double scan only
    for bad in (lpa.LPA_MODE_DET | lpa.LPA_HUB_SHARED,
                lpa.LPA_MODE_ASYNC | lpa.LPA_HUB_SHARED | lpa.LPA_RESCAN,
                lpa.LPA_MODE_ASYNC | lpa.LPA_HUB_SHARED | lpa.LPA_RULE_BM_PAPER):
        cfg.flags = bad
        assert L.lpa_workspace_bytes(10, 20, 1, 20, ctypes.byref(cfg), ctypes.byref(out)) == \
            lpa.LPA_ERR_ARG
    cfg.flags = lpa.LPA_MODE_ASYNC | lpa.LPA_HUB_SHARED
    assert L.lpa_workspace_bytes(10, 20, 8, 20, ctypes.byref(cfg), ctypes.byref(out)) == lpa.LPA_OK
    # the double scan needs the sketch rule
    cfg.flags = lpa.LPA_MODE_DET | lpa.LPA_RULE_BM_PAPER | lpa.LPA_RESCAN
    assert L.lpa_workspace_bytes(10, 20, 1, 20, ctypes.byref(cfg), ctypes.byref(out)) == lpa.LPA_ERR_ARG
    # the double scan needs hub candidates only in async mode
    assert lpa.workspace_bytes(5000, 80000, k=8, mode="det", rescan=True) == \
        lpa.workspace_bytes(5000, 80000, k=8, mode="det")
    assert lpa.workspace_bytes(5000, 80000, k=8, mode="async", rescan=True) > \
        lpa.workspace_bytes(5000, 80000, k=8, mode="async")
    b = ctypes.c_void_p()
    cfg.flags = lpa.LPA_MODE_DET | lpa.LPA_RULE_BM_PAPER
    assert L.lpa_batch_create(4, 8, ctypes.byref(cfg), ctypes.byref(b)) == lpa.LPA_ERR_ARG


def test_offsets64_workspace_bounds():
    """The workspace size does not depend on the offset width; graphs of
    2^31 or more entries are sized, up to 2^62 entries, as long as the
    async hub segments stay below 2^30."""
    L = lpa.load()
    out = ctypes.c_size_t(0)
    cfg = lpa.lpa_config_default()
    for flags in (lpa.LPA_MODE_DET, lpa.LPA_MODE_ASYNC):
        cfg.flags = flags
        assert L.lpa_workspace_bytes(1 << 25, 1 << 32, 8, 20, ctypes.byref(cfg),
                                     ctypes.byref(out)) == lpa.LPA_OK
        assert out.value > (1 << 25) * 9
        assert L.lpa_workspace_bytes(1 << 25, 1 << 62, 8, 20, ctypes.byref(cfg),
                                     ctypes.byref(out)) == lpa.LPA_ERR_ARG
    cfg.flags = lpa.LPA_MODE_ASYNC
    cfg.lane_max_degree = 1  # one segment per entry: far too many
    assert L.lpa_workspace_bytes(1 << 25, 1 << 31, 8, 20, ctypes.byref(cfg),
                                 ctypes.byref(out)) == lpa.LPA_ERR_UNSUPPORTED
    cfg.flags = lpa.LPA_MODE_DET  # no segments in det mode
    assert L.lpa_workspace_bytes(1 << 25, 1 << 31, 8, 20, ctypes.byref(cfg),
                                 ctypes.byref(out)) == lpa.LPA_OK


def test_stream_csr_config():
    """Streaming excludes the shared hub sketch; the chunk size and the
    reserved words are checked before any device work."""
    L = lpa.load()
    out = ctypes.c_size_t(0)
    cfg = lpa.lpa_config_default()
    cfg.flags = lpa.LPA_MODE_DET | lpa.LPA_STREAM_CSR
    cfg.stream_chunk_kib = 64
    assert L.lpa_workspace_bytes(1000, 20000, 8, 20, ctypes.byref(cfg), ctypes.byref(out)) == \
        lpa.LPA_OK
    cfg.flags = lpa.LPA_MODE_ASYNC | lpa.LPA_STREAM_CSR
    assert L.lpa_workspace_bytes(1000, 20000, 8, 20, ctypes.byref(cfg), ctypes.byref(out)) == \
        lpa.LPA_OK
    cfg.flags = lpa.LPA_MODE_ASYNC | lpa.LPA_STREAM_CSR | lpa.LPA_HUB_SHARED
    assert L.lpa_workspace_bytes(1000, 20000, 8, 20, ctypes.byref(cfg), ctypes.byref(out)) == \
        lpa.LPA_ERR_ARG
    cfg.flags = lpa.LPA_MODE_DET | lpa.LPA_STREAM_CSR
    cfg.stream_chunk_kib = -1
    assert L.lpa_workspace_bytes(1000, 20000, 8, 20, ctypes.byref(cfg), ctypes.byref(out)) == \
        lpa.LPA_ERR_ARG
    cfg.stream_chunk_kib = 0
    cfg.reserved[0] = 1
    assert L.lpa_workspace_bytes(1000, 20000, 8, 20, ctypes.byref(cfg), ctypes.byref(out)) == \
        lpa.LPA_ERR_ARG
    cfg.reserved[0] = 0
    for blocks, code in ((-1, lpa.LPA_ERR_ARG), (65, lpa.LPA_ERR_ARG), (1, lpa.LPA_OK),
                         (64, lpa.LPA_OK)):
        cfg.move_blocks_per_cu = blocks
        assert L.lpa_workspace_bytes(1000, 20000, 8, 20, ctypes.byref(cfg),
                                     ctypes.byref(out)) == code


def test_ranked_layout_workspace():
    # the ranked layout adds the rewritten column indices (4 B per entry) and
    # a 4 B per vertex transfer buffer; it cannot be combined with streaming
    for mode in ("det", "async"):
        plain = lpa.workspace_bytes(5000, 80000, k=8, mode=mode)
        ranked = lpa.workspace_bytes(5000, 80000, k=8, mode=mode, ranked=True)
        assert ranked >= plain + 4 * 80000 + 4 * 5000
        assert ranked <= plain + 4 * 80000 + 4 * 5000 + 1024
    L = lpa.load()
    out = ctypes.c_size_t(0)
    cfg = lpa.lpa_config_default()
    cfg.flags = lpa.LPA_MODE_DET | lpa.LPA_RANKED_LAYOUT | lpa.LPA_STREAM_CSR
    assert L.lpa_workspace_bytes(10, 20, 8, 20, ctypes.byref(cfg), ctypes.byref(out)) == lpa.LPA_ERR_ARG
