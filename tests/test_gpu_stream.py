"""Streaming a graph from pinned host memory (LPA_STREAM_CSR).

The rows are copied to the device range by range every iteration.  In det
mode the synchronous update reads only the previous iteration's labels, so
the result must equal the oracle bit for bit whatever the cut: labels,
iteration count, changed and scanned counts, modularity.  Chunks from
1 KiB (256 entries, so a star's centre is a range of its own and the
buffers grow to hold it) to one range for the whole graph; every rule and
option of det mode; int64 offsets; rejections.  Async mode (each range with
its own hub segments): valid labels, every entry scanned in the first
iteration, modularity equal to the oracle's of the same labels and quality
on the planted partition.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2411_19901_amd import inputs, lpa  # noqa: E402
from test_gpu_parity import graph  # noqa: E402  (the parity graph suite)

pytestmark = pytest.mark.gpu


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def pinned(g, offsets64=False):
    rp = g.row_ptr.astype(np.int64) if offsets64 else np.ascontiguousarray(g.row_ptr)
    return (torch.from_numpy(rp).pin_memory(), torch.from_numpy(np.ascontiguousarray(g.col)).pin_memory(),
            torch.from_numpy(g.w).pin_memory() if g.w is not None else None)


def oracle_run(g, k, **kw):
    ok = oracle.BM_PAPER if kw.get("rule") == "bm_paper" else k
    return oracle.lpa_run(g.row_ptr, g.col, g.w, k=ok, rescan=kw.get("rescan", False))


def check(g, chunk_kib, offsets64=False, **kw):
    need_gpu()
    rp, col, w = pinned(g, offsets64)
    k = kw.pop("k", 8)
    s = lpa.LPA(rp, col, w, k=k, mode="det", stream_csr=True, stream_chunk_kib=chunk_kib, **kw)
    it = s.run()
    lab = s.labels(device=False)
    dn, sc = s.trace()
    ref, rit, rdn, rsc = oracle_run(g, k, **kw)
    assert it == rit and np.array_equal(dn, rdn) and np.array_equal(sc, rsc), (g.name, chunk_kib)
    assert np.array_equal(lab, ref), (g.name, chunk_kib)
    assert abs(s.modularity() - oracle.modularity(g.row_ptr, g.col, g.w, ref)) <= 1e-9
    core, _ = s.memory()
    s.close()
    return core


@pytest.mark.parametrize("name", ["two-cliques-5", "sbm1-s2-w", "rmat14-w", "star5000",
                                  "rmat10-selfloops", "sbm1-iso"])
@pytest.mark.parametrize("chunk_kib", [1, 16, 0])
def test_stream_det_parity(name, chunk_kib):
    check(graph(name), chunk_kib)


@pytest.mark.parametrize("variant", [dict(k=1), dict(k=32), dict(k=8, lane_max_degree=64),
                                     dict(k=1, rule="bm_paper"), dict(k=8, rescan=True),
                                     dict(k=8, shared_vars=True, lane_max_degree=16)])
def test_stream_variants(variant):
    check(graph("rmat14-w"), 4, **variant)


def test_stream_offsets64_and_device_offsets():
    need_gpu()
    g = graph("rmat14-w")
    check(g, 8, offsets64=True)
    # row offsets in device memory, rows in pinned host memory
    rp, col, w = pinned(g)
    s = lpa.LPA(rp.cuda(), col, w, k=8, mode="det", stream_csr=True, stream_chunk_kib=8)
    s.run()
    assert np.array_equal(s.labels(device=False), oracle_run(g, 8)[0])
    s.close()


def test_stream_larger_graph():
    g = inputs.with_uniform_weights(inputs.rmat(18), 18)
    core = check(g, 256)  # about 16 ranges of 64K entries
    assert core < 64 * g.n + 8 * (1 << 20)  # O(|V|) plus two 256 KiB slices


def test_stream_step_reset_profile():
    need_gpu()
    g = graph("sbm1-s2-w")
    rp, col, w = pinned(g)
    s = lpa.LPA(rp, col, w, k=8, mode="det", stream_csr=True, stream_chunk_kib=2)
    s.profile(True)
    steps = 0
    while True:
        _, done = s.step()
        steps += 1
        if done:
            break
    lab = s.labels(device=False)
    ref, rit, _, _ = oracle_run(g, 8)
    assert steps == rit and np.array_equal(lab, ref)
    ms = s.move_ms()
    assert len(ms) == rit and np.all(ms > 0)
    s.reset()
    assert s.run() == rit and np.array_equal(s.labels(device=False), ref)
    s.close()


def test_stream_rejections():
    need_gpu()
    g = graph("sbm1-s1")
    rp, col, w = pinned(g)
    with pytest.raises(lpa.LpaError) as ei:  # no shared hub sketch when streaming
        lpa.LPA(rp, col, w, k=8, mode="async", stream_csr=True, hub_shared=True)
    assert ei.value.code == lpa.LPA_ERR_ARG
    with pytest.raises(lpa.LpaError) as ei:  # rows must be in pinned host memory
        lpa.LPA(rp, col.cuda(), w, k=8, mode="det", stream_csr=True)
    assert ei.value.code == lpa.LPA_ERR_ARG
    s = lpa.LPA(rp, col, w, k=8, mode="det", stream_csr=True, stream_chunk_kib=4)
    batch = lpa.Batch(2, k=8)
    with pytest.raises(lpa.LpaError):  # streamed graphs run alone
        batch.run([s])
    batch.close()
    s.close()


@pytest.mark.parametrize("chunk_kib", [1, 16, 0])
@pytest.mark.parametrize("variant", [dict(k=8), dict(k=8, lane_max_degree=64),
                                     dict(k=1, rule="bm_paper"), dict(k=8, rescan=True)])
def test_stream_async(chunk_kib, variant):
    need_gpu()
    for name in ("sbm1-s1", "rmat14-w", "star5000"):
        g = graph(name)
        rp, col, w = pinned(g)
        s = lpa.LPA(rp, col, w, mode="async", stream_csr=True, stream_chunk_kib=chunk_kib,
                    **variant)
        it = s.run()
        lab = s.labels(device=False)
        assert 1 <= it <= 20 and lab.min() >= 0 and lab.max() < g.n
        assert s.trace()[1][0] == g.nnz  # every entry scanned in the first iteration
        q = s.modularity()
        assert abs(q - oracle.modularity(g.row_ptr, g.col, g.w, lab)) <= 1e-9
        if name == "sbm1-s1" and variant.get("rule") != "bm_paper":
            q_exact = oracle.modularity(g.row_ptr, g.col, None,
                                        oracle.lpa_run(g.row_ptr, g.col, None, k=0)[0])
            assert q > 0.9 * q_exact, (q, q_exact)
        s.close()
