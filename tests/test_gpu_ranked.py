"""LPA_RANKED_LAYOUT: labels and flags stored by degree-order position, with
the column indices rewritten as positions.  The layout changes where state
lives, not what is computed: LPA_MODE_DET must still reproduce the oracle
bit for bit (labels, iterations, per-iteration changed and scanned counts,
and the unprocessed flags of every iteration), whatever k, rule, threshold
or offset width, alone or batched with handles of the default layout;
checkpoints cross between the layouts; modularity agrees to 1e-9; the
all-hub async graphs stay exact against the partial-sketch oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2411_19901_amd import inputs, lpa  # noqa: E402
from test_gpu_hub_segments import graph as hub_graph  # noqa: E402
from test_gpu_hub_segments import run_and_check  # noqa: E402
from test_gpu_parity import GRAPHS, graph, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def solve(g, k, ranked=True, offsets64=False, **kw):
    rp, col, w = to_dev(g)
    if offsets64:
        rp = rp.to(torch.int64)
    s = lpa.LPA(rp, col, w, k=k, ranked=ranked, **kw)
    it = s.run()
    out = (s.labels(device=False), it, *s.trace(), s.modularity())
    s.close()
    return out


def oracle_run(g, k, **kw):
    kk = oracle.BM_PAPER if kw.get("rule") == "bm_paper" else k
    return oracle.lpa_run(g.row_ptr, g.col, g.w, k=kk, rescan=kw.get("rescan", False))


def check(g, k, **kw):
    labels, it, dn, sc, q = solve(g, k, **kw)
    okw = {x: kw[x] for x in ("rule", "rescan") if x in kw}
    ref, rit, rdn, rsc = oracle_run(g, k, **okw)
    assert it == rit, (g.name, k, it, rit)
    assert np.array_equal(dn, rdn) and np.array_equal(sc, rsc), (g.name, k)
    bad = np.nonzero(labels != ref)[0]
    assert bad.size == 0, (g.name, k, bad[:5])
    assert abs(q - oracle.modularity(g.row_ptr, g.col, g.w, ref)) <= 1e-9


@pytest.mark.parametrize("name", GRAPHS)
@pytest.mark.parametrize("k", [1, 8, 16])
def test_ranked_det_parity(name, k):
    check(graph(name), k)


@pytest.mark.parametrize("lane_max", [1, 64])
@pytest.mark.parametrize("variant", ["mg32", "bm_paper", "rescan", "shared_vars", "offsets64"])
def test_ranked_det_variants(variant, lane_max):
    g = graph("rmat14-w")
    kw = dict(mode="det", lane_max_degree=lane_max)
    if variant == "mg32":
        check(g, 32, **kw)
    elif variant == "bm_paper":
        check(g, 1, rule="bm_paper", **kw)
    elif variant == "rescan":
        check(g, 8, rescan=True, **kw)
    elif variant == "shared_vars":
        check(g, 8, shared_vars=True, **kw)
    else:
        check(g, 8, offsets64=True, **kw)


def test_ranked_every_iteration_with_flags():
    # iteration by iteration, state read back by vertex id: labels, the
    # flags the next iteration reads, the changed counts
    g = graph("rmat14-w")
    rp, col, w = to_dev(g)
    s = lpa.LPA(rp, col, w, k=8, ranked=True)
    deg = g.degrees()
    for _ in range(20):
        C, act, l = s.get_state()
        ch, done = s.step()
        C2, act2, _ = s.get_state()
        Cr, actr, dnr, _ = oracle.lpa_move(g.row_ptr, g.col, g.w, 8, l % 8 == 0, C, act)
        assert ch == dnr
        assert np.array_equal(C2, Cr)
        nz = deg > 0
        assert np.array_equal(act2[nz] != 0, actr[nz] != 0)
        if done:
            break
    s.close()


def test_checkpoint_across_layouts():
    g = graph("sbm1-s2-w")
    rp, col, w = to_dev(g)
    a = lpa.LPA(rp, col, w, k=8, ranked=True)
    for _ in range(3):
        a.step()
    lab, flags, it = a.get_state()
    b = lpa.LPA(rp, col, w, k=8)           # default layout continues the ranked run
    b.set_state(lab, flags, it)
    c = lpa.LPA(rp, col, w, k=8, ranked=True)  # and a second ranked handle
    c.set_state(lab, flags, it)
    a.run()
    b.run()
    c.run()
    ref, _, _, _ = oracle.lpa_run(g.row_ptr, g.col, g.w, k=8)
    for s in (a, b, c):
        assert np.array_equal(s.labels(device=False), ref)
        s.close()


def test_ranked_device_labels_and_given_modularity():
    g = graph("rmat14-w")
    rp, col, w = to_dev(g)
    s = lpa.LPA(rp, col, w, k=8, ranked=True)
    s.run()
    dev_lab = s.labels(device=True)
    host_lab = s.labels(device=False)
    assert np.array_equal(dev_lab.cpu().numpy(), host_lab)
    rng = np.random.default_rng(3)
    given = rng.integers(0, g.n, g.n).astype(np.int32)
    q = s.modularity(torch.from_numpy(given).to(rp.device))
    assert abs(q - oracle.modularity(g.row_ptr, g.col, g.w, given)) <= 1e-9
    q0 = s.modularity()
    assert abs(q0 - oracle.modularity(g.row_ptr, g.col, g.w, host_lab)) <= 1e-9
    assert abs(lpa.lpa_modularity_noalloc(s.h) - q0) <= 1e-9
    core, _ = s.memory()
    s.close()
    plain = lpa.LPA(rp, col, w, k=8)
    core0, _ = plain.memory()
    plain.close()
    assert core >= core0 + 4 * g.nnz  # the rewritten column indices
    assert lpa.workspace_bytes(g.n, g.nnz, ranked=True) >= core


@pytest.mark.parametrize("mode", ["det", "async"])
def test_batch_mixes_layouts(mode):
    gs = [graph(x) for x in ("sbm1-s1", "rmat12", "sbm1-iso", "grid64", "rmat14-w")]
    d = to_dev(gs[0])[0].device
    stream = torch.cuda.current_stream(d)
    solvers = []
    for i, g in enumerate(gs):
        rp, col, w = to_dev(g)
        solvers.append(lpa.LPA(rp, col, w, k=8, mode=mode, ranked=i % 2 == 0, stream=stream))
    b = lpa.Batch(len(solvers), k=8, mode=mode, stream=stream)
    b.reset(solvers)
    b.run(solvers)
    for g, s in zip(gs, solvers):
        lab = s.labels(device=False)
        if mode == "det":
            ref, it, _, _ = oracle.lpa_run(g.row_ptr, g.col, g.w, k=8)
            assert np.array_equal(lab, ref), g.name
            assert s.iterations() == it
        else:
            assert lab.min() >= 0 and lab.max() < g.n
            assert abs(s.modularity() - oracle.modularity(g.row_ptr, g.col, g.w, lab)) <= 1e-9
        s.close()
    b.close()


def test_ranked_async_quality_sbm():
    g = graph("sbm1-s1")
    labels, it, _, _, q = solve(g, 8, mode="async")
    assert 1 <= it <= 20 and labels.min() >= 0 and labels.max() < g.n
    ref, _, _, _ = oracle.lpa_run(g.row_ptr, g.col, None, k=0)
    q_exact = oracle.modularity(g.row_ptr, g.col, None, ref)
    assert q >= 0.9 * q_exact, (q, q_exact)


@pytest.mark.parametrize("kind", ["narrow", "wide"])
@pytest.mark.parametrize("k", [1, 8, 16])
def test_ranked_all_hub_async_exact(kind, k):
    run_and_check(hub_graph(kind, "unit"), k, rescan=False, ranked=True)


def test_ranked_refused_with_streamed_csr():
    g = graph("rmat12")
    rp = torch.from_numpy(g.row_ptr).pin_memory()
    col = torch.from_numpy(g.col).pin_memory()
    with pytest.raises(lpa.LpaError) as e:
        lpa.LPA(rp, col, None, k=8, stream_csr=True, ranked=True)
    assert e.value.code == lpa.LPA_ERR_ARG
