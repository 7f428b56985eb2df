"""GPU parity: the HIP path through the C ABI against the CPU oracle.

LPA_MODE_DET must reproduce the oracle bit for bit (labels, iteration
count, per-iteration changed and scanned counts) for every k, on graphs
that span many tiles and ragged tails, with hubs, self-loops, isolated
vertices and weighted edges; modularity must agree to |dQ| <= 1e-9.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2411_19901_amd import inputs, lpa  # noqa: E402

pytestmark = pytest.mark.gpu

KS = [1, 2, 4, 8, 16, 32]


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev(g):
    d = dev()
    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(d)
    col = torch.from_numpy(np.ascontiguousarray(g.col)).to(d)
    w = torch.from_numpy(g.w).to(d) if g.w is not None else None
    return rp, col, w


def gpu_run(g, k, mode="det", tol=0.05, max_iter=20, rho=8, lane_max_degree=0, rule="mg",
            rescan=False, shared_vars=False):
    rp, col, w = to_dev(g)
    s = lpa.LPA(rp, col, w, k=k, tol=tol, max_iter=max_iter, rho=rho, mode=mode,
                lane_max_degree=lane_max_degree, rule=rule, rescan=rescan,
                shared_vars=shared_vars)
    it = s.run()
    labels = s.labels(device=False)
    dn, sc = s.trace()
    q = s.modularity()
    s.close()
    return labels, it, dn, sc, q


def with_self_loops(g, every=7):
    """Add a self-loop to every `every`-th vertex (kept sorted)."""
    n = g.n
    rows = []
    ws = []
    for i in range(n):
        r = list(g.col[g.row_ptr[i]:g.row_ptr[i + 1]])
        wr = list(g.w[g.row_ptr[i]:g.row_ptr[i + 1]]) if g.w is not None else [1.0] * len(r)
        if i % every == 0:
            pos = int(np.searchsorted(r, i))
            r.insert(pos, i)
            wr.insert(pos, 0.5)
        rows.append(r)
        ws.append(wr)
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([j for r in rows for j in r], np.int32)
    w = np.array([x for r in ws for x in r], np.float32)
    return inputs.Graph(rp, col, w, g.name + "-selfloops")


def star(leaves):
    edges = [(0, i) for i in range(1, leaves + 1)]
    # a few leaf-leaf edges so leaves have something to choose between
    edges += [(i, i + 1) for i in range(1, leaves, 3)]
    return inputs.from_edges(leaves + 1, edges, name=f"star{leaves}")


def with_isolated(g, extra=37):
    rp = np.concatenate([g.row_ptr, np.full(extra, g.row_ptr[-1], np.int32)])
    return inputs.Graph(rp, g.col, g.w, g.name + "-iso")


_cache = {}


def graph(name):
    if name in _cache:
        return _cache[name]
    if name == "two-cliques-5":
        g = inputs.two_cliques(5)
    elif name == "two-cliques-10":
        g = inputs.two_cliques(10)
    elif name == "sbm1-s1":
        g = inputs.sbm1(1)
    elif name == "sbm1-s2-w":
        g = inputs.with_uniform_weights(inputs.sbm1(2), 7)
    elif name == "rmat12":
        g = inputs.rmat(12)
    elif name == "rmat14":
        g = inputs.rmat(14)
    elif name == "rmat14-w":
        g = inputs.with_uniform_weights(inputs.rmat(14), 24)
    elif name == "grid64":
        g = inputs.grid(64, 64, 0.05, 0.01, seed=9)
    elif name == "star5000":
        g = star(5000)
    elif name == "rmat10-selfloops":
        g = with_self_loops(inputs.rmat(10))
    elif name == "sbm1-iso":
        g = with_isolated(inputs.sbm1(3))
    else:
        raise KeyError(name)
    _cache[name] = g
    return g


GRAPHS = ["two-cliques-5", "two-cliques-10", "sbm1-s1", "sbm1-s2-w", "rmat12", "rmat14",
          "rmat14-w", "grid64", "star5000", "rmat10-selfloops", "sbm1-iso"]


def check_det(g, k, **kw):
    labels, it, dn, sc, q = gpu_run(g, k, "det", **kw)
    tol = kw.get("tol", 0.05)
    ok = oracle.BM_PAPER if kw.get("rule") == "bm_paper" else k
    ref, rit, rdn, rsc = oracle.lpa_run(g.row_ptr, g.col, g.w, k=ok, tol=tol,
                                        max_iter=kw.get("max_iter", 20), rho=kw.get("rho", 8),
                                        rescan=kw.get("rescan", False))
    assert it == rit, (g.name, k, it, rit)
    assert np.array_equal(dn, rdn), (g.name, k, dn, rdn)
    assert np.array_equal(sc, rsc), (g.name, k, sc, rsc)
    bad = np.nonzero(labels != ref)[0]
    assert bad.size == 0, (g.name, k, bad[:10], labels[bad[:10]], ref[bad[:10]])
    qr = oracle.modularity(g.row_ptr, g.col, g.w, ref)
    assert abs(q - qr) <= 1e-9, (q, qr)


@pytest.mark.parametrize("name", GRAPHS)
@pytest.mark.parametrize("k", KS)
def test_det_parity(name, k):
    check_det(graph(name), k)


@pytest.mark.parametrize("lane_max", [1, 8, 64, 1024])
def test_det_independent_of_bins(lane_max):
    check_det(graph("rmat14-w"), 8, lane_max_degree=lane_max)
    check_det(graph("star5000"), 4, lane_max_degree=lane_max)


@pytest.mark.parametrize("lane_max", [2, 3, 4, 5])
@pytest.mark.parametrize("k", [1, 8])
def test_det_short_rows_near_threshold(lane_max, k):
    # rows of up to 4 entries below the lane threshold run two per lane
    # without the stage: thresholds around that degree move vertices between
    # hubs, staged lane rows and short rows without changing any result
    check_det(graph("grid64"), k, lane_max_degree=lane_max)
    check_det(graph("rmat12"), k, lane_max_degree=lane_max)
    check_det(graph("rmat10-selfloops"), k, lane_max_degree=lane_max)


def test_det_first_iteration_from_restored_labels():
    # a state restored at iteration 0 is not the initial labelling: hub rows
    # then see repeated labels and must take the general chain (the first
    # iteration's shortcut for distinct labels would be wrong here)
    g = graph("rmat14")
    rng = np.random.default_rng(14)
    lab0 = rng.integers(0, 40, g.n).astype(np.int32)
    act0 = np.ones(g.n, np.uint8)
    rp, col, w = to_dev(g)
    for lane_max in (16, 0):
        s = lpa.LPA(rp, col, w, k=8, lane_max_degree=lane_max)
        s.set_state(lab0, act0, 0)
        s.step()
        got = s.labels(device=False)
        s.close()
        ref, _, _, _ = oracle.lpa_move(g.row_ptr, g.col, g.w, 8, True, lab0, act0)
        assert np.array_equal(got, ref), (lane_max, np.nonzero(got != ref)[0][:10])


@pytest.mark.parametrize("lane_max", [1, 8])
@pytest.mark.parametrize("k", [1, 4, 8, 16, 32])
def test_det_unit_weight_hub_chain(lane_max, k):
    # unit weights: hub rows add runs of hits to their slots as counts and
    # take full-sketch decrements of exactly 1; low thresholds send nearly
    # every vertex of these converging graphs through that chain, whose
    # later iterations are mostly hits
    check_det(graph("sbm1-s1"), k, lane_max_degree=lane_max)
    check_det(graph("rmat12"), k, lane_max_degree=lane_max)


def test_det_hub_rows_with_repeated_neighbours():
    # a multigraph: hub rows that name a neighbour several times keep the
    # general chain at iteration 0 (labels repeat within the row)
    base = star(3000)
    rows = [list(base.col[base.row_ptr[i]:base.row_ptr[i + 1]]) for i in range(base.n)]
    rows[0] = sorted(rows[0] + rows[0][::7])  # the hub repeats every 7th leaf
    for j in rows[0][::7]:
        rows[j] = sorted(rows[j] + [0])
    rp = np.zeros(base.n + 1, np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.array([c for r in rows for c in r], np.int32)
    rng = np.random.default_rng(3)
    w = rng.uniform(0.5, 1.0, len(col)).astype(np.float32)
    g = inputs.Graph(rp, col, w, "star3000-repeats")
    gu = inputs.Graph(rp, col, None, "star3000-repeats-unit")  # runs of hits as counts
    for k in (2, 8):
        check_det(g, k, lane_max_degree=64)
        check_det(gu, k, lane_max_degree=64)


def test_det_tolerances_and_limits():
    g = graph("sbm1-s1")
    check_det(g, 8, tol=0.0)
    check_det(g, 8, tol=1.0)
    check_det(g, 8, max_iter=1)
    check_det(g, 8, max_iter=0)
    check_det(g, 8, rho=0, max_iter=7)
    check_det(g, 8, rho=1)


def test_step_matches_run():
    g = graph("rmat14")
    rp, col, w = to_dev(g)
    s = lpa.LPA(rp, col, w, k=8)
    changed = []
    while True:
        ch, done = s.step()
        changed.append(ch)
        if done:
            break
    ch, done = s.step()
    assert ch == 0 and done
    labels = s.labels(device=False)
    s.close()
    ref, rit, rdn, _ = oracle.lpa_run(g.row_ptr, g.col, None, k=8)
    assert changed == rdn.tolist()
    assert np.array_equal(labels, ref)


def test_checkpoint_resume_bit_exact():
    g = graph("sbm1-s2-w")
    rp, col, w = to_dev(g)
    a = lpa.LPA(rp, col, w, k=8)
    for _ in range(3):
        a.step()
    lab, flags, it = a.get_state()
    assert it == 3
    b = lpa.LPA(rp, col, w, k=8)
    b.set_state(lab, flags, it)
    b.run()
    a.run()
    assert np.array_equal(a.labels(device=False), b.labels(device=False))
    ref, _, _, _ = oracle.lpa_run(g.row_ptr, g.col, g.w, k=8)
    assert np.array_equal(b.labels(device=False), ref)
    a.close()
    b.close()


def test_profile_marks_untimed_iterations():
    # iterations whose move kernel was not timed read -1, and reading them
    # leaves the handle usable (no HIP error from events never recorded)
    g = graph("rmat12")
    rp, col, w = to_dev(g)
    s = lpa.LPA(rp, col, w, k=8, max_iter=20)
    s.step()  # before profiling
    s.profile(True)
    s.step()
    s.step()
    ms = s.move_ms()
    assert len(ms) == 3 and ms[0] == -1.0 and ms[1] >= 0.0 and ms[2] >= 0.0
    lab, flags, it = s.get_state()
    s.set_state(lab, flags, it)  # restored at iteration 3: nothing timed yet
    assert (s.move_ms() == -1.0).all()
    s.run()
    ms = s.move_ms()
    assert (ms[:3] == -1.0).all() and (ms[3:] >= 0.0).all()
    s.reset()
    s.run()
    assert (s.move_ms() >= 0.0).all()
    s.close()


def test_reset_reproduces():
    g = graph("rmat12")
    rp, col, w = to_dev(g)
    s = lpa.LPA(rp, col, w, k=8)
    s.run()
    first = s.labels(device=False)
    s.reset()
    s.run()
    assert np.array_equal(first, s.labels(device=False))
    s.close()


def test_trivial_graphs():
    d = dev()
    # a single vertex, no edges
    g = inputs.Graph(np.array([0, 0], np.int32), np.zeros(0, np.int32), None, "one")
    labels, it, dn, sc, q = gpu_run(g, 8)
    ref, rit, _, _ = oracle.lpa_run(g.row_ptr, g.col, None, k=8)
    assert labels.tolist() == [0] and it == rit and q == 0.0
    # empty graph
    rp = torch.zeros(1, dtype=torch.int32, device=d)
    col = torch.zeros(0, dtype=torch.int32, device=d)
    s = lpa.LPA(rp, col, None, k=8)
    assert s.run() == 0
    assert s.modularity() == 0.0
    s.close()


def test_modularity_of_given_labels():
    g = graph("rmat14-w")
    rp, col, w = to_dev(g)
    s = lpa.LPA(rp, col, w, k=8)
    rng = np.random.default_rng(3)
    for lab in (np.zeros(g.n, np.int32), np.arange(g.n, dtype=np.int32),
                rng.integers(0, 50, g.n).astype(np.int32)):
        q = s.modularity(torch.from_numpy(lab).to(rp.device))
        assert abs(q - oracle.modularity(g.row_ptr, g.col, g.w, lab)) <= 1e-9
    bad = np.zeros(g.n, np.int32)
    bad[5] = g.n
    with pytest.raises(lpa.LpaError) as ei:
        s.modularity(torch.from_numpy(bad).to(rp.device))
    assert ei.value.code == lpa.LPA_ERR_GRAPH
    # the handle still works after the rejected call
    q = s.modularity(torch.from_numpy(np.zeros(g.n, np.int32)).to(rp.device))
    assert abs(q) < 1e-12
    s.close()


def test_invalid_graph_rejected():
    d = dev()
    g = inputs.rmat(8)
    col = g.col.copy()
    col[10] = g.n + 5  # out of range
    rp = torch.from_numpy(g.row_ptr).to(d)
    with pytest.raises(lpa.LpaError) as ei:
        lpa.LPA(rp, torch.from_numpy(col).to(d), None, k=8)
    assert ei.value.code == lpa.LPA_ERR_GRAPH
    w = np.ones(g.nnz, np.float32)
    w[3] = -1.0
    with pytest.raises(lpa.LpaError) as ei:
        lpa.LPA(rp, torch.from_numpy(g.col).to(d), torch.from_numpy(w).to(d), k=8)
    assert ei.value.code == lpa.LPA_ERR_GRAPH
    bad_rp = g.row_ptr.copy()
    bad_rp[5], bad_rp[6] = bad_rp[6] + 1, bad_rp[5]
    with pytest.raises(lpa.LpaError) as ei:
        lpa.LPA(torch.from_numpy(bad_rp).to(d), torch.from_numpy(g.col).to(d), None, k=8)
    assert ei.value.code == lpa.LPA_ERR_GRAPH


def test_set_state_rejects_bad_labels():
    g = graph("rmat12")
    rp, col, w = to_dev(g)
    s = lpa.LPA(rp, col, w, k=8)
    lab = np.arange(g.n, dtype=np.int32)
    lab[3] = -1
    with pytest.raises(lpa.LpaError) as ei:
        s.set_state(lab, np.ones(g.n, np.uint8), 0)
    assert ei.value.code == lpa.LPA_ERR_GRAPH
    s.close()


@pytest.mark.parametrize("k", [1, 8, 16])
def test_async_quality_and_validity(k):
    g = graph("sbm1-s1")
    labels, it, dn, sc, q = gpu_run(g, k, "async")
    assert 1 <= it <= 20
    assert labels.min() >= 0 and labels.max() < g.n
    q_exact = oracle.modularity(g.row_ptr, g.col, None,
                                oracle.lpa_run(g.row_ptr, g.col, None, k=0)[0])
    assert abs(q - oracle.modularity(g.row_ptr, g.col, None, labels)) <= 1e-9
    if k >= 8:
        assert q > 0.9 * q_exact, (q, q_exact)


# ---- the one-candidate vote of Algorithm 3 (LPA_RULE_BM_PAPER) ----------

BM_GRAPHS = GRAPHS + ["rmat16"]


@pytest.mark.parametrize("name", BM_GRAPHS)
def test_bm_paper_det_parity(name):
    if name == "rmat16" and name not in _cache:
        _cache[name] = inputs.with_uniform_weights(inputs.rmat(16), 16)
    check_det(graph(name), 1, rule="bm_paper")


@pytest.mark.parametrize("lane_max", [1, 5, 64])
def test_bm_paper_det_independent_of_bins(lane_max):
    # lane_max 1 sends every vertex of degree > 1 through the wavefront path
    check_det(graph("rmat14-w"), 1, rule="bm_paper", lane_max_degree=lane_max)


def test_bm_paper_differs_from_one_slot_sketch():
    # path 0-2-1: the vote moves vertex 2 in iteration 0, the sketch empties
    g = inputs.from_edges(3, [(0, 2), (1, 2)], name="path021")
    lab_bm = gpu_run(g, 1, "det", rule="bm_paper")[0]
    lab_mg = gpu_run(g, 1, "det")[0]
    assert lab_bm.tolist() == [1, 1, 1] and lab_mg.tolist() == [0, 1, 2]


@pytest.mark.parametrize("lane_max", [0, 64])
def test_bm_paper_async_validity(lane_max):
    g = graph("rmat14-w")
    labels, it, dn, sc, q = gpu_run(g, 1, "async", rule="bm_paper", lane_max_degree=lane_max)
    assert 1 <= it <= 20
    assert labels.min() >= 0 and labels.max() < g.n
    assert abs(q - oracle.modularity(g.row_ptr, g.col, g.w, labels)) <= 1e-9


def test_bm_paper_rejects_k():
    rp, col, w = to_dev(graph("two-cliques-5"))
    with pytest.raises(lpa.LpaError) as ei:
        lpa.LPA(rp, col, w, k=8, rule="bm_paper")
    assert ei.value.code == lpa.LPA_ERR_ARG


def test_bm_paper_batch():
    gs = [graph("sbm1-s1"), graph("rmat12"), graph("sbm1-s2-w"), graph("star5000")]
    solvers = []
    for g in gs:
        rp, col, w = to_dev(g)
        solvers.append(lpa.LPA(rp, col, w, k=1, rule="bm_paper"))
    batch = lpa.Batch(len(gs), k=1, rule="bm_paper")
    batch.run(solvers)
    for g, s in zip(gs, solvers):
        ref = oracle.lpa_run(g.row_ptr, g.col, g.w, k=oracle.BM_PAPER)[0]
        assert np.array_equal(s.labels(device=False), ref), g.name
    # a sketch handle cannot join a batch of the vote, nor the reverse
    rp, col, w = to_dev(gs[0])
    mg = lpa.LPA(rp, col, w, k=1)
    with pytest.raises(lpa.LpaError):
        batch.run([mg])
    mg_batch = lpa.Batch(2, k=1)
    with pytest.raises(lpa.LpaError):
        mg_batch.run([solvers[0]])
    for x in solvers + [mg, batch, mg_batch]:
        x.close()


# ---- the double scan (LPA_RESCAN, Section 4.4 / Algorithm 4) --------------

@pytest.mark.parametrize("name", GRAPHS)
@pytest.mark.parametrize("k", [1, 2, 8])
def test_rescan_det_parity(name, k):
    check_det(graph(name), k, rescan=True)


@pytest.mark.parametrize("lane_max", [1, 64])
def test_rescan_det_independent_of_bins(lane_max):
    # lane_max 1 sends every vertex of degree > 1 through the wavefront path
    check_det(graph("rmat14-w"), 8, rescan=True, lane_max_degree=lane_max)


@pytest.mark.parametrize("lane_max", [0, 64])
def test_rescan_async_quality_and_validity(lane_max):
    # lane_max 64 splits every vertex above 64 into hub segments, so the
    # segment re-weighting and hub decision kernels run on many hubs
    for name in ("sbm1-s1", "rmat14-w"):
        g = graph(name)
        labels, it, dn, sc, q = gpu_run(g, 8, "async", rescan=True, lane_max_degree=lane_max)
        assert 1 <= it <= 20
        assert labels.min() >= 0 and labels.max() < g.n
        assert abs(q - oracle.modularity(g.row_ptr, g.col, g.w, labels)) <= 1e-9
        if name == "sbm1-s1":
            q_exact = oracle.modularity(g.row_ptr, g.col, None,
                                        oracle.lpa_run(g.row_ptr, g.col, None, k=0)[0])
            assert q > 0.9 * q_exact, (q, q_exact)


def test_rescan_batch_and_rejections():
    gs = [graph("sbm1-s1"), graph("rmat12"), graph("star5000")]
    solvers = []
    for g in gs:
        rp, col, w = to_dev(g)
        solvers.append(lpa.LPA(rp, col, w, k=4, rescan=True))
    batch = lpa.Batch(len(gs), k=4, rescan=True)
    batch.run(solvers)
    for g, s in zip(gs, solvers):
        ref = oracle.lpa_run(g.row_ptr, g.col, g.w, k=4, rescan=True)[0]
        assert np.array_equal(s.labels(device=False), ref), g.name
    rp, col, w = to_dev(gs[0])
    single = lpa.LPA(rp, col, w, k=4)
    with pytest.raises(lpa.LpaError):
        batch.run([single])
    with pytest.raises(lpa.LpaError) as ei:
        lpa.LPA(rp, col, w, k=1, rule="bm_paper", rescan=True)
    assert ei.value.code == lpa.LPA_ERR_ARG
    for x in solvers + [single, batch]:
        x.close()


# ---- one shared sketch per hub (LPA_HUB_SHARED, ablation of Section 4.3) --

@pytest.mark.parametrize("lane_max", [0, 64])
def test_hub_shared_validity(lane_max):
    # lane_max 64 sends every vertex above 64 through the shared-sketch
    # workgroups; results race, so check validity, counters and quality
    for name in ("rmat14-w", "sbm1-s1", "star5000"):
        g = graph(name)
        rp, col, w = to_dev(g)
        s = lpa.LPA(rp, col, w, k=8, mode="async", hub_shared=True, lane_max_degree=lane_max)
        it = s.run()
        lab = s.labels(device=False)
        assert 1 <= it <= 20
        assert lab.min() >= 0 and lab.max() < g.n
        dn, sc = s.trace()
        assert sc[0] == g.nnz  # every entry scanned once in the first iteration
        q = s.modularity()
        assert abs(q - oracle.modularity(g.row_ptr, g.col, g.w, lab)) <= 1e-9
        if name == "sbm1-s1":
            q_exact = oracle.modularity(g.row_ptr, g.col, None,
                                        oracle.lpa_run(g.row_ptr, g.col, None, k=0)[0])
            assert q > 0.9 * q_exact, (q, q_exact)
        s.close()
    with pytest.raises(lpa.LpaError):
        rp, col, w = to_dev(graph("sbm1-s1"))
        lpa.LPA(rp, col, w, k=8, mode="det", hub_shared=True)


# ---- shared variables instead of votes (LPA_SHARED_VARS, Section 4.1) ----

@pytest.mark.parametrize("name", ["two-cliques-10", "sbm1-s2-w", "rmat14-w", "star5000",
                                  "rmat10-selfloops", "sbm1-iso"])
@pytest.mark.parametrize("k", KS)
@pytest.mark.parametrize("lane_max", [0, 1, 16])
def test_shared_vars_det_parity(name, k, lane_max):
    # lane_max 1 and 16 send (nearly) every vertex through the
    # one-wavefront-per-vertex path whose lanes talk through LDS variables
    check_det(graph(name), k, lane_max_degree=lane_max, shared_vars=True)


def test_shared_vars_batch_and_rejections():
    gs = [graph("sbm1-s1"), graph("rmat14-w"), graph("star5000")]
    solvers = []
    for g in gs:
        rp, col, w = to_dev(g)
        solvers.append(lpa.LPA(rp, col, w, k=8, shared_vars=True, lane_max_degree=16))
    batch = lpa.Batch(len(gs), k=8, shared_vars=True)
    batch.run(solvers)
    for g, s in zip(gs, solvers):
        assert np.array_equal(s.labels(device=False), oracle.lpa_run(g.row_ptr, g.col, g.w, k=8)[0])
    rp, col, w = to_dev(gs[0])
    plain = lpa.LPA(rp, col, w, k=8)
    with pytest.raises(lpa.LpaError):
        batch.run([plain])  # a handle without the flag cannot join
    for kw in (dict(mode="async"), dict(rescan=True), dict(k=1, rule="bm_paper")):
        args = dict(k=8, shared_vars=True)
        args.update(kw)
        with pytest.raises(lpa.LpaError) as ei:
            lpa.LPA(rp, col, w, **args)
        assert ei.value.code == lpa.LPA_ERR_ARG
    for x in solvers + [plain, batch]:
        x.close()
