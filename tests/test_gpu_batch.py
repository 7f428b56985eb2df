"""GPU tests of the batched launch: many graphs iterate with one set of
kernel launches per iteration and each ends exactly as its own solo run (and
the CPU oracle) in LPA_MODE_DET, also when graphs join a running batch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2411_19901_amd import inputs, lpa  # noqa: E402

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def mixed_graphs(count=20, seed=77, weighted_every=3):
    specs = inputs.batch_specs(count, seed, n_lo=150, n_hi=6000)
    gs = [inputs.batch_graph(s, seed, i) for i, s in enumerate(specs)]
    gs = [inputs.with_uniform_weights(g, i) if i % weighted_every == 0 else g for i, g in enumerate(gs)]
    gs.append(inputs.two_cliques(5))
    gs.append(inputs.Graph(np.array([0, 0, 0], np.int32), np.zeros(0, np.int32), None, "iso2"))
    gs.append(inputs.rmat(10))
    return gs


def make_solver(g, k=8, mode="det", **kw):
    d = dev()
    rp = torch.from_numpy(g.row_ptr).to(d)
    col = torch.from_numpy(g.col).to(d)
    w = torch.from_numpy(g.w).to(d) if g.w is not None else None
    return lpa.LPA(rp, col, w, k=k, mode=mode, **kw)


def oracle_labels(g, k=8):
    return oracle.lpa_run(g.row_ptr, g.col, g.w, k=k)


@pytest.mark.parametrize("k", [1, 8])
def test_batch_run_matches_oracle_and_solo(k):
    gs = mixed_graphs()
    solvers = [make_solver(g, k=k) for g in gs]
    batch = lpa.Batch(len(solvers), k=k, mode="det")
    batch.run(solvers)
    solo = [make_solver(g, k=k) for g in gs]
    for g, s, t in zip(gs, solvers, solo):
        t.run()
        ref, rit, rdn, rsc = oracle_labels(g, k)
        lab = s.labels(device=False)
        assert np.array_equal(lab, ref), g.name
        assert np.array_equal(lab, t.labels(device=False)), g.name
        dn, sc = s.trace()
        assert np.array_equal(dn, rdn) and np.array_equal(sc, rsc), g.name
        if g.n:
            assert abs(s.modularity() - oracle.modularity(g.row_ptr, g.col, g.w, ref)) <= 1e-9
    batch.close()
    for s in solvers + solo:
        s.close()


def test_continuous_batching_join_midway():
    gs = mixed_graphs(count=12, seed=5)
    solvers = [make_solver(g) for g in gs]
    batch = lpa.Batch(len(solvers), k=8, mode="det")
    first, rest = solvers[:5], solvers[5:]
    for _ in range(3):
        batch.step(first)
    resident = list(first) + list(rest)
    done = False
    steps = 0
    while not done:
        _, done = batch.step(resident)
        steps += 1
        assert steps <= 40
    for g, s in zip(gs, solvers):
        ref = oracle_labels(g)[0]
        assert np.array_equal(s.labels(device=False), ref), g.name
    batch.close()
    for s in solvers:
        s.close()


def test_batch_async_valid():
    gs = mixed_graphs(count=10, seed=9)
    solvers = [make_solver(g, mode="async") for g in gs]
    batch = lpa.Batch(len(solvers), k=8, mode="async")
    it = batch.run(solvers)
    assert 1 <= it <= 20
    for g, s in zip(gs, solvers):
        lab = s.labels(device=False)
        if g.n:
            assert lab.min() >= 0 and lab.max() < g.n
    batch.close()
    for s in solvers:
        s.close()


def test_batch_rejects_mismatched_handles():
    gs = mixed_graphs(count=2, seed=3)
    a = make_solver(gs[0], k=8)
    b = make_solver(gs[1], k=4)
    batch = lpa.Batch(4, k=8, mode="det")
    with pytest.raises(lpa.LpaError) as ei:
        batch.run([a, b])
    assert ei.value.code == lpa.LPA_ERR_ARG
    with pytest.raises(lpa.LpaError):
        batch.run([a, a])
    small = lpa.Batch(1, k=8, mode="det")
    with pytest.raises(lpa.LpaError):
        small.run([a, make_solver(gs[1], k=8)])
    for x in (batch, small, a, b):
        x.close()


@pytest.mark.parametrize("mode", ["det", "async"])
def test_workspace_handles(mode):
    g = inputs.with_uniform_weights(inputs.rmat(12), 3)
    nbytes = lpa.workspace_bytes(g.n, g.nnz, k=8, mode=mode)
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev())
    s = make_solver(g, mode=mode, workspace=ws)
    assert s.memory()[0] == nbytes
    s.run()
    if mode == "det":
        assert np.array_equal(s.labels(device=False), oracle_labels(g)[0])
    s.close()
    too_small = torch.empty(nbytes - 512, dtype=torch.uint8, device=dev())
    with pytest.raises(lpa.LpaError) as ei:
        make_solver(g, mode=mode, workspace=too_small)
    assert ei.value.code == lpa.LPA_ERR_NOMEM


def test_batch_reset_equals_reset():
    gs = mixed_graphs(count=10, seed=41)
    solvers = [make_solver(g) for g in gs]
    batch = lpa.Batch(len(solvers), k=8, mode="det")
    batch.run(solvers)
    ref = [s.labels(device=False) for s in solvers]
    for rep in range(2):
        batch.reset(solvers)
        for g, s in zip(gs, solvers):  # back to the initial state
            C, act, it = s.get_state()
            assert it == 0 and np.array_equal(C, np.arange(g.n, dtype=np.int32))
            assert g.n == 0 or act.min() == 1
            dn, sc = s.trace()
            assert len(dn) == 0
        batch.run(solvers)
        for g, s, r in zip(gs, solvers, ref):
            assert np.array_equal(s.labels(device=False), r), g.name
            dn, sc = s.trace()
            assert np.array_equal(dn, oracle_labels(g)[2]), g.name
    batch.close()
    for s in solvers:
        s.close()


_big = {}


def batch512():
    """The many-graph workload at full size: 512 planted-partition graphs
    (seed 512, n log-uniform in [1e3, 2e5]; 21.7M vertices, 304M entries),
    with the oracle's whole run of each."""
    if not _big:
        specs = inputs.batch_specs(512, 512)
        gs = [inputs.batch_graph(s, 512, i) for i, s in enumerate(specs)]
        _big["gs"] = gs
        _big["refs"] = [oracle.lpa_run(g.row_ptr, g.col, None, k=8) for g in gs]
    return _big["gs"], _big["refs"]


@pytest.mark.timeout(900)
@pytest.mark.parametrize("capture", [False, True])
def test_batch512_every_graph_matches_oracle(capture):
    gs, refs = batch512()
    d = dev()
    stream = torch.cuda.current_stream(d)
    solvers = [make_solver(g, stream=stream) for g in gs]
    batch = lpa.Batch(len(solvers), k=8, mode="det", stream=stream, capture=capture)
    for rep in range(2):  # a second batched solve from a one-launch reset
        batch.reset(solvers)
        batch.run(solvers)
        for g, s, (ref, rit, rdn, rsc) in zip(gs, solvers, refs):
            assert s.iterations() == rit, (g.name, rep)
            dn, sc = s.trace()
            assert np.array_equal(dn, rdn) and np.array_equal(sc, rsc), (g.name, rep)
            assert np.array_equal(s.labels(device=False), ref), (g.name, rep)
    batch.close()
    for s in solvers:
        s.close()
