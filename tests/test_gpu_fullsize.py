"""Parity at the benchmark sizes.

* R-MAT scale 22 (128M CSR entries), det mode: every iteration is checked in
  full against the oracle's one-iteration function from the same state —
  labels, next flags and changed count, bit for bit (k = 8); whole runs
  against the oracle's whole run for the other sketch sizes of the k sweep
  (k = 1, 4, 16), the vote of Algorithm 3 and the double scan.
* R-MAT scale 24 (0.52B entries, weights uniform in (0, 1]), det mode: the
  whole run against the oracle's whole run (labels, iterations, changed and
  scanned counts of every iteration).
* Modularity of the asynchronous run on R-MAT scale 24 (the benchmark
  configuration) against the oracle's fp64 modularity of the same labels.
* The 4096 x 4096 rewired grid, det mode, whole run.
* The ranked state layout: R-MAT scale 22 det whole run against the oracle,
  R-MAT scale 24 async modularity.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2411_19901_amd import inputs, lpa  # noqa: E402

pytestmark = pytest.mark.gpu

_graphs = {}


def graph(scale, weighted):
    key = (scale, weighted)
    if key not in _graphs:
        g = inputs.rmat(scale)
        _graphs[key] = inputs.with_uniform_weights(g, scale) if weighted else g
    return _graphs[key]


def solver(g, **kw):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    return lpa.LPA(torch.from_numpy(g.row_ptr).to(d), torch.from_numpy(g.col).to(d),
                   torch.from_numpy(g.w).to(d) if g.w is not None else None, **kw)


@pytest.mark.timeout(600)
def test_rmat22_det_every_iteration_exact():
    g = graph(22, False)
    s = solver(g, k=8, mode="det")
    deg = g.degrees()
    for it in range(20):
        C, act, l = s.get_state()
        ch, done = s.step()
        C2, act2, l2 = s.get_state()
        pl = l % 8 == 0
        Cr, actr, dnr, scr = oracle.lpa_move(g.row_ptr, g.col, None, 8, pl, C, act)
        assert ch == dnr, (l, ch, dnr)
        assert np.array_equal(C2, Cr), l
        nz = deg > 0  # flags of isolated vertices are unspecified
        assert np.array_equal(act2[nz] != 0, actr[nz] != 0), l
        dn, sc = s.trace()
        assert sc[l] == scr
        if done:
            break
    q = s.modularity()
    assert abs(q - oracle.modularity(g.row_ptr, g.col, None, s.labels(device=False))) <= 1e-9
    s.close()


def whole_run_exact(g, k, **kw):
    s = solver(g, k=k, mode="det", **kw)
    it = s.run()
    ref, rit, rdn, rsc = oracle.lpa_run(g.row_ptr, g.col, g.w, k=k, rescan=kw.get("rescan", False))
    assert it == rit, (it, rit)
    dn, sc = s.trace()
    assert np.array_equal(dn, rdn) and np.array_equal(sc, rsc), (dn, rdn, sc, rsc)
    lab = s.labels(device=False)
    bad = np.nonzero(lab != ref)[0]
    assert bad.size == 0, (bad.size, bad[:5], lab[bad[:5]], ref[bad[:5]])
    q = s.modularity()
    assert abs(q - oracle.modularity(g.row_ptr, g.col, g.w, ref)) <= 1e-9
    s.close()
    return it


@pytest.mark.timeout(600)
@pytest.mark.parametrize("k", [1, 4, 16])
def test_rmat22_det_whole_run_k_sweep(k):
    it = whole_run_exact(graph(22, False), k)
    print(f"rmat22 det k={k}: {it} iterations equal to the oracle")


@pytest.mark.timeout(600)
def test_rmat22_ranked_det_whole_run():
    # the ranked state layout at full size: same run as the default layout
    it = whole_run_exact(graph(22, False), 8, ranked=True)
    print(f"rmat22 det k=8 ranked: {it} iterations equal to the oracle")


@pytest.mark.timeout(600)
def test_rmat24_ranked_async_modularity_parity():
    g = graph(24, True)
    s = solver(g, k=8, mode="async", ranked=True)
    it = s.run()
    assert 1 <= it <= 20
    lab = s.labels(device=False)
    assert lab.min() >= 0 and lab.max() < g.n
    assert abs(s.modularity() - oracle.modularity(g.row_ptr, g.col, g.w, lab)) <= 1e-9
    s.close()


@pytest.mark.timeout(900)
def test_rmat24_det_whole_run():
    it = whole_run_exact(graph(24, True), 8)
    print(f"rmat24 det k=8: {it} iterations equal to the oracle")


@pytest.mark.timeout(600)
def test_rmat24_async_modularity_parity():
    g = graph(24, True)
    s = solver(g, k=8, mode="async")
    it = s.run()
    assert 1 <= it <= 20
    lab = s.labels(device=False)
    assert lab.min() >= 0 and lab.max() < g.n
    q = s.modularity()
    assert abs(q - oracle.modularity(g.row_ptr, g.col, g.w, lab)) <= 1e-9
    s.close()


@pytest.mark.timeout(600)
def test_grid4096_det_exact():
    # the road-network stand-in at full size (16.8M vertices, 63.7M entries):
    # whole det run against the oracle's whole run
    g = inputs.grid(4096, 4096, 0.05, 0.01, seed=4096)
    s = solver(g, k=8, mode="det")
    it = s.run()
    ref, rit, rdn, rsc = oracle.lpa_run(g.row_ptr, g.col, None, k=8)
    assert it == rit
    dn, sc = s.trace()
    assert np.array_equal(dn, rdn) and np.array_equal(sc, rsc)
    assert np.array_equal(s.labels(device=False), ref)
    assert abs(s.modularity() - oracle.modularity(g.row_ptr, g.col, None, ref)) <= 1e-9
    s.close()


@pytest.mark.timeout(600)
def test_rmat22_bm_paper_det_exact():
    # the vote of Algorithm 3 at full size, whole run against the oracle
    g = graph(22, False)
    s = solver(g, k=1, mode="det", rule="bm_paper")
    it = s.run()
    ref, rit, rdn, rsc = oracle.lpa_run(g.row_ptr, g.col, None, k=oracle.BM_PAPER)
    assert it == rit
    dn, sc = s.trace()
    assert np.array_equal(dn, rdn) and np.array_equal(sc, rsc)
    assert np.array_equal(s.labels(device=False), ref)
    s.close()


@pytest.mark.timeout(600)
def test_rmat22_rescan_det_exact():
    # the double scan at full size, whole det run against the oracle
    g = graph(22, False)
    s = solver(g, k=8, mode="det", rescan=True)
    it = s.run()
    ref, rit, rdn, rsc = oracle.lpa_run(g.row_ptr, g.col, None, k=8, rescan=True)
    assert it == rit
    dn, sc = s.trace()
    assert np.array_equal(dn, rdn) and np.array_equal(sc, rsc)
    assert np.array_equal(s.labels(device=False), ref)
    s.close()
