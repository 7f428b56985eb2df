"""Neighbour marking for graphs of short rows.

A changed vertex flags its neighbours as unprocessed for the next iteration
(pruning, Section 4.6).  Wavefronts whose rows all fit one staging step of 4
or 8 entries mark from the column indices kept in the LDS stage; rows of 5,
9 or more entries take the other widths or the path that reads the row
again.  Graphs with every degree capped at 3, 4, 5, 8, 9 or 16 (most
vertices at the cap, so wavefronts sit on each side of those widths) must
give the oracle's labels, iteration count and per-iteration changed and
scanned counts bit for bit in det mode: a missed or extra mark changes what
the next iteration scans.  Async runs are checked for valid labels and for
modularity equal to the oracle's on the same labels.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2411_19901_amd import inputs, lpa  # noqa: E402
from test_gpu_parity import check_det, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu

CAPS = [3, 4, 5, 8, 9, 16]
N = 20_000  # 313 wavefronts of lane vertices, the last one ragged


def capped(cap, n=N, block=40, p_in=0.85, seed=None):
    """Block-structured random graph with every degree at most `cap`: edges
    drawn mostly inside blocks of `block` vertices and kept while both ends
    are below the cap; uniform (0, 1] weights."""
    seed = 1000 + cap if seed is None else seed
    rng = np.random.default_rng(seed)
    m = n * cap
    u = rng.integers(0, n, m)
    inside = rng.random(m) < p_in
    v = np.where(inside, (u // block) * block + rng.integers(0, block, m), rng.integers(0, n, m))
    v = np.minimum(v, n - 1)
    deg = [0] * n
    edges = set()
    for a, b in zip(u.tolist(), v.tolist()):
        if a == b or deg[a] >= cap or deg[b] >= cap:
            continue
        key = (a, b) if a < b else (b, a)
        if key in edges:
            continue
        edges.add(key)
        deg[a] += 1
        deg[b] += 1
    g = inputs.from_edges(n, sorted(edges), name=f"cap{cap}")
    return inputs.with_uniform_weights(g, seed)


_cache = {}


def graph(cap):
    if cap not in _cache:
        _cache[cap] = capped(cap)
    return _cache[cap]


@pytest.mark.parametrize("cap", CAPS)
def test_graphs_sit_on_the_widths(cap):
    d = np.diff(graph(cap).row_ptr)
    assert d.max() == cap and (d == cap).mean() > 0.5, (cap, np.bincount(d))


@pytest.mark.parametrize("cap", CAPS)
@pytest.mark.parametrize("k", [1, 4, 8, 16, 32])
def test_det_parity_short_rows(cap, k):
    check_det(graph(cap), k)


@pytest.mark.parametrize("cap", CAPS)
def test_det_parity_short_rows_vote(cap):
    check_det(graph(cap), 1, rule="bm_paper")


@pytest.mark.parametrize("cap", [4, 8, 9])
def test_det_parity_short_rows_rescan(cap):
    check_det(graph(cap), 8, rescan=True)


@pytest.mark.parametrize("cap", CAPS)
def test_det_parity_short_rows_no_pickless(cap):
    # rho = 0: every iteration may move to any label, so more vertices move
    # (and mark) in iteration 0
    check_det(graph(cap), 8, rho=0)


@pytest.mark.parametrize("cap", CAPS)
@pytest.mark.parametrize("k", [8, 32])
def test_async_short_rows(cap, k):
    g = graph(cap)
    rp, col, w = to_dev(g)
    s = lpa.LPA(rp, col, w, k=k, mode="async")
    it = s.run()
    lab = s.labels(device=False)
    dn, sc = s.trace()
    assert 1 <= it <= 20 and lab.min() >= 0 and lab.max() < g.n
    assert sc[0] == g.nnz and all(0 <= x <= g.nnz for x in sc)
    assert dn[0] > 0
    assert abs(s.modularity() - oracle.modularity(g.row_ptr, g.col, g.w, lab)) <= 1e-9
    s.close()
