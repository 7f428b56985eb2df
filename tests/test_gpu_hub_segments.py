"""Async hub path against the oracle's partial-sketch choice.

On a graph where every vertex is a hub (degree above the lane threshold S),
LPA_MODE_ASYNC labels change only in the hub merge, after every segment of
the iteration has been scanned, so each iteration is a synchronous update
and can be checked exactly: every active vertex takes the label the oracle
computes from its row's S-entry segments (partial sketches merged as
Section 4.3 describes, in the order of reading R9: up to 64 partials in
segment order into one sketch, more through 64 chains combined pairwise),
under the pick-less rule of that iteration.  Per iteration the labels, the
number of changed vertices and the unprocessed flags (exactly the
neighbours of the vertices that moved) must match.

Two graphs: one whose hubs have at most 64 segments and one whose hubs have
65 to about 400; uniform (0, 1] weights and unit weights (ties and
decrements everywhere, which is where the order of the slots matters); the
double scan (Section 4.4) on unit weights, whose fp32 sums are exact in any
order.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2411_19901_amd import inputs, lpa  # noqa: E402
from test_gpu_parity import to_dev  # noqa: E402

pytestmark = pytest.mark.gpu

S = 8
RHO = 8


def narrow_graph(n=1200, block=60, extra=18, seed=11):
    """Ring lattice (every vertex joined to the 5 next ones, so degree >= 10
    > S) plus random edges inside blocks of `block` vertices."""
    rng = np.random.default_rng(seed)
    edges = set()
    for i in range(n):
        for j in range(1, 6):
            a, b = i, (i + j) % n
            edges.add((min(a, b), max(a, b)))
    u = rng.integers(0, n, n * extra)
    v = (u // block) * block + rng.integers(0, block, n * extra)
    v = np.minimum(v, n - 1)
    for a, b in zip(u.tolist(), v.tolist()):
        if a != b:
            edges.add((min(a, b), max(a, b)))
    return inputs.from_edges(n, sorted(edges), name="allhub")


def wide_graph(n=3300, seed=12):
    """Chung-Lu graph with expected degrees uniform in [600, 3000] and a
    planted bias inside blocks of 100 vertices: every row has more than
    64 x S entries."""
    rng = np.random.default_rng(seed)
    d = rng.uniform(600, 3000, n)
    p = np.minimum(1.0, np.outer(d, d) / d.sum())
    blk = np.arange(n) // 100
    p = np.where(blk[:, None] == blk[None, :], np.minimum(1.0, 3 * p), p)
    a = np.triu(rng.random((n, n)) < p, 1)
    iu, ju = np.nonzero(a)
    return inputs.from_edges(n, list(zip(iu.tolist(), ju.tolist())), name="allhub-wide")


_g = {}


def graph(kind, weights):
    key = (kind, weights)
    if key not in _g:
        if kind not in _g:
            _g[kind] = narrow_graph() if kind == "narrow" else wide_graph()
        g = _g[kind]
        _g[key] = inputs.with_uniform_weights(g, 11) if weights == "uniform" else g
    return _g[key]


def test_every_vertex_is_a_hub():
    d = np.diff(graph("narrow", "unit").row_ptr)
    assert d.min() > S and int(np.ceil(d.max() / S)) <= 64
    d = np.diff(graph("wide", "unit").row_ptr)
    assert d.min() > 64 * S
    segs = np.ceil(d / S)
    assert segs.min() > 64 and segs.max() >= 300


def run_and_check(g, k, rescan, iters=4, ranked=False):
    rp, col, w = to_dev(g)
    s = lpa.LPA(rp, col, w, k=k, mode="async", lane_max_degree=S, rho=RHO, rescan=rescan,
                ranked=ranked)
    try:
        for _ in range(iters):
            C, act, l = s.get_state()
            changed, done = s.step()
            C2, act2, _ = s.get_state()
            pickless = RHO > 0 and l % RHO == 0
            expect = C.copy()
            verts = np.nonzero(act)[0].astype(np.int32)
            expect[verts] = oracle.hub_choose(g.row_ptr, g.col, g.w, k, S, pickless, C, verts,
                                              rescan=rescan)
            bad = np.nonzero(C2 != expect)[0]
            assert bad.size == 0, (k, l, bad[:10], C2[bad[:10]], expect[bad[:10]])
            moved = np.nonzero(expect != C)[0]
            assert changed == moved.size, (k, l, changed, moved.size)
            flags = np.zeros(g.n, bool)
            for v in moved:
                flags[g.col[g.row_ptr[v]:g.row_ptr[v + 1]]] = True
            assert np.array_equal(act2 != 0, flags), (k, l)
            if done:
                break
    finally:
        s.close()


@pytest.mark.parametrize("weights", ["uniform", "unit"])
@pytest.mark.parametrize("k", [1, 2, 4, 8, 16])
def test_narrow_hubs_match_partial_sketch_oracle(k, weights):
    run_and_check(graph("narrow", weights), k, rescan=False)


@pytest.mark.parametrize("weights", ["uniform", "unit"])
@pytest.mark.parametrize("k", [1, 2, 4, 8, 16])
def test_wide_hubs_match_partial_sketch_oracle(k, weights):
    run_and_check(graph("wide", weights), k, rescan=False)


@pytest.mark.parametrize("kind", ["narrow", "wide"])
@pytest.mark.parametrize("k", [2, 8])
def test_double_scan_hubs_match_oracle(kind, k):
    run_and_check(graph(kind, "unit"), k, rescan=True)
