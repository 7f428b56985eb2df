"""Async hub path against the oracle's partial-sketch choice.

On a graph where every vertex is a hub (degree above the lane threshold S),
LPA_MODE_ASYNC labels change only in the hub merge, after every segment of
the iteration has been scanned, so each iteration is a synchronous update
and can be checked exactly: every active vertex takes the label the oracle
computes from its row's S-entry segments (partial sketches merged in
segment order, Section 4.3), under the pick-less rule of that iteration.
Per iteration the labels, the number of changed vertices and the
unprocessed flags (exactly the neighbours of the vertices that moved) must
match.  Hubs here have at most 64 segments, the partial count the merge
feeds one by one.
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


def all_hub_graph(n=1200, block=60, extra=18, seed=11):
    """Ring lattice (every vertex joined to the 5 next ones, so degree >= 10
    > S) plus random edges inside blocks of `block` vertices; uniform
    (0, 1] weights."""
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
    g = inputs.from_edges(n, sorted(edges), name="allhub")
    return inputs.with_uniform_weights(g, seed)


_g = {}


def graph():
    if "g" not in _g:
        _g["g"] = all_hub_graph()
    return _g["g"]


def test_every_vertex_is_a_hub_with_few_segments():
    d = np.diff(graph().row_ptr)
    assert d.min() > S and int(np.ceil(d.max() / S)) <= 64


@pytest.mark.parametrize("k", [1, 4, 8, 16])
def test_async_hub_iterations_match_partial_sketch_oracle(k):
    g = graph()
    rp, col, w = to_dev(g)
    s = lpa.LPA(rp, col, w, k=k, mode="async", lane_max_degree=S, rho=RHO)
    for _ in range(4):
        C, act, l = s.get_state()
        changed, done = s.step()
        C2, act2, _ = s.get_state()
        pickless = RHO > 0 and l % RHO == 0
        expect = C.copy()
        for v in np.nonzero(act)[0]:
            c = oracle.hub_segment_choice(g.row_ptr, g.col, g.w, k, S, C, int(v))
            if c != C[v] and (not pickless or c < C[v]):
                expect[v] = c
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
    s.close()
