"""The seeded generators produce valid symmetric CSR graphs, deterministically."""
import numpy as np
import pytest


def check_csr(g):
    rp, col = g.row_ptr, g.col
    assert rp.dtype == np.int32 and col.dtype == np.int32
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == len(col)
    n = g.n
    if len(col):
        assert col.min() >= 0 and col.max() < n
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    assert not np.any(src == col), "self-loop"
    # sorted, no duplicates inside each row
    same_row = src[1:] == src[:-1]
    assert np.all(col[1:][same_row] > col[:-1][same_row])
    # symmetric: the sorted (src, dst) set equals the sorted (dst, src) set
    a = src * n + col
    b = col.astype(np.int64) * n + src
    assert np.array_equal(np.sort(a), np.sort(b))
    if g.w is not None:
        order_a, order_b = np.argsort(a), np.argsort(b)
        assert np.array_equal(g.w[order_a], g.w[order_b]), "weights not symmetric"
        assert np.all(g.w > 0) and np.all(g.w <= 1)


def test_sbm1(gen):
    g = gen.sbm1(1)
    check_csr(g)
    assert g.n == 10_000 and 100_000 < g.nnz < 120_000
    g2 = gen.sbm1(1)
    assert np.array_equal(g.col, g2.col)
    assert not np.array_equal(gen.sbm1(2).col[:1000], g.col[:1000])
    # mostly intra-block edges: expected 9.95 intra vs 1.0 inter per vertex
    src = np.repeat(np.arange(g.n), g.degrees())
    intra = np.mean(src // 200 == g.col // 200)
    assert 0.85 < intra < 0.95


def test_rmat_small(gen):
    g = gen.rmat(12)
    check_csr(g)
    assert g.n == 4096
    assert np.array_equal(gen.rmat(12).col, g.col)
    deg = g.degrees()
    assert deg.max() > 20 * deg.mean()  # skewed
    gw = gen.with_uniform_weights(g, 24)
    check_csr(gw)
    # exact multiples of 2^-24
    assert np.all((gw.w.astype(np.float64) * 2**24) % 1 == 0)


def test_grid_small(gen):
    g = gen.grid(64, 64, 0.05, 0.01, seed=3)
    check_csr(g)
    full = 2 * (64 * 63 * 2)
    assert 0.9 * full < g.nnz < full


def test_batch_specs(gen):
    specs = gen.batch_specs(512, 512)
    ns = np.array([s.n for s in specs])
    assert ns.min() >= 1000 and ns.max() <= 200_000
    assert 20_000 < ns.mean() < 60_000
    assert all(1 <= s.blocks <= max(1, s.n // 16) for s in specs)
    g = gen.batch_graph(specs[0], 512, 0)
    check_csr(g)
    assert g.n == specs[0].n


def test_two_cliques(gen):
    g = gen.two_cliques(4)
    check_csr(g)
    assert g.nnz == 2 * (4 * 3 + 1)


def test_permuted_is_isomorphic():
    from paper_2411_19901_amd import inputs
    g = inputs.with_uniform_weights(inputs.rmat(10), 3)
    h = inputs.permuted(g, 7)
    assert h.n == g.n and h.nnz == g.nnz
    assert np.all(np.diff(h.row_ptr) >= 0)
    # rows sorted, symmetric, degree multiset and weight multiset kept
    for i in range(h.n):
        r = h.col[h.row_ptr[i]:h.row_ptr[i + 1]]
        assert np.all(np.diff(r) > 0)
    assert sorted(np.diff(g.row_ptr)) == sorted(np.diff(h.row_ptr))
    assert np.array_equal(np.sort(g.w), np.sort(h.w))
    edges = {(i, int(j)): float(x) for i in range(h.n)
             for j, x in zip(h.col[h.row_ptr[i]:h.row_ptr[i + 1]], h.w[h.row_ptr[i]:h.row_ptr[i + 1]])}
    assert all(edges[(j, i)] == x for (i, j), x in edges.items())


def test_ring_hubs_closed_form():
    """The device builder (run here with torch on the CPU) and the per-row
    recomputation give the same CSR, which is symmetric with matching
    weights, has the stated degrees and no self-loops or duplicates."""
    torch = pytest.importorskip("torch")
    from paper_2411_19901_amd import inputs
    L, H, r, seed = 1500, 9, 4, 11
    rp, col, w = inputs.ring_hubs_device(L, H, r, seed, "cpu", chunk=256)
    rp, col, w = rp.numpy(), col.numpy(), w.numpy()
    n = L + H
    assert rp.dtype == np.int64 and rp[-1] == L * (2 * r + 2) == len(col) == len(w)
    rps, cols, ws = inputs.ring_hubs_rows(L, H, r, seed, np.arange(n))
    assert np.array_equal(rp, rps) and np.array_equal(col, cols) and np.array_equal(w, ws)
    deg = np.diff(rp)
    assert np.all(deg[:L] == 2 * r + 1)
    assert deg[L:].sum() == L and deg[L:].max() - deg[L:].min() <= 1
    assert np.all((w > 0) & (w <= 1)) and np.all(w * 2.0 ** 24 == np.round(w * 2.0 ** 24))
    edges = {}
    for i in range(n):
        row = col[rp[i]:rp[i + 1]]
        assert len(set(row.tolist())) == len(row) and i not in row
        for j, x in zip(row, w[rp[i]:rp[i + 1]]):
            edges[(i, int(j))] = float(x)
    assert all(edges[(j, i)] == x for (i, j), x in edges.items())
    with pytest.raises(ValueError):
        inputs.ring_hubs_offsets(5, 1, 2)
