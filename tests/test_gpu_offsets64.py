"""Graphs whose row offsets are int64 (lpa_graph.row_ptr64).

* The parity graphs with their offsets handed over as int64: det runs equal
  the oracle bit for bit (labels, iterations, changed and scanned counts)
  for the sketch rule, the vote of Algorithm 3 and the double scan; async
  runs are valid and their modularity is the oracle's for the same labels;
  a batch mixing int32 and int64 offsets gives every graph its solo result;
  int64 offsets in pinned host memory work too.
* A ring-plus-hubs graph of 2,232,000,000 CSR entries (beyond 2^31; every
  hub row and the rows of lane vertices above id 35.2M start past entry
  2^31): two det iterations checked against the oracle's label choice on
  sampled vertices, every hub included; the async run's modularity against
  Q evaluated from its definition in fp64 with torch on the device.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2411_19901_amd import inputs, lpa  # noqa: E402
from test_gpu_parity import graph  # noqa: E402  (the parity graph suite)

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def to_dev64(g, pinned=False):
    rp = torch.from_numpy(g.row_ptr.astype(np.int64))
    col = torch.from_numpy(np.ascontiguousarray(g.col))
    w = torch.from_numpy(g.w) if g.w is not None else None
    if pinned:
        return rp.pin_memory(), col.pin_memory(), (w.pin_memory() if w is not None else None)
    d = dev()
    return rp.to(d), col.to(d), (w.to(d) if w is not None else None)


def to_dev32(g):
    d = dev()
    return (torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(d),
            torch.from_numpy(np.ascontiguousarray(g.col)).to(d),
            torch.from_numpy(g.w).to(d) if g.w is not None else None)


def oracle_run(g, k, **kw):
    ok = oracle.BM_PAPER if kw.get("rule") == "bm_paper" else k
    return oracle.lpa_run(g.row_ptr, g.col, g.w, k=ok, rescan=kw.get("rescan", False))


SMALL = ["two-cliques-5", "sbm1-s2-w", "rmat14-w", "star5000", "rmat10-selfloops", "sbm1-iso"]


@pytest.mark.parametrize("name", SMALL)
@pytest.mark.parametrize("variant", [dict(k=1), dict(k=8), dict(k=32),
                                     dict(k=8, lane_max_degree=64), dict(k=1, rule="bm_paper"),
                                     dict(k=8, rescan=True)])
def test_det_parity_offsets64(name, variant):
    g = graph(name)
    rp, col, w = to_dev64(g)
    assert rp.dtype == torch.int64
    s = lpa.LPA(rp, col, w, mode="det", **variant)
    it = s.run()
    lab = s.labels(device=False)
    dn, sc = s.trace()
    ref, rit, rdn, rsc = oracle_run(g, **variant)
    assert it == rit and np.array_equal(dn, rdn) and np.array_equal(sc, rsc), (name, variant)
    assert np.array_equal(lab, ref), (name, variant)
    assert abs(s.modularity() - oracle.modularity(g.row_ptr, g.col, g.w, ref)) <= 1e-9
    s.close()


@pytest.mark.parametrize("variant", [dict(k=8), dict(k=8, lane_max_degree=64),
                                     dict(k=1, rule="bm_paper"), dict(k=8, rescan=True),
                                     dict(k=8, hub_shared=True, lane_max_degree=64)])
def test_async_offsets64(variant):
    for name in ("sbm1-s1", "rmat14-w", "star5000"):
        g = graph(name)
        rp, col, w = to_dev64(g)
        s = lpa.LPA(rp, col, w, mode="async", **variant)
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


@pytest.mark.parametrize("mode", ["det", "async"])
def test_batch_mixes_offset_widths(mode):
    gs = [graph("sbm1-s1"), graph("rmat14-w"), graph("star5000"), graph("sbm1-iso")]
    solvers = []
    for i, g in enumerate(gs):
        rp, col, w = to_dev64(g) if i % 2 else to_dev32(g)
        solvers.append(lpa.LPA(rp, col, w, k=8, mode=mode))
    batch = lpa.Batch(len(gs), k=8, mode=mode)
    batch.run(solvers)
    for g, s in zip(gs, solvers):
        lab = s.labels(device=False)
        if mode == "det":
            assert np.array_equal(lab, oracle_run(g, 8)[0]), g.name
        else:
            assert lab.min() >= 0 and lab.max() < g.n
            assert abs(s.modularity() - oracle.modularity(g.row_ptr, g.col, g.w, lab)) <= 1e-9
    for x in solvers + [batch]:
        x.close()


def test_modularity_same_for_both_widths():
    g = graph("rmat14-w")
    ref = oracle_run(g, 8)[0]
    lab = torch.from_numpy(ref).to(dev())
    qs = []
    for rp, col, w in (to_dev32(g), to_dev64(g)):
        s = lpa.LPA(rp, col, w, k=8)
        qs.append(s.modularity(lab))
        s.close()
    qr = oracle.modularity(g.row_ptr, g.col, g.w, ref)
    assert abs(qs[0] - qr) <= 1e-9 and abs(qs[1] - qr) <= 1e-9


def test_pinned_host_offsets64():
    dev()
    g = graph("rmat14-w")
    rp, col, w = to_dev64(g, pinned=True)
    assert lpa.pointer_location(rp.data_ptr()) == lpa.LPA_PTR_HOST
    s = lpa.LPA(rp, col, w, k=8, mode="det")
    it = s.run()
    ref, rit, _, _ = oracle_run(g, 8)
    assert it == rit and np.array_equal(s.labels(device=False), ref)
    s.close()


def test_invalid_offsets64_rejected():
    g = graph("sbm1-s1")
    rp, col, w = to_dev64(g)
    bad = rp.clone()
    bad[-1] += 1  # row_ptr[n] != nnz
    with pytest.raises(lpa.LpaError):
        lpa.LPA(bad, col, w, k=8)
    bad = rp.clone()
    bad[5] = bad[6] + 1  # decreasing
    with pytest.raises(lpa.LpaError):
        lpa.LPA(bad, col, w, k=8)


# ---- beyond 2^31 entries ---------------------------------------------------

L_BIG, H_BIG, R_BIG, SEED_BIG = 36_000_000, 64, 30, 2024  # nnz = 62 L = 2.232e9


def q_definition(rp, col, w, lab, L, H, D, chunk=1 << 27):
    """Q = sigma / 2m - sum_c (Sigma_c / 2m)^2 in fp64, rows from the closed
    form (lane row j holds entries [jD, (j+1)D), hubs follow)."""
    labl = lab.long()
    n = L + H
    k_row = torch.zeros(n, dtype=torch.float64, device=lab.device)
    sigma = torch.zeros((), dtype=torch.float64, device=lab.device)
    two_m = torch.zeros((), dtype=torch.float64, device=lab.device)
    rows_per = chunk // D
    for j0 in range(0, L, rows_per):
        j1 = min(L, j0 + rows_per)
        wc = w[j0 * D:j1 * D].double().view(j1 - j0, D)
        cc = col[j0 * D:j1 * D].long().view(j1 - j0, D)
        same = labl[cc] == labl[j0:j1, None]
        sigma += (wc * same).sum()
        k_row[j0:j1] = wc.sum(1)
        two_m += wc.sum()
    rph = rp[L:].cpu().numpy()
    for t in range(H):
        b, e = int(rph[t]), int(rph[t + 1])
        wc = w[b:e].double()
        same = labl[col[b:e].long()] == labl[L + t]
        sigma += (wc * same).sum()
        k_row[L + t] = wc.sum()
        two_m += wc.sum()
    tot = torch.zeros(n, dtype=torch.float64, device=lab.device).index_add_(0, labl, k_row)
    return float(sigma / two_m - ((tot / two_m) ** 2).sum())


@pytest.mark.timeout(900)
def test_beyond_2_31_entries():
    d = dev()
    free, _ = torch.cuda.mem_get_info(d)
    L, H, r, seed = L_BIG, H_BIG, R_BIG, SEED_BIG
    D = 2 * r + 1
    nnz = L * (D + 1)
    if free < nnz * 8 + (8 << 30):
        pytest.skip("not enough device memory for a 2^31+ entry graph")
    print(f"building ring+hubs L={L} H={H} r={r} nnz={nnz}", flush=True)
    rp, col, w = inputs.ring_hubs_device(L, H, r, seed, d)
    n = L + H
    assert int(rp[-1]) == nnz > 2 ** 31
    rng = np.random.default_rng(31)
    past = int(np.ceil(2 ** 31 / D))  # lane rows starting beyond entry 2^31
    sample = np.unique(np.concatenate([rng.choice(L, 2000, replace=False),
                                       rng.integers(past, L, 1000),
                                       np.arange(L, n)])).astype(np.int32)
    srp, scol, sw = inputs.ring_hubs_rows(L, H, r, seed, sample)
    # the device graph agrees with the closed form on sampled rows
    for i in list(range(0, len(sample), 97)) + list(range(len(sample) - H, len(sample))):
        v = int(sample[i])
        b, e = int(rp[v]), int(rp[v + 1])
        assert np.array_equal(col[b:e].cpu().numpy(), scol[srp[i]:srp[i + 1]]), v
        assert np.array_equal(w[b:e].cpu().numpy(), sw[srp[i]:srp[i + 1]]), v
    # the sampled rows as a CSR over all n vertices for the oracle
    deg = np.zeros(n + 1, np.int64)
    deg[sample.astype(np.int64) + 1] = np.diff(srp)
    orp = np.cumsum(deg).astype(np.int32)

    print("det run", flush=True)
    s = lpa.LPA(rp, col, w, k=8, mode="det")
    for _ in range(2):
        C, act, l = s.get_state()
        ch, _ = s.step()
        C2, _, _ = s.get_state()
        assert ch == int(np.count_nonzero(C2 != C))
        pl = l % 8 == 0
        chosen = oracle.lpa_choose(orp, scol, sw, 8, pl, C, sample)
        expect = np.where(act[sample] != 0, chosen, C[sample])
        bad = np.nonzero(C2[sample] != expect)[0]
        assert bad.size == 0, (l, sample[bad[:10]], C2[sample[bad[:10]]], expect[bad[:10]])
    dn, sc = s.trace()
    assert sc[0] == nnz  # every entry scanned in iteration 0
    s.close()

    print("async run", flush=True)
    s = lpa.LPA(rp, col, w, k=8, mode="async")
    it = s.run()
    lab = s.labels(device=True)
    assert 1 <= it <= 20
    assert int(lab.min()) >= 0 and int(lab.max()) < n
    q = s.modularity()
    qd = q_definition(rp, col, w, lab, L, H, D)
    assert abs(q - qd) <= 1e-9, (q, qd)
    print(f"async iterations {it} Q {q:.6f}", flush=True)
    s.close()
