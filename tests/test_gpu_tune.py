"""The autotuner picks its launch shape by timing the graph, reuses a cached
decision for a graph of the same shape, and never changes a det result:
every configuration it can emit (lane thresholds, workgroup caps, layouts)
gives the oracle's labels; the batch tuner gives each graph of a batch its
group's threshold and one workgroup cap for the launch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2411_19901_amd import inputs, lpa, tune  # noqa: E402

pytestmark = pytest.mark.gpu


def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def on_dev(g):
    d = dev()
    return (torch.from_numpy(g.row_ptr).to(d), torch.from_numpy(g.col).to(d),
            torch.from_numpy(g.w).to(d) if g.w is not None else None)


@pytest.mark.parametrize("mode", ["async", "det"])
def test_tune_and_cache(mode):
    g = inputs.with_uniform_weights(inputs.rmat(14), 3)
    rp, col, w = on_dev(g)
    cache = {}
    cand = (256, 1024, 4096)
    r = tune.tune(rp, col, w, k=8, mode=mode, candidates=cand, blocks=(0, 2), allow_ranked=True,
                  cache=cache)
    assert r["lane_max_degree"] in cand and r["move_blocks_per_cu"] in (0, 2) and not r["cached"]
    assert isinstance(r["ranked"], bool)
    assert len(r["table"]) >= 3 and all(v > 0 for v in r["table"].values())
    again = tune.tune(rp, col, w, k=8, mode=mode, candidates=cand, blocks=(0, 2),
                      allow_ranked=True, cache=cache)
    assert again["cached"]
    for key in ("lane_max_degree", "move_blocks_per_cu", "ranked"):
        assert again[key] == r[key]
    s = lpa.LPA(rp, col, w, k=8, mode=mode, lane_max_degree=r["lane_max_degree"],
                move_blocks_per_cu=r["move_blocks_per_cu"], ranked=r["ranked"])
    s.run()
    lab = s.labels(device=False)
    if mode == "det":
        assert np.array_equal(lab, oracle.lpa_run(g.row_ptr, g.col, g.w, k=8)[0])
    else:
        assert lab.min() >= 0 and lab.max() < g.n
    s.close()


@pytest.mark.parametrize("k", [1, 8, 16])
def test_every_emitted_config_keeps_det_labels(k):
    g = inputs.with_uniform_weights(inputs.rmat(13), 5)
    rp, col, w = on_dev(g)
    ref, it, dn, sc = oracle.lpa_run(g.row_ptr, g.col, g.w, k=k)
    for S in tune.DEFAULT_CANDIDATES:
        for b in tune.DEFAULT_BLOCKS + (1,):
            for ranked in (False, True):
                s = lpa.LPA(rp, col, w, k=k, mode="det", lane_max_degree=S,
                            move_blocks_per_cu=b, ranked=ranked)
                assert s.run() == it
                assert np.array_equal(s.labels(device=False), ref), (S, b, ranked)
                assert np.array_equal(s.trace()[1], sc)
                s.close()


def test_tune_batch():
    specs = inputs.batch_specs(24, 77, n_lo=500, n_hi=20000)
    gs = [inputs.batch_graph(sp, 77, i) for i, sp in enumerate(specs)]
    tensors = [on_dev(g) for g in gs]
    r = tune.tune_batch(tensors, k=8, mode="det", candidates=(256, 1024, 4096), blocks=(0, 2))
    assert len(r["lane_max_degree"]) == len(gs)
    assert set(r["lane_max_degree"]) <= {256, 1024, 4096}
    assert r["move_blocks_per_cu"] in (0, 2) and set(r["batch_ms"]) == {0, 2}
    # the tuned batch still gives the oracle's labels
    stream = torch.cuda.current_stream(dev())
    solvers = [lpa.LPA(rp, col, w, k=8, mode="det", lane_max_degree=S, stream=stream)
               for (rp, col, w), S in zip(tensors, r["lane_max_degree"])]
    b = lpa.Batch(len(solvers), k=8, mode="det", stream=stream,
                  move_blocks_per_cu=r["move_blocks_per_cu"])
    b.run(solvers)
    for g, s in zip(gs, solvers):
        assert np.array_equal(s.labels(device=False), oracle.lpa_run(g.row_ptr, g.col, None, k=8)[0])
        s.close()
    b.close()
