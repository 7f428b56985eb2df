"""The autotuner picks one of its candidates by timing the graph, reuses a
cached decision for a graph of the same shape, and never changes a det
result."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2411_19901_amd import inputs, lpa, tune  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mode", ["async", "det"])
def test_tune_and_cache(mode):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    d = torch.device("cuda:0")
    g = inputs.with_uniform_weights(inputs.rmat(14), 3)
    rp, col, w = (torch.from_numpy(g.row_ptr).to(d), torch.from_numpy(g.col).to(d),
                  torch.from_numpy(g.w).to(d))
    cache = {}
    cand = (256, 1024, 4096)
    r = tune.tune(rp, col, w, k=8, mode=mode, candidates=cand, cache=cache)
    assert r["lane_max_degree"] in cand and not r["cached"]
    assert set(r["table"]) <= set(cand) and all(v > 0 for v in r["table"].values())
    again = tune.tune(rp, col, w, k=8, mode=mode, candidates=cand, cache=cache)
    assert again["cached"] and again["lane_max_degree"] == r["lane_max_degree"]
    s = lpa.LPA(rp, col, w, k=8, mode=mode, lane_max_degree=r["lane_max_degree"])
    s.run()
    lab = s.labels(device=False)
    if mode == "det":
        assert np.array_equal(lab, oracle.lpa_run(g.row_ptr, g.col, g.w, k=8)[0])
    else:
        assert lab.min() >= 0 and lab.max() < g.n
    s.close()
