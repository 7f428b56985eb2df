"""GPU serving loop: requests admitted as they arrive, iterated together with
one batched launch per tick; in det mode each result equals the same graph
solved alone (and the CPU oracle)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2411_19901_amd import inputs  # noqa: E402
from paper_2411_19901_amd.serve import Backend, Server, poisson_arrivals  # noqa: E402

pytestmark = pytest.mark.gpu


def test_serving_mix_equals_alone():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    specs = inputs.batch_specs(16, 55, n_lo=200, n_hi=20000)
    gs = [inputs.batch_graph(s, 55, i) for i, s in enumerate(specs)]
    gs = [inputs.with_uniform_weights(g, i) if i % 2 else g for i, g in enumerate(gs)]
    gs += [inputs.with_uniform_weights(inputs.rmat(s), s) for s in (11, 13)]
    be = Backend(k=8, mode="det", capacity=8)
    srv = Server(be, max_resident=8, hbm_reserve=0)
    t0 = srv.clock()
    for g, a in zip(gs, poisson_arrivals(len(gs), rate=500.0, seed=2, start=t0)):
        srv.submit(g.row_ptr, g.col, g.w, arrival=float(a))
    srv.run_until_idle()
    assert len(srv.completed) == len(gs)
    by_id = {r.rid: r for r in srv.completed}
    for i, g in enumerate(gs):
        ref, it, _, _ = oracle.lpa_run(g.row_ptr, g.col, g.w, k=8)
        assert np.array_equal(by_id[i].labels, ref), g.name
        assert by_id[i].iterations == it
    st = srv.latency_stats()
    assert st["count"] == len(gs) and st["p99_s"] >= st["p50_s"] > 0
    be.close()
