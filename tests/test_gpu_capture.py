"""Iterations replayed from a captured hipGraph (LPA_CAPTURE) give the same
results as kernels launched one by one.  Each graph is replayed several
times with eager work and synchronisations in between, and every replay is
checked against the eager result."""
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


def tensors(g):
    d = dev()
    return (torch.from_numpy(g.row_ptr).to(d), torch.from_numpy(g.col).to(d),
            torch.from_numpy(g.w).to(d) if g.w is not None else None)


def graphs(count=12, seed=31):
    specs = inputs.batch_specs(count, seed, n_lo=200, n_hi=5000)
    gs = [inputs.batch_graph(s, seed, i) for i, s in enumerate(specs)]
    gs = [inputs.with_uniform_weights(g, i) if i % 2 else g for i, g in enumerate(gs)]
    gs.append(inputs.rmat(11))
    return gs


@pytest.mark.parametrize("mode", ["det", "async"])
def test_single_handle_replays(mode):
    g = inputs.with_uniform_weights(inputs.rmat(13), 5)
    rp, col, w = tensors(g)
    eager = lpa.LPA(rp, col, w, k=8, mode=mode)
    eager.run()
    ref = eager.labels(device=False)
    cap = lpa.LPA(rp, col, w, k=8, mode=mode, capture=True)
    other = lpa.LPA(*tensors(inputs.sbm1()), k=8)
    for rep in range(4):
        cap.reset()
        it = cap.run()
        lab = cap.labels(device=False)
        assert 1 <= it <= 20
        if mode == "det":
            assert np.array_equal(lab, ref), rep
            assert it == eager.iterations()
        else:
            assert lab.min() >= 0 and lab.max() < g.n
        other.reset()  # eager work between replays
        other.run()
        torch.cuda.synchronize()
    if mode == "det":
        assert np.array_equal(ref, oracle.lpa_run(g.row_ptr, g.col, g.w, k=8)[0])
    for x in (eager, cap, other):
        x.close()


def test_batch_replays_match_eager():
    gs = graphs()
    eager = [lpa.LPA(*tensors(g), k=8) for g in gs]
    lpa.Batch(len(gs), k=8).run(eager)
    ref = [s.labels(device=False) for s in eager]
    cap = [lpa.LPA(*tensors(g), k=8) for g in gs]
    batch = lpa.Batch(len(gs), k=8, capture=True)
    for rep in range(3):
        for s in cap:
            s.reset()
        batch.run(cap)
        for g, s, r in zip(gs, cap, ref):
            assert np.array_equal(s.labels(device=False), r), (rep, g.name)
        eager[0].reset()  # eager work between replays
        eager[0].run()
        torch.cuda.synchronize()
    # a different set of graphs changes the launch shape: captured again
    batch.run(cap[:5])
    for s in cap[:5]:
        s.reset()
    batch.run(cap[:5])
    for g, s, r in zip(gs, cap[:5], ref):
        assert np.array_equal(s.labels(device=False), r), g.name
    for s in eager + cap:
        s.close()
    batch.close()


def test_step_by_step_capture():
    g = inputs.sbm1(2)
    rp, col, w = tensors(g)
    s = lpa.LPA(rp, col, w, k=8, capture=True)
    steps = 0
    done = False
    while not done:
        _, done = s.step()
        steps += 1
        assert steps <= 20
    ref, rit, _, _ = oracle.lpa_run(g.row_ptr, g.col, g.w, k=8)
    assert steps == rit and np.array_equal(s.labels(device=False), ref)
    s.close()
