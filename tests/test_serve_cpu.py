"""The continuous-batching scheduler on the CPU: a stand-in backend steps each
resident graph with the oracle's one-iteration function, and a fake
free-memory probe forces admission waits.  Each result must equal a solo
oracle run of the same graph, whatever the mix and admission order."""
import numpy as np
import pytest

import oracle
from paper_2411_19901_amd import inputs
from paper_2411_19901_amd.serve import Server, poisson_arrivals


class _State:
    def __init__(self, req, k):
        self.req = req
        self.k = k
        self.C = np.arange(req.n, dtype=np.int32)
        self.act = np.ones(req.n, np.uint8)
        self.iter = 0
        self.done = req.n == 0


class OracleBackend:
    def __init__(self, k=8, tol=0.05, max_iter=20, rho=8):
        self.k, self.tol, self.max_iter, self.rho = k, tol, max_iter, rho
        self.max_seen = 0

    def bytes_needed(self, req):
        return 16 * req.n + 8 * req.nnz + 4096

    def free_bytes(self):
        return 1 << 40

    def admit(self, req):
        return _State(req, self.k)

    def step(self, states):
        self.max_seen = max(self.max_seen, len(states))
        self.max_bytes = max(getattr(self, "max_bytes", 0), sum(s.req.bytes_needed for s in states))
        for s in states:
            if s.done:
                continue
            pl = self.rho > 0 and s.iter % self.rho == 0
            r = s.req
            C, act, dn, _ = oracle.lpa_move(r.row_ptr, r.col, r.w, s.k, pl, s.C, s.act)
            s.C, s.act = C, act
            s.iter += 1
            if (not pl and dn / r.n < self.tol) or s.iter >= self.max_iter:
                s.done = True

    def finished(self, s):
        return s.done

    def result(self, s):
        return s.C.copy(), s.iter

    def release(self, s):
        pass


def request_mix(count=14, seed=21):
    specs = inputs.batch_specs(count, seed, n_lo=100, n_hi=3000)
    gs = [inputs.batch_graph(s, seed, i) for i, s in enumerate(specs)]
    gs = [inputs.with_uniform_weights(g, i) if i % 2 else g for i, g in enumerate(gs)]
    gs.append(inputs.rmat(9))
    return gs


def check_results(server, graphs, k=8):
    assert len(server.completed) == len(graphs)
    by_id = {r.rid: r for r in server.completed}
    for i, g in enumerate(graphs):
        ref, it, _, _ = oracle.lpa_run(g.row_ptr, g.col, g.w, k=k)
        assert np.array_equal(by_id[i].labels, ref), g.name
        assert by_id[i].iterations == it


def test_all_at_once_equals_solo():
    gs = request_mix()
    srv = Server(OracleBackend(), max_resident=64, hbm_reserve=0)
    for g in gs:
        srv.submit(g.row_ptr, g.col, g.w, arrival=0.0)
    srv.run_until_idle()
    check_results(srv, gs)
    st = srv.latency_stats()
    assert st["count"] == len(gs) and st["p99_s"] >= st["p50_s"] >= 0


def test_resident_cap():
    gs = request_mix(count=9, seed=4)
    be = OracleBackend()
    srv = Server(be, max_resident=3, hbm_reserve=0)
    for g in gs:
        srv.submit(g.row_ptr, g.col, g.w, arrival=0.0)
    srv.run_until_idle()
    assert be.max_seen <= 3
    check_results(srv, gs)


def test_admission_waits_for_memory():
    gs = request_mix(count=8, seed=8)
    be = OracleBackend()
    budget = max(be.bytes_needed(type("R", (), {"n": g.n, "nnz": g.nnz})) for g in gs) + 10
    srv = Server(be, max_resident=64, hbm_reserve=0)
    # free memory = budget minus what the resident requests hold
    srv.free_bytes = lambda: budget - sum(r.bytes_needed for r in srv.resident)
    for g in gs:
        srv.submit(g.row_ptr, g.col, g.w, arrival=0.0)
    srv.run_until_idle()
    assert srv.waits_for_memory > 0
    assert be.max_bytes <= budget
    assert be.max_seen < len(gs)
    check_results(srv, gs)


def test_staggered_arrivals():
    gs = request_mix(count=6, seed=13)
    srv = Server(OracleBackend(), max_resident=64, hbm_reserve=0)
    t0 = srv.clock()
    arrivals = poisson_arrivals(len(gs), rate=2000.0, seed=1, start=t0)
    for g, a in zip(gs, arrivals):
        srv.submit(g.row_ptr, g.col, g.w, arrival=float(a))
    srv.run_until_idle()
    check_results(srv, gs)
    for r in srv.completed:
        assert r.admitted >= r.arrival and r.finished >= r.admitted


def test_poisson_arrivals_rate():
    a = poisson_arrivals(20000, rate=50.0, seed=3)
    assert np.all(np.diff(a) > 0)
    assert abs(len(a) / a[-1] - 50.0) < 2.0


class SlowAdmitBackend(OracleBackend):
    """Admission that takes a while (as copies and binning do), called from
    the server's admission thread."""

    def admit(self, req, overlap=False):
        assert overlap
        import time
        time.sleep(0.002)
        return _State(req, self.k)


def test_overlapped_admission_equals_solo():
    gs = request_mix(count=10, seed=31)
    be = SlowAdmitBackend()
    srv = Server(be, max_resident=4, hbm_reserve=0, overlap_admission=True)
    t0 = srv.clock()
    arrivals = poisson_arrivals(len(gs), rate=3000.0, seed=7, start=t0)
    for g, a in zip(gs, arrivals):
        srv.submit(g.row_ptr, g.col, g.w, arrival=float(a))
    srv.run_until_idle()
    srv.close()
    assert be.max_seen <= 4
    check_results(srv, gs)
    for r in srv.completed:
        assert r.admitted >= r.arrival and r.finished >= r.admitted


def test_overlapped_admission_waits_for_memory():
    gs = request_mix(count=8, seed=8)
    be = SlowAdmitBackend()
    budget = max(be.bytes_needed(type("R", (), {"n": g.n, "nnz": g.nnz})) for g in gs) + 10
    srv = Server(be, max_resident=64, hbm_reserve=0, overlap_admission=True)
    # free memory = budget minus what admitted requests hold
    srv.free_bytes = lambda: budget - sum(r.bytes_needed for r in srv.resident + list(srv.ready))
    for g in gs:
        srv.submit(g.row_ptr, g.col, g.w, arrival=0.0)
    srv.run_until_idle()
    srv.close()
    assert srv.waits_for_memory > 0
    assert be.max_bytes <= budget
    check_results(srv, gs)
