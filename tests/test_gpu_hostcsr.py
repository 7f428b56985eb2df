"""Graph arrays in pinned host memory: the kernels read the CSR over the host
link while labels, flags and counters stay in device memory.  Results must
equal the oracle exactly in det mode; memory the device cannot map is
refused before any kernel runs."""
import ctypes

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2411_19901_amd import inputs, lpa  # noqa: E402

pytestmark = pytest.mark.gpu


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_pointer_locations():
    need_gpu()
    d = torch.zeros(16, dtype=torch.int32, device="cuda:0")
    p = torch.zeros(16, dtype=torch.int32).pin_memory()
    a = np.zeros(16, np.int32)
    assert lpa.pointer_location(d.data_ptr()) == lpa.LPA_PTR_DEVICE
    assert lpa.pointer_location(p.data_ptr()) == lpa.LPA_PTR_HOST
    assert lpa.pointer_location(a.ctypes.data) == lpa.LPA_PTR_UNUSABLE
    assert lpa.pointer_location(0) == lpa.LPA_PTR_UNUSABLE


@pytest.mark.parametrize("mode", ["det", "async"])
def test_pinned_host_csr(mode):
    need_gpu()
    g = inputs.with_uniform_weights(inputs.rmat(14), 7)
    rp = torch.from_numpy(g.row_ptr).pin_memory()
    col = torch.from_numpy(g.col).pin_memory()
    w = torch.from_numpy(g.w).pin_memory()
    assert lpa.pointer_location(col.data_ptr()) == lpa.LPA_PTR_HOST
    s = lpa.LPA(rp, col, w, k=8, mode=mode)
    it = s.run()
    lab = s.labels(device=False)
    if mode == "det":
        ref, rit, rdn, rsc = oracle.lpa_run(g.row_ptr, g.col, g.w, k=8)
        assert it == rit and np.array_equal(lab, ref)
    assert abs(s.modularity() - oracle.modularity(g.row_ptr, g.col, g.w, lab)) <= 1e-9
    core, _ = s.memory()
    assert core < 64 * g.n + (1 << 20)  # O(|V|) device state, no copy of the CSR
    s.close()


def test_pageable_memory_refused():
    need_gpu()
    g = inputs.rmat(10)
    rp = np.ascontiguousarray(g.row_ptr)
    col = np.ascontiguousarray(g.col)
    # only hand the arrays to lpa_init once the library has classified them
    # as unusable: it must then refuse them without launching anything
    assert lpa.pointer_location(rp.ctypes.data) == lpa.LPA_PTR_UNUSABLE
    assert lpa.pointer_location(col.ctypes.data) == lpa.LPA_PTR_UNUSABLE
    L = lpa.load()
    graph = lpa.LpaGraph(g.n, g.nnz, rp.ctypes.data, col.ctypes.data)
    cfg = lpa.lpa_config_default()
    h = ctypes.c_void_p(0)
    rc = L.lpa_init(ctypes.byref(graph), None, 8, 0.05, 20, 0, ctypes.byref(cfg), ctypes.byref(h))
    assert rc == lpa.LPA_ERR_ARG and not h.value
    # labels for modularity are checked the same way
    d = torch.device("cuda:0")
    s = lpa.LPA(torch.from_numpy(g.row_ptr).to(d), torch.from_numpy(g.col).to(d), None, k=8)
    bad = np.zeros(g.n, np.int32)
    assert lpa.pointer_location(bad.ctypes.data) == lpa.LPA_PTR_UNUSABLE
    q = ctypes.c_double(0)
    assert L.lpa_modularity(s.h, bad.ctypes.data, ctypes.byref(q)) == lpa.LPA_ERR_ARG
    s.close()
