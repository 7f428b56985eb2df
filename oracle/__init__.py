"""CPU oracle for memory-efficient label propagation (arXiv 2411.19901).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product path (the HIP
library in ``paper_2411_19901_amd``) never imports it.

The arithmetic lives in ``lpa_oracle.c`` (plain C, fp32 sketch as fixed by
Section 5.1.2 Configuration, fp64 modularity); this module only marshals
numpy arrays through ctypes.  See that file's header for the readings of the
paper it takes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lpa_oracle.c")
_LIB = os.path.join(_HERE, "liblpa_oracle.so")

_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_f32p = ctypes.POINTER(ctypes.c_float)
_u8p = ctypes.POINTER(ctypes.c_uint8)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no fp contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
               "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
               "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.orc_sketch_accumulate.argtypes = [ctypes.c_int, _i32p, _f32p, ctypes.c_int32, ctypes.c_float]
        L.orc_sketch_accumulate.restype = None
        L.orc_sketch_max_key.argtypes = [ctypes.c_int, _i32p, _f32p, ctypes.c_int32]
        L.orc_sketch_max_key.restype = ctypes.c_int32
        L.orc_sketch_feed.argtypes = [ctypes.c_int, ctypes.c_int64, _i32p, _f32p, _i32p, _f32p]
        L.orc_sketch_feed.restype = None
        L.orc_lpa_move.argtypes = [ctypes.c_int32, _i32p, _i32p, _f32p, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, _i32p, _u8p, _i32p, _u8p, ctypes.c_int, _i64p]
        L.orc_lpa_move.restype = ctypes.c_int64
        L.orc_lpa_run.argtypes = [ctypes.c_int32, _i32p, _i32p, _f32p, ctypes.c_int, ctypes.c_int,
                                  ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int, _i32p,
                                  _i64p, _i64p]
        L.orc_lpa_run.restype = ctypes.c_int
        L.orc_lpa_choose.argtypes = [ctypes.c_int32, _i32p, _i32p, _f32p, ctypes.c_int, ctypes.c_int,
                                     ctypes.c_int, _i32p, ctypes.c_int64, _i32p, _i32p, ctypes.c_int]
        L.orc_lpa_choose.restype = None
        L.orc_modularity.argtypes = [ctypes.c_int32, _i32p, _i32p, _f32p, _i32p]
        L.orc_modularity.restype = ctypes.c_double
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t):
    return None if a is None else a.ctypes.data_as(t)


def _csr(row_ptr, col, w):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    w = None if w is None else np.ascontiguousarray(w, dtype=np.float32)
    return row_ptr, col, w


def sketch_feed(k: int, labels, weights=None):
    """Feed a stream into an empty k-slot sketch; returns (keys, vals)."""
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    weights = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
    key = np.empty(k, np.int32)
    val = np.empty(k, np.float32)
    lib().orc_sketch_feed(k, len(labels), _p(labels, _i32p), _p(weights, _f32p),
                          _p(key, _i32p), _p(val, _f32p))
    return key, val


#: value of ``k`` that selects the one-candidate vote of Algorithm 3
BM_PAPER = -1


def bm_paper_feed(labels, weights=None, init: int = -1):
    """Feed a stream into the vote of Algorithm 3 starting at (init, 0);
    returns (candidate, weight)."""
    L = lib()
    f = L.orc_bm_paper_feed
    f.argtypes = [ctypes.c_int64, _i32p, _f32p, ctypes.c_int32, _f32p]
    f.restype = ctypes.c_int32
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    weights = None if weights is None else np.ascontiguousarray(weights, dtype=np.float32)
    wt = np.zeros(1, np.float32)
    c = f(len(labels), _p(labels, _i32p), _p(weights, _f32p), init, _p(wt, _f32p))
    return int(c), float(wt[0])


def sketch_max_key(keys, vals, keep: int) -> int:
    keys = np.ascontiguousarray(keys, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float32)
    return int(lib().orc_sketch_max_key(len(keys), _p(keys, _i32p), _p(vals, _f32p), keep))


def lpa_run(row_ptr, col, w=None, k: int = 8, tol: float = 0.05, max_iter: int = 20,
            rho: int = 8, nthreads: int = 0, rescan: bool = False):
    """Algorithm 1 in Jacobi form; k=0 selects the exact argmax of Eq. 3,
    k=BM_PAPER the vote of Algorithm 3; rescan=True the double scan.

    Returns (labels, iterations, dN_trace, scanned_trace)."""
    row_ptr, col, w = _csr(row_ptr, col, w)
    n = len(row_ptr) - 1
    labels = np.empty(n, np.int32)
    dn = np.zeros(max(max_iter, 1), np.int64)
    sc = np.zeros(max(max_iter, 1), np.int64)
    it = lib().orc_lpa_run(n, _p(row_ptr, _i32p), _p(col, _i32p), _p(w, _f32p), k, int(rescan), tol,
                           max_iter, rho, nthreads, _p(labels, _i32p), _p(dn, _i64p), _p(sc, _i64p))
    if it < 0:
        raise ValueError("oracle rejected its arguments")
    return labels, it, dn[:it].copy(), sc[:it].copy()


def lpa_move(row_ptr, col, w, k: int, pickless: bool, C, act, nthreads: int = 0,
             rescan: bool = False):
    """One Jacobi iteration from (C, act). Returns (C_next, act_next, dN, scanned)."""
    row_ptr, col, w = _csr(row_ptr, col, w)
    n = len(row_ptr) - 1
    C = np.ascontiguousarray(C, dtype=np.int32)
    act = np.ascontiguousarray(act, dtype=np.uint8)
    Cn = np.empty(n, np.int32)
    an = np.zeros(n, np.uint8)
    sc = np.zeros(1, np.int64)
    dn = lib().orc_lpa_move(n, _p(row_ptr, _i32p), _p(col, _i32p), _p(w, _f32p), k, int(rescan),
                            int(pickless),
                            _p(C, _i32p), _p(act, _u8p), _p(Cn, _i32p), _p(an, _u8p), nthreads,
                            _p(sc, _i64p))
    return Cn, an, int(dn), int(sc[0])


def lpa_choose(row_ptr, col, w, k: int, pickless: bool, C, verts, nthreads: int = 0,
               rescan: bool = False):
    """Label each vertex in ``verts`` would hold after one iteration from C
    (assuming it is processed)."""
    row_ptr, col, w = _csr(row_ptr, col, w)
    n = len(row_ptr) - 1
    C = np.ascontiguousarray(C, dtype=np.int32)
    verts = np.ascontiguousarray(verts, dtype=np.int32)
    out = np.empty(len(verts), np.int32)
    lib().orc_lpa_choose(n, _p(row_ptr, _i32p), _p(col, _i32p), _p(w, _f32p), k, int(rescan),
                         int(pickless),
                         _p(C, _i32p), len(verts), _p(verts, _i32p), _p(out, _i32p), nthreads)
    return out


def modularity(row_ptr, col, w, labels) -> float:
    row_ptr, col, w = _csr(row_ptr, col, w)
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    n = len(row_ptr) - 1
    if len(labels) != n or (n and (labels.min() < 0 or labels.max() >= n)):
        raise ValueError("labels must be int32[n] with values in [0, n)")
    return float(lib().orc_modularity(n, _p(row_ptr, _i32p), _p(col, _i32p), _p(w, _f32p),
                                      _p(labels, _i32p)))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def hub_merged_sketch(row_ptr, col, w, k: int, seg_len: int, C, v: int):
    """Merged partial sketch of vertex ``v`` (Section 4.3): its row cut into
    segments of ``seg_len`` entries, each summarised by a k-slot sketch in
    CSR order (``v`` itself skipped); up to 64 partials are fed, segment by
    segment and live slot by live slot, into one sketch; above 64, partial q
    goes to chain q mod 64 and the 64 chains are combined pairwise in rounds
    at distances 32, 16, ..., 1 (chain t absorbs what chain t ^ distance held
    at the start of the round), the result being chain 0.  Returns (keys,
    vals, segments)."""
    row_ptr, col, w = _csr(row_ptr, col, w)
    C = np.ascontiguousarray(C, dtype=np.int32)
    f = lib().orc_hub_merged_sketch
    f.argtypes = [_i32p, _i32p, _f32p, ctypes.c_int, ctypes.c_int32, _i32p, ctypes.c_int32,
                  _i32p, _f32p]
    f.restype = ctypes.c_int64
    key = np.empty(k, np.int32)
    val = np.empty(k, np.float32)
    np_ = f(_p(row_ptr, _i32p), _p(col, _i32p), _p(w, _f32p), k, seg_len, _p(C, _i32p), v,
            _p(key, _i32p), _p(val, _f32p))
    if np_ < 0:
        raise ValueError("oracle rejected its arguments")
    return key, val, int(np_)


def hub_segment_choice(row_ptr, col, w, k: int, seg_len: int, C, v: int) -> int:
    """Label vertex ``v`` picks from its merged partial sketch
    (``hub_merged_sketch``): the heaviest label, ties to the lowest, an empty
    sketch keeps ``C[v]``.  Whether the vertex adopts it (pick-less rule) is
    the caller's."""
    key, val, _ = hub_merged_sketch(row_ptr, col, w, k, seg_len, C, v)
    return sketch_max_key(key, val, int(C[v]))


def hub_choose(row_ptr, col, w, k: int, seg_len: int, pickless: bool, C, verts,
               rescan: bool = False, nthreads: int = 0):
    """Label each vertex in ``verts`` holds after one iteration in which it is
    processed through its partial sketches (``hub_merged_sketch``): the
    merged sketch's heaviest label, or with ``rescan`` its live labels
    re-weighted exactly over the whole row (Section 4.4), adopted under the
    pick-less rule."""
    row_ptr, col, w = _csr(row_ptr, col, w)
    n = len(row_ptr) - 1
    C = np.ascontiguousarray(C, dtype=np.int32)
    verts = np.ascontiguousarray(verts, dtype=np.int32)
    out = np.empty(len(verts), np.int32)
    f = lib().orc_hub_choose
    f.argtypes = [ctypes.c_int32, _i32p, _i32p, _f32p, ctypes.c_int, ctypes.c_int, ctypes.c_int32,
                  ctypes.c_int, _i32p, ctypes.c_int64, _i32p, _i32p, ctypes.c_int]
    f.restype = None
    f(n, _p(row_ptr, _i32p), _p(col, _i32p), _p(w, _f32p), k, int(rescan), seg_len,
      int(pickless), _p(C, _i32p), len(verts), _p(verts, _i32p), _p(out, _i32p), nthreads)
    return out
