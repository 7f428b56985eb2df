"""Python binding of liblpa.so (the C ABI declared in include/lpa.h).

Argument marshalling only: every step of label propagation runs in the
library's HIP kernels.  PyTorch supplies device memory (tensors passed by
pointer) and the stream.  If the library is missing or cannot be loaded the
calls raise; there is no CPU fallback.

The functions mirror the C names (``lpa_init``, ``lpa_step``, ``lpa_run``,
``lpa_modularity``, ...); :class:`LPA` wraps a handle for convenience.
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Tuple

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblpa.so")
HEADER = os.path.join(os.path.dirname(PKG), "include", "lpa.h")

LPA_OK = 0
LPA_ERR_ARG = 1
LPA_ERR_GRAPH = 2
LPA_ERR_UNSUPPORTED = 3
LPA_ERR_NOMEM = 4
LPA_ERR_HIP = 5
LPA_ERR_STATE = 6

LPA_MODE_DET = 0
LPA_MODE_ASYNC = 1
LPA_VALIDATE = 0x100
LPA_RULE_BM_PAPER = 0x200
LPA_RESCAN = 0x400
LPA_HUB_SHARED = 0x800
LPA_CAPTURE = 0x1000
LPA_SHARED_VARS = 0x2000
LPA_STREAM_CSR = 0x4000
LPA_RANKED_LAYOUT = 0x8000

MODES = {"det": LPA_MODE_DET, "async": LPA_MODE_ASYNC}
# per-vertex rule: the k-slot weighted Misra-Gries sketch, or the
# one-candidate vote of Algorithm 3 (needs k=1)
RULES = {"mg": 0, "bm_paper": LPA_RULE_BM_PAPER}


class LpaGraph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("row_ptr64", ctypes.c_void_p)]


class LpaConfig(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("rho", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("lane_max_degree", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("workspace", ctypes.c_void_p),
                ("workspace_bytes", ctypes.c_size_t), ("stream_chunk_kib", ctypes.c_int32),
                ("move_blocks_per_cu", ctypes.c_int32), ("reserved", ctypes.c_int32 * 2)]


class LpaError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {error_string(code)} ({code})")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load liblpa.so (raises OSError when it is not built or not loadable)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(path)
    H = ctypes.c_void_p
    pH = ctypes.POINTER(ctypes.c_void_p)
    i64p = ctypes.POINTER(ctypes.c_int64)
    ip = ctypes.POINTER(ctypes.c_int)
    szp = ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "lpa_config_default": (None, [ctypes.POINTER(LpaConfig)]),
        "lpa_init": (ctypes.c_int, [ctypes.POINTER(LpaGraph), ctypes.c_void_p, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_int, ctypes.c_uint64,
                                    ctypes.POINTER(LpaConfig), pH]),
        "lpa_reset": (ctypes.c_int, [H]),
        "lpa_set_stream": (ctypes.c_int, [H, ctypes.c_void_p]),
        "lpa_step": (ctypes.c_int, [H, i64p, ip]),
        "lpa_run": (ctypes.c_int, [H, ip]),
        "lpa_modularity": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double)]),
        "lpa_modularity_noalloc": (ctypes.c_int, [H, ctypes.c_void_p,
                                                  ctypes.POINTER(ctypes.c_double)]),
        "lpa_get_labels": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.c_int]),
        "lpa_get_trace": (ctypes.c_int, [H, i64p, i64p, ctypes.c_int, ip]),
        "lpa_get_state": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.c_void_p, ip, ctypes.c_int]),
        "lpa_set_state": (ctypes.c_int, [H, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                         ctypes.c_int]),
        "lpa_memory": (ctypes.c_int, [H, szp, szp]),
        "lpa_progress": (ctypes.c_int, [H, ip, ip]),
        "lpa_profile": (ctypes.c_int, [H, ctypes.c_int]),
        "lpa_memory_floor": (ctypes.c_int, [H, ctypes.c_int, ctypes.POINTER(ctypes.c_float)]),
        "lpa_get_profile": (ctypes.c_int, [H, ctypes.POINTER(ctypes.c_float), ctypes.c_int, ip]),
        "lpa_free": (ctypes.c_int, [H]),
        "lpa_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int,
                                               ctypes.c_int, ctypes.POINTER(LpaConfig), szp]),
        "lpa_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(LpaConfig),
                                            pH]),
        "lpa_batch_step": (ctypes.c_int, [H, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, i64p,
                                          ip]),
        "lpa_batch_run": (ctypes.c_int, [H, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ip]),
        "lpa_batch_free": (ctypes.c_int, [H]),
        "lpa_batch_reset": (ctypes.c_int, [H, ctypes.POINTER(ctypes.c_void_p), ctypes.c_int]),
        "lpa_error_string": (ctypes.c_char_p, [ctypes.c_int]),
        "lpa_last_error": (ctypes.c_char_p, [H]),
        "lpa_pointer_location": (ctypes.c_int, [ctypes.c_void_p, ip]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def header_functions(header: str = HEADER):
    """Names of the functions declared in include/lpa.h."""
    text = open(header).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lpa_\w+)\s*\(", text, re.M)))


LPA_PTR_UNUSABLE, LPA_PTR_DEVICE, LPA_PTR_HOST = 0, 1, 2


def pointer_location(ptr: int) -> int:
    """Where the kernels would read an array at address ``ptr`` from."""
    loc = ctypes.c_int(-1)
    _check(load().lpa_pointer_location(ctypes.c_void_p(ptr), ctypes.byref(loc)),
           "lpa_pointer_location")
    return loc.value


def error_string(code: int) -> str:
    try:
        return load().lpa_error_string(code).decode()
    except OSError:
        return "liblpa.so not loaded"


def _check(code: int, what: str, h=None):
    if code != LPA_OK:
        msg = what
        if h:
            last = load().lpa_last_error(h)
            if last:
                msg += f" [{last.decode()}]"
        raise LpaError(code, msg)


# ----------------------------------------------------------------- C names
def lpa_config_default() -> LpaConfig:
    cfg = LpaConfig()
    load().lpa_config_default(ctypes.byref(cfg))
    return cfg


def lpa_init(n: int, nnz: int, row_ptr_ptr: int, col_ptr: int, weights_ptr: Optional[int],
             k: int, tol: float, max_iter: int, seed: int, cfg: LpaConfig,
             offsets64: bool = False):
    """``offsets64``: ``row_ptr_ptr`` points to int64 offsets (row_ptr64)."""
    g = (LpaGraph(n, nnz, None, col_ptr, row_ptr_ptr) if offsets64
         else LpaGraph(n, nnz, row_ptr_ptr, col_ptr))
    h = ctypes.c_void_p()
    rc = load().lpa_init(ctypes.byref(g), weights_ptr or None, k, tol, max_iter, seed,
                         ctypes.byref(cfg), ctypes.byref(h))
    _check(rc, "lpa_init")
    return h


def lpa_step(h) -> Tuple[int, bool]:
    ch = ctypes.c_int64(0)
    dn = ctypes.c_int(0)
    _check(load().lpa_step(h, ctypes.byref(ch), ctypes.byref(dn)), "lpa_step", h)
    return int(ch.value), bool(dn.value)


def lpa_run(h) -> int:
    it = ctypes.c_int(0)
    _check(load().lpa_run(h, ctypes.byref(it)), "lpa_run", h)
    return int(it.value)


def lpa_reset(h) -> None:
    _check(load().lpa_reset(h), "lpa_reset", h)


def lpa_modularity(h, labels_ptr: Optional[int] = None) -> float:
    q = ctypes.c_double(0.0)
    _check(load().lpa_modularity(h, labels_ptr or None, ctypes.byref(q)), "lpa_modularity", h)
    return float(q.value)


def lpa_modularity_noalloc(h, labels_ptr: Optional[int] = None) -> float:
    q = ctypes.c_double(0.0)
    _check(load().lpa_modularity_noalloc(h, labels_ptr or None, ctypes.byref(q)),
           "lpa_modularity_noalloc", h)
    return float(q.value)


def lpa_get_labels(h, out_ptr: int, out_is_host: bool) -> None:
    _check(load().lpa_get_labels(h, out_ptr, int(out_is_host)), "lpa_get_labels", h)


def lpa_get_trace(h, capacity: int):
    ch = np.zeros(max(capacity, 1), np.int64)
    sc = np.zeros(max(capacity, 1), np.int64)
    cnt = ctypes.c_int(0)
    i64p = ctypes.POINTER(ctypes.c_int64)
    _check(load().lpa_get_trace(h, ch.ctypes.data_as(i64p), sc.ctypes.data_as(i64p), capacity,
                                ctypes.byref(cnt)), "lpa_get_trace", h)
    m = min(cnt.value, capacity)
    return ch[:m].copy(), sc[:m].copy()


def lpa_get_state(h, labels_ptr: int, flags_ptr: int, is_host: bool) -> int:
    it = ctypes.c_int(0)
    _check(load().lpa_get_state(h, labels_ptr, flags_ptr, ctypes.byref(it), int(is_host)),
           "lpa_get_state", h)
    return int(it.value)


def lpa_set_state(h, labels_ptr: int, flags_ptr: int, iteration: int, is_host: bool) -> None:
    _check(load().lpa_set_state(h, labels_ptr, flags_ptr, iteration, int(is_host)),
           "lpa_set_state", h)


def lpa_progress(h) -> Tuple[int, bool]:
    it = ctypes.c_int(0)
    fin = ctypes.c_int(0)
    _check(load().lpa_progress(h, ctypes.byref(it), ctypes.byref(fin)), "lpa_progress", h)
    return int(it.value), bool(fin.value)


def lpa_memory(h) -> Tuple[int, int]:
    core = ctypes.c_size_t(0)
    ev = ctypes.c_size_t(0)
    _check(load().lpa_memory(h, ctypes.byref(core), ctypes.byref(ev)), "lpa_memory", h)
    return int(core.value), int(ev.value)


def lpa_profile(h, enable: bool) -> None:
    _check(load().lpa_profile(h, int(enable)), "lpa_profile", h)


def lpa_get_profile(h, capacity: int) -> np.ndarray:
    ms = np.zeros(max(capacity, 1), np.float32)
    cnt = ctypes.c_int(0)
    _check(load().lpa_get_profile(h, ms.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), capacity,
                                  ctypes.byref(cnt)), "lpa_get_profile", h)
    return ms[:min(cnt.value, capacity)].copy()


def lpa_memory_floor(h, reps: int = 3) -> float:
    ms = ctypes.c_float(0.0)
    _check(load().lpa_memory_floor(h, reps, ctypes.byref(ms)), "lpa_memory_floor", h)
    return float(ms.value)


def lpa_free(h) -> None:
    if h:
        load().lpa_free(h)


def lpa_workspace_bytes(n: int, nnz: int, k: int, max_iter: int, cfg: LpaConfig) -> int:
    out = ctypes.c_size_t(0)
    _check(load().lpa_workspace_bytes(n, nnz, k, max_iter, ctypes.byref(cfg), ctypes.byref(out)),
           "lpa_workspace_bytes")
    return int(out.value)


def lpa_batch_create(capacity: int, k: int, cfg: LpaConfig):
    b = ctypes.c_void_p()
    _check(load().lpa_batch_create(capacity, k, ctypes.byref(cfg), ctypes.byref(b)),
           "lpa_batch_create")
    return b


def _handle_array(handles):
    arr = (ctypes.c_void_p * max(1, len(handles)))()
    for i, h in enumerate(handles):
        arr[i] = h.value if isinstance(h, ctypes.c_void_p) else h
    return arr


def lpa_batch_step(b, handles) -> Tuple[int, bool]:
    ch = ctypes.c_int64(0)
    dn = ctypes.c_int(0)
    _check(load().lpa_batch_step(b, _handle_array(handles), len(handles), ctypes.byref(ch),
                                 ctypes.byref(dn)), "lpa_batch_step")
    return int(ch.value), bool(dn.value)


def lpa_batch_run(b, handles) -> int:
    it = ctypes.c_int(0)
    _check(load().lpa_batch_run(b, _handle_array(handles), len(handles), ctypes.byref(it)),
           "lpa_batch_run")
    return int(it.value)


def lpa_batch_free(b) -> None:
    if b:
        load().lpa_batch_free(b)


# ----------------------------------------------------------------- wrapper
class LPA:
    """One label-propagation problem on device-resident torch tensors.

    ``row_ptr`` (int32, or int64 for graphs of 2^31 or more entries) and
    ``col`` (int32) are CUDA tensors holding a symmetric CSR, ``weights`` a
    float32 CUDA tensor or None (unit weights); pinned host tensors are
    accepted too.  The tensors are kept alive by this object, as the
    library borrows them."""

    def __init__(self, row_ptr, col, weights=None, k: int = 8, tol: float = 0.05,
                 max_iter: int = 20, seed: int = 0, mode: str = "det", rho: int = 8,
                 validate: bool = True, lane_max_degree: int = 0, check_every: int = 0,
                 stream=None, workspace=None, rule: str = "mg", rescan: bool = False,
                 hub_shared: bool = False, capture: bool = False, shared_vars: bool = False,
                 stream_csr: bool = False, stream_chunk_kib: int = 0, ranked: bool = False,
                 move_blocks_per_cu: int = 0):
        import torch

        def usable(t):  # device memory, or pinned host memory the device maps
            return t.is_cuda or (t.device.type == "cpu" and t.is_pinned())

        for t, dts in ((row_ptr, (torch.int32, torch.int64)), (col, (torch.int32,))):
            if t.dtype not in dts or not usable(t) or not t.is_contiguous():
                raise ValueError("row_ptr (int32 / int64) and col (int32) must be contiguous "
                                 "CUDA (or pinned) tensors")
        if weights is not None and (weights.dtype != torch.float32 or not usable(weights)
                                    or not weights.is_contiguous()):
            raise ValueError("weights must be a contiguous float32 CUDA (or pinned) tensor")
        self._keep = (row_ptr, col, weights)
        self.n = row_ptr.numel() - 1
        self.nnz = col.numel()
        self.max_iter = max_iter
        self.device = (row_ptr.device if row_ptr.is_cuda
                       else torch.device("cuda", torch.cuda.current_device()))
        cfg = lpa_config_default()
        cfg.flags = (MODES[mode] | RULES[rule] | (LPA_VALIDATE if validate else 0)
                     | (LPA_RESCAN if rescan else 0) | (LPA_HUB_SHARED if hub_shared else 0)
                     | (LPA_SHARED_VARS if shared_vars else 0)
                     | (LPA_CAPTURE if capture else 0) | (LPA_STREAM_CSR if stream_csr else 0)
                     | (LPA_RANKED_LAYOUT if ranked else 0))
        cfg.stream_chunk_kib = stream_chunk_kib
        cfg.move_blocks_per_cu = move_blocks_per_cu
        cfg.rho = rho
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        cfg.stream = stream.cuda_stream
        cfg.lane_max_degree = lane_max_degree
        cfg.check_every = check_every
        if workspace is not None:  # a uint8 CUDA tensor kept alive by this object
            cfg.workspace = workspace.data_ptr()
            cfg.workspace_bytes = workspace.numel()
            self._keep = self._keep + (workspace,)
        self.k = k
        self.mode = mode
        self.rule = rule
        self.rescan = rescan
        with torch.cuda.device(self.device):
            self.h = lpa_init(self.n, self.nnz, row_ptr.data_ptr(), col.data_ptr() if self.nnz else 0,
                              weights.data_ptr() if weights is not None else None, k, tol,
                              max_iter, seed, cfg, offsets64=row_ptr.dtype == torch.int64)

    def step(self) -> Tuple[int, bool]:
        return lpa_step(self.h)

    def set_stream(self, stream) -> None:
        """Enqueue all later work of this handle on ``stream`` (a torch stream)."""
        _check(load().lpa_set_stream(self.h, stream.cuda_stream), "lpa_set_stream", self.h)
        self.stream = stream

    def run(self) -> int:
        return lpa_run(self.h)

    def reset(self) -> None:
        lpa_reset(self.h)

    def labels(self, device: bool = True):
        import torch
        if device:
            out = torch.empty(self.n, dtype=torch.int32, device=self.device)
            lpa_get_labels(self.h, out.data_ptr(), False)
            return out
        out = np.empty(self.n, np.int32)
        lpa_get_labels(self.h, out.ctypes.data, True)
        return out

    def modularity(self, labels=None) -> float:
        return lpa_modularity(self.h, None if labels is None else labels.data_ptr())

    def trace(self):
        return lpa_get_trace(self.h, self.max_iter)

    def get_state(self):
        lab = np.empty(self.n, np.int32)
        fl = np.empty(self.n, np.uint8)
        it = lpa_get_state(self.h, lab.ctypes.data, fl.ctypes.data, True)
        return lab, fl, it

    def set_state(self, labels, flags, iteration: int) -> None:
        labels = np.ascontiguousarray(labels, np.int32)
        flags = np.ascontiguousarray(flags, np.uint8)
        lpa_set_state(self.h, labels.ctypes.data, flags.ctypes.data, iteration, True)

    def iterations(self) -> int:
        return lpa_progress(self.h)[0]

    def finished(self) -> bool:
        return lpa_progress(self.h)[1]

    def profile(self, enable: bool = True) -> None:
        lpa_profile(self.h, enable)

    def move_ms(self) -> np.ndarray:
        return lpa_get_profile(self.h, self.max_iter)

    def memory_floor_ms(self, reps: int = 3) -> float:
        return lpa_memory_floor(self.h, reps)

    def memory(self) -> Tuple[int, int]:
        return lpa_memory(self.h)

    def close(self) -> None:
        if getattr(self, "h", None):
            lpa_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workspace_bytes(n: int, nnz: int, k: int = 8, max_iter: int = 20, mode: str = "det",
                    lane_max_degree: int = 0, rule: str = "mg", rescan: bool = False,
                    ranked: bool = False) -> int:
    """Device bytes one handle needs (for LPA(..., workspace=...))."""
    cfg = lpa_config_default()
    cfg.flags = (MODES[mode] | RULES[rule] | LPA_VALIDATE | (LPA_RESCAN if rescan else 0)
                 | (LPA_RANKED_LAYOUT if ranked else 0))
    cfg.lane_max_degree = lane_max_degree
    return lpa_workspace_bytes(n, nnz, k, max_iter, cfg)


class Batch:
    """Runs iterations of many LPA handles with one set of launches per
    iteration (see lpa_batch_create in include/lpa.h)."""

    def __init__(self, capacity: int, k: int = 8, mode: str = "det", check_every: int = 0,
                 stream=None, device=None, rule: str = "mg", rescan: bool = False,
                 hub_shared: bool = False, capture: bool = False, shared_vars: bool = False,
                 move_blocks_per_cu: int = 0):
        import torch
        cfg = lpa_config_default()
        cfg.move_blocks_per_cu = move_blocks_per_cu
        cfg.flags = (MODES[mode] | RULES[rule] | (LPA_RESCAN if rescan else 0)
                     | (LPA_HUB_SHARED if hub_shared else 0) | (LPA_CAPTURE if capture else 0)
                     | (LPA_SHARED_VARS if shared_vars else 0))
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        cfg.stream = stream.cuda_stream
        cfg.check_every = check_every
        self.capacity = capacity
        self.b = lpa_batch_create(capacity, k, cfg)

    def step(self, solvers) -> Tuple[int, bool]:
        return lpa_batch_step(self.b, [s.h for s in solvers])

    def run(self, solvers) -> int:
        return lpa_batch_run(self.b, [s.h for s in solvers])

    def reset(self, solvers) -> None:
        """lpa_reset of every solver with one kernel launch."""
        hs = [s.h for s in solvers]
        _check(load().lpa_batch_reset(self.b, _handle_array(hs), len(hs)), "lpa_batch_reset")

    def close(self) -> None:
        if getattr(self, "b", None):
            lpa_batch_free(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
