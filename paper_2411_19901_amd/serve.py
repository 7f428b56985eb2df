"""Serving loop: continuous batching of label-propagation requests.

Requests (one graph each) arrive at any time.  A request is admitted when a
resident slot is free and its device memory (CSR, weights, library
workspace) fits in the free HBM the budget allows; its CSR and label state
then stay on the device.  Every tick runs one iteration of every resident
graph with a single batched launch (``lpa_batch_step``), so requests that
arrive while others run join at the next iteration boundary and their work
overlaps on the GPU.  Finished graphs copy their labels to the host, free
their memory and leave.  In det mode each result is bit-identical to a solo
run of the same graph, whatever the mix.

With ``overlap_admission`` a thread of the server admits requests while the
ticks run: the backend copies the CSR to the device and builds the handle
(degree binning) on an admission stream of its own, then moves the handle to
the compute stream, and the next tick picks it up.  The copies and the
binning of new requests then overlap the iterations of resident ones
instead of stalling them.

The scheduler is independent of the device: ``Backend`` does the GPU work,
and tests drive the same scheduler with a CPU stand-in backend and a fake
free-memory probe.
"""
from __future__ import annotations

import collections
import math
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, Deque, Dict, List, Optional

import numpy as np


@dataclass
class Request:
    rid: int
    row_ptr: np.ndarray
    col: np.ndarray
    w: Optional[np.ndarray]
    arrival: float
    admitted: float = math.nan
    finished: float = math.nan
    labels: Optional[np.ndarray] = None
    iterations: int = 0
    bytes_needed: int = 0
    state: object = None  # backend-owned solver
    done_event: threading.Event = field(default_factory=threading.Event)

    @property
    def n(self) -> int:
        return len(self.row_ptr) - 1

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


class Backend:
    """GPU backend: one liblpa handle per resident request, one batch object
    for the launches; torch supplies device memory and the stream."""

    def __init__(self, k: int = 8, mode: str = "det", tol: float = 0.05, max_iter: int = 20,
                 capacity: int = 256, device: int = 0):
        import torch

        from . import lpa
        self.torch = torch
        self.lpa = lpa
        self.k, self.mode, self.tol, self.max_iter = k, mode, tol, max_iter
        self.device = torch.device(f"cuda:{device}")
        self.stream = torch.cuda.current_stream(self.device)
        # admission work (host-to-device copies, lpa_init) when it overlaps
        # the ticks; default priority like every other stream here
        self.admit_stream = torch.cuda.Stream(self.device)
        self.batch = lpa.Batch(capacity, k=k, mode=mode, stream=self.stream)

    def bytes_needed(self, req: Request) -> int:
        ws = self.lpa.workspace_bytes(req.n, req.nnz, k=self.k, max_iter=self.max_iter,
                                      mode=self.mode)
        graph = 4 * (req.n + 1) + 4 * req.nnz + (4 * req.nnz if req.w is not None else 0)
        return ws + graph

    def free_bytes(self) -> int:
        return int(self.torch.cuda.mem_get_info(self.device)[0])

    def admit(self, req: Request, overlap: bool = False):
        """Device state of one request.  overlap: called by the admission
        thread; the copies and lpa_init run on the admission stream (lpa_init
        synchronises it, so the handle is complete when it returns), then the
        handle moves to the compute stream."""
        t = self.torch
        stream = self.admit_stream if overlap else self.stream
        with t.cuda.device(self.device), t.cuda.stream(stream):
            def up(a):
                host = t.from_numpy(a)
                if overlap:
                    host = host.pin_memory()
                return host.to(self.device, non_blocking=overlap)
            rp = up(req.row_ptr)
            col = up(req.col)
            w = up(req.w) if req.w is not None else None
            ws = t.empty(self.lpa.workspace_bytes(req.n, req.nnz, k=self.k,
                                                  max_iter=self.max_iter, mode=self.mode),
                         dtype=t.uint8, device=self.device)
            s = self.lpa.LPA(rp, col, w, k=self.k, tol=self.tol, max_iter=self.max_iter,
                             mode=self.mode, stream=stream, workspace=ws)
        if overlap:
            s.set_stream(self.stream)
        return s

    def step(self, solvers) -> None:
        if solvers:
            self.batch.step(solvers)

    def finished(self, solver) -> bool:
        return solver.finished()

    def result(self, solver):
        return solver.labels(device=False), solver.iterations()

    def release(self, solver) -> None:
        solver.close()

    def close(self) -> None:
        self.batch.close()


class Server:
    """Continuous-batching scheduler over a Backend.

    ``submit`` may be called from any thread; ``tick`` (or ``serve_forever``
    in a thread) does the work.  ``hbm_reserve`` bytes of free device memory
    are always left unused; ``max_resident`` bounds the batch."""

    def __init__(self, backend, max_resident: int = 64, hbm_reserve: int = 1 << 30,
                 free_bytes: Optional[Callable[[], int]] = None, clock=time.perf_counter,
                 overlap_admission: bool = False):
        self.backend = backend
        self.max_resident = max_resident
        self.hbm_reserve = hbm_reserve
        self.free_bytes = free_bytes or backend.free_bytes
        self.clock = clock
        self.pending: Deque[Request] = collections.deque()
        self.resident: List[Request] = []
        self.completed: List[Request] = []
        self.lock = threading.Lock()
        self.next_id = 0
        self.ticks = 0
        self.waits_for_memory = 0
        self._stop = False
        # overlapped admission: requests being admitted, and admitted ones
        # that the next tick adds to the resident set
        self.overlap_admission = overlap_admission
        self.preparing = 0
        self.ready: Deque[Request] = collections.deque()
        self._cv = threading.Condition(self.lock)
        self._adm_stop = False
        self._adm_error: Optional[BaseException] = None
        self._adm_thread: Optional[threading.Thread] = None
        self._waited = -1
        if overlap_admission:
            self._adm_thread = threading.Thread(target=self._admission_loop, daemon=True)
            self._adm_thread.start()

    def submit(self, row_ptr, col, w=None, arrival: Optional[float] = None) -> Request:
        with self.lock:
            req = Request(self.next_id, np.ascontiguousarray(row_ptr, np.int32),
                          np.ascontiguousarray(col, np.int32),
                          None if w is None else np.ascontiguousarray(w, np.float32),
                          self.clock() if arrival is None else arrival)
            self.next_id += 1
            req.bytes_needed = self.backend.bytes_needed(req)
            self.pending.append(req)
            self._cv.notify_all()
        return req

    def _admit(self) -> None:
        while True:
            with self.lock:
                if not self.pending or len(self.resident) >= self.max_resident:
                    return
                req = self.pending[0]
                if req.arrival > self.clock():
                    return  # not arrived yet (pre-scheduled arrivals)
                if req.bytes_needed + self.hbm_reserve > self.free_bytes():
                    self.waits_for_memory += 1
                    return  # head of line waits until memory frees up
                self.pending.popleft()
            req.state = self.backend.admit(req)
            req.admitted = self.clock()
            self.resident.append(req)

    def _admissible(self) -> Optional[Request]:
        """Head of the queue if it has arrived and fits (slots and memory);
        called with the lock held."""
        if not self.pending:
            return None
        if len(self.resident) + self.preparing + len(self.ready) >= self.max_resident:
            return None
        req = self.pending[0]
        if req.arrival > self.clock():
            return None
        if req.bytes_needed + self.hbm_reserve > self.free_bytes():
            if self._waited != req.rid:  # count each request's wait once
                self._waited = req.rid
                self.waits_for_memory += 1
            return None
        return req

    def _admission_loop(self) -> None:
        while True:
            with self._cv:
                while not self._adm_stop:
                    req = self._admissible()
                    if req is not None:
                        break
                    # wake on submit / retire, or to see a future arrival come due
                    self._cv.wait(timeout=5e-4)
                if self._adm_stop:
                    return
                self.pending.popleft()
                self.preparing += 1
            try:
                state = self.backend.admit(req, overlap=True)
            except BaseException as e:  # handed to the tick loop, which raises it
                with self._cv:
                    self._adm_error = e
                    self.preparing -= 1
                return
            with self._cv:
                req.state = state
                req.admitted = self.clock()
                self.ready.append(req)
                self.preparing -= 1

    def _take_ready(self) -> None:
        with self._cv:
            if self._adm_error is not None:
                raise RuntimeError("admission failed") from self._adm_error
            while self.ready:
                self.resident.append(self.ready.popleft())

    def _retire(self) -> None:
        keep = []
        for req in self.resident:
            if self.backend.finished(req.state):
                req.labels, req.iterations = self.backend.result(req.state)
                self.backend.release(req.state)
                req.state = None
                req.finished = self.clock()
                self.completed.append(req)
                req.done_event.set()
            else:
                keep.append(req)
        with self._cv:
            self.resident = keep
            self._cv.notify_all()

    def _busy(self) -> bool:
        with self.lock:
            return bool(self.resident or self.pending or self.preparing or self.ready)

    def tick(self) -> bool:
        """Admit, run one batched iteration, retire.  Returns False when
        nothing is resident (requests may still be queued or being admitted:
        see ``_busy``)."""
        if self.overlap_admission:
            self._take_ready()
        else:
            self._admit()
        if not self.resident:
            return False
        self.backend.step([r.state for r in self.resident])
        self.ticks += 1
        self._retire()
        return True

    def run_until_idle(self, max_ticks: int = 10_000_000) -> None:
        for _ in range(max_ticks):
            if not self.tick():
                if not self._busy():
                    return
                time.sleep(0)  # waiting for an arrival or an admission

    def serve_forever(self, poll: float = 1e-4) -> None:
        while not self._stop:
            if not self.tick():
                time.sleep(poll)

    def stop(self) -> None:
        self._stop = True
        self.close()

    def close(self) -> None:
        """Stop the admission thread (requests it has not started stay queued)."""
        if self._adm_thread is not None:
            with self._cv:
                self._adm_stop = True
                self._cv.notify_all()
            self._adm_thread.join()
            self._adm_thread = None

    def latency_stats(self) -> Dict[str, float]:
        lat = np.array([r.latency for r in self.completed], dtype=np.float64)
        if lat.size == 0:
            return {"count": 0}
        return {"count": int(lat.size), "p50_s": float(np.percentile(lat, 50)),
                "p99_s": float(np.percentile(lat, 99)), "mean_s": float(lat.mean())}


def poisson_arrivals(count: int, rate: float, seed: int, start: float = 0.0) -> np.ndarray:
    """Arrival times of a Poisson process of `rate` requests per second."""
    rng = np.random.default_rng(seed)
    return start + np.cumsum(rng.exponential(1.0 / rate, size=count))
