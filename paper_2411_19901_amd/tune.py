"""Autotuner for the degree-bin threshold of a graph.

The lane threshold S (``lane_max_degree``) splits the vertices: degree <= S
is scanned by one lane; above S a vertex is cut into S-entry segments whose
partial sketches are merged (LPA_MODE_ASYNC) or fed by a whole wavefront in
CSR order (LPA_MODE_DET).  The best S depends on the degree distribution.
``tune`` times each candidate on the first iterations of the graph itself
(whole iterations, measured with device events around ``lpa_step``) and
keeps the fastest per scanned entry.  In det mode the labels do not depend
on S, so tuning never changes a det result.  Results are cached by a coarse
signature of the graph (size and log-scale degree histogram) so that graphs
of the same shape reuse a decision.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, Optional, Tuple

import numpy as np

DEFAULT_CANDIDATES = (256, 512, 1024, 2048, 4096, 8192)


def signature(row_ptr: np.ndarray, mode: str, k: int, rule: str = "mg") -> str:
    """Coarse key of a graph's shape: log2 of n and nnz, and the share of
    CSR entries in rows of degree <= 16, 128, 1024 and 8192 (in tenths)."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    deg = np.diff(rp)
    n, nnz = len(deg), int(rp[-1]) if len(rp) else 0
    share = []
    for t in (16, 128, 1024, 8192):
        share.append(int(round(10.0 * deg[deg <= t].sum() / nnz)) if nnz else 0)
    return json.dumps([mode, k, rule, int(np.log2(max(n, 1))), int(np.log2(max(nnz, 1))), share])


def _time_candidate(lpa, torch, rp, col, w, S: int, k: int, mode: str, rule: str,
                    iters: int) -> Tuple[float, int]:
    s = lpa.LPA(rp, col, w, k=k, mode=mode, rule=rule, lane_max_degree=S)
    try:
        s.step()  # warm the code path and caches
        s.reset()
        stream = s.stream
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        done = False
        steps = 0
        while steps < iters and not done:
            _, done = s.step()
            steps += 1
        t1.record(stream)
        t1.synchronize()
        _, scanned = s.trace()
        return float(t0.elapsed_time(t1)), int(scanned.sum())
    finally:
        s.close()


def tune(row_ptr, col, weights=None, k: int = 8, mode: str = "async", rule: str = "mg",
         candidates: Iterable[int] = DEFAULT_CANDIDATES, iters: int = 2,
         cache: Optional[Dict[str, int]] = None) -> Dict:
    """Pick lane_max_degree for a device-resident graph (torch tensors, as
    for ``lpa.LPA``).  Returns {"lane_max_degree": S, "table": {S: ns per
    scanned entry}, "cached": bool}; ``cache`` (a dict, e.g. from
    ``load_cache``) is consulted and updated."""
    import torch

    from . import lpa

    rp_host = row_ptr.cpu().numpy() if hasattr(row_ptr, "cpu") else np.asarray(row_ptr)
    key = signature(rp_host, mode, k, rule)
    if cache is not None and key in cache:
        return {"lane_max_degree": int(cache[key]), "table": {}, "cached": True}
    maxdeg = int(np.diff(rp_host.astype(np.int64)).max()) if len(rp_host) > 1 else 0
    table = {}
    for S in sorted(set(int(c) for c in candidates)):
        if S > 65536:
            continue
        if S > 2 * max(maxdeg, 1) and table:
            break  # larger thresholds give the same bins as the previous one
        ms, scanned = _time_candidate(lpa, torch, row_ptr, col, weights, S, k, mode, rule, iters)
        table[S] = ms * 1e6 / max(scanned, 1)
    best = min(table, key=table.get)
    if cache is not None:
        cache[key] = best
    return {"lane_max_degree": best, "table": table, "cached": False}


def load_cache(path: str) -> Dict[str, int]:
    if os.path.exists(path):
        with open(path) as f:
            return {k: int(v) for k, v in json.load(f).items()}
    return {}


def save_cache(cache: Dict[str, int], path: str) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
