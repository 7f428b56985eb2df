"""Autotuner for the launch shape of a graph.

Three knobs, none of which changes a det-mode result:

* the lane threshold S (``lane_max_degree``), which splits the vertices:
  degree <= S is scanned by one lane; above S a vertex is cut into S-entry
  segments whose partial sketches are merged (LPA_MODE_ASYNC) or fed by a
  whole wavefront in CSR order (LPA_MODE_DET).  It sets the degree bins;
* the move kernel's resident workgroups per compute unit
  (``move_blocks_per_cu``, 0 = as many as fit): fewer wavefronts hide less
  latency but share the caches among fewer rows in flight;
* optionally the ranked state layout (``LPA_RANKED_LAYOUT``), which costs 4
  bytes per CSR entry of device memory and is only tried when allowed.

``tune`` times candidates on the first iterations of the graph itself
(whole iterations, measured with device events around ``lpa_step``), one
knob after the other (S first, then the workgroups, then the layout), and
keeps the fastest per scanned entry.  ``tune_batch`` does the same for a
batch: one tuning per group of graphs of the same shape gives each graph its
S; the workgroup cap, which applies to a whole launch, is then chosen by
timing the batched solve.  Decisions are cached by GPU architecture and a
coarse signature of the graph (size and log-scale degree histogram), so
graphs of the same shape reuse them.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Iterable, List, Optional, Sequence, Tuple

import numpy as np

DEFAULT_CANDIDATES = (256, 512, 1024, 2048, 4096, 8192)
DEFAULT_BLOCKS = (0, 3, 2)


def arch_name(device=None) -> str:
    import torch
    props = torch.cuda.get_device_properties(device if device is not None else 0)
    return str(getattr(props, "gcnArchName", props.name))


def signature(row_ptr: np.ndarray, mode: str, k: int, rule: str = "mg", arch: str = "") -> str:
    """Coarse key of a graph's shape: log2 of n and nnz, and the share of
    CSR entries in rows of degree <= 16, 128, 1024 and 8192 (in tenths),
    with the mode, k, rule and GPU architecture."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    deg = np.diff(rp)
    n, nnz = len(deg), int(rp[-1]) if len(rp) else 0
    share = []
    for t in (16, 128, 1024, 8192):
        share.append(int(round(10.0 * deg[deg <= t].sum() / nnz)) if nnz else 0)
    return json.dumps([arch, mode, k, rule, int(np.log2(max(n, 1))), int(np.log2(max(nnz, 1))),
                       share])


def _time_config(lpa, torch, rp, col, w, cfg: Dict, k: int, mode: str, rule: str,
                 iters: int) -> float:
    """ns per scanned entry of the first `iters` iterations."""
    s = lpa.LPA(rp, col, w, k=k, mode=mode, rule=rule, lane_max_degree=cfg["lane_max_degree"],
                move_blocks_per_cu=cfg["move_blocks_per_cu"], ranked=cfg["ranked"])
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
        return float(t0.elapsed_time(t1)) * 1e6 / max(int(scanned.sum()), 1)
    finally:
        s.close()


def _key(cfg: Dict) -> str:
    return f"S={cfg['lane_max_degree']},blocks={cfg['move_blocks_per_cu']},ranked={int(cfg['ranked'])}"


def tune(row_ptr, col, weights=None, k: int = 8, mode: str = "async", rule: str = "mg",
         candidates: Iterable[int] = DEFAULT_CANDIDATES,
         blocks: Iterable[int] = DEFAULT_BLOCKS, allow_ranked: bool = False, iters: int = 2,
         cache: Optional[Dict[str, Dict]] = None) -> Dict:
    """Pick the launch shape for a device-resident graph (torch tensors, as
    for ``lpa.LPA``).  Returns {"lane_max_degree": S, "move_blocks_per_cu":
    b, "ranked": bool, "table": {config: ns per scanned entry}, "cached":
    bool}; ``cache`` (a dict, e.g. from ``load_cache``) is consulted and
    updated."""
    import torch

    from . import lpa

    rp_host = row_ptr.cpu().numpy() if hasattr(row_ptr, "cpu") else np.asarray(row_ptr)
    dev = row_ptr.device if hasattr(row_ptr, "is_cuda") and row_ptr.is_cuda else None
    key = signature(rp_host, mode, k, rule, arch_name(dev)) + (":ranked" if allow_ranked else "")
    if cache is not None and key in cache:
        out = dict(cache[key])
        out.update(table={}, cached=True)
        return out
    maxdeg = int(np.diff(rp_host.astype(np.int64)).max()) if len(rp_host) > 1 else 0
    table: Dict[str, float] = {}

    def timed(cfg):
        kk = _key(cfg)
        if kk not in table:
            table[kk] = _time_config(lpa, torch, row_ptr, col, weights, cfg, k, mode, rule, iters)
        return table[kk]

    best = {"lane_max_degree": 0, "move_blocks_per_cu": 0, "ranked": False}
    # 1. the lane threshold
    best_t = None
    for S in sorted(set(int(c) for c in candidates)):
        if S > 65536:
            continue
        if S > 2 * max(maxdeg, 1) and best_t is not None:
            break  # larger thresholds give the same bins as the previous one
        cfg = dict(best, lane_max_degree=S)
        t = timed(cfg)
        if best_t is None or t < best_t:
            best, best_t = cfg, t
    # 2. the resident workgroups, 3. the layout
    for b in blocks:
        cfg = dict(best, move_blocks_per_cu=int(b))
        t = timed(cfg)
        if t < best_t:
            best, best_t = cfg, t
    if allow_ranked:
        cfg = dict(best, ranked=True)
        t = timed(cfg)
        if t < best_t:
            best, best_t = cfg, t
    if cache is not None:
        cache[key] = dict(best)
    out = dict(best)
    out.update(table=table, cached=False)
    return out


def tune_batch(graphs: Sequence[Tuple], k: int = 8, mode: str = "det", rule: str = "mg",
               candidates: Iterable[int] = DEFAULT_CANDIDATES,
               blocks: Iterable[int] = DEFAULT_BLOCKS, iters: int = 2, reps: int = 2,
               cache: Optional[Dict[str, Dict]] = None) -> Dict:
    """Launch shape for a batch of device-resident graphs (a sequence of
    (row_ptr, col, weights) tensors): the graphs are grouped by signature,
    the largest graph of each group is tuned for its lane threshold (with
    ``tune``, workgroups left at the default), and every graph gets its
    group's S; then the workgroup cap of the launch is chosen by timing the
    whole batched solve with each candidate.  Returns {"lane_max_degree":
    [S per graph], "move_blocks_per_cu": b, "groups": {signature: S},
    "batch_ms": {b: ms per batched solve}}."""
    import torch

    from . import lpa

    arch = arch_name(graphs[0][0].device) if graphs else ""
    groups: Dict[str, List[int]] = {}
    for i, (rp, _, _) in enumerate(graphs):
        groups.setdefault(signature(rp.cpu().numpy(), mode, k, rule, arch), []).append(i)
    per_graph = [0] * len(graphs)
    chosen = {}
    for sig, idx in groups.items():
        rep = max(idx, key=lambda i: int(graphs[i][1].numel()))
        rp, col, w = graphs[rep]
        r = tune(rp, col, w, k=k, mode=mode, rule=rule, candidates=candidates, blocks=(),
                 iters=iters, cache=cache)
        chosen[sig] = r["lane_max_degree"]
        for i in idx:
            per_graph[i] = r["lane_max_degree"]
    stream = torch.cuda.current_stream(graphs[0][0].device) if graphs else None
    solvers = [lpa.LPA(rp, col, w, k=k, mode=mode, rule=rule, lane_max_degree=S, stream=stream)
               for (rp, col, w), S in zip(graphs, per_graph)]
    times = {}
    try:
        for b in blocks:
            batch = lpa.Batch(len(solvers), k=k, mode=mode, rule=rule, stream=stream,
                              move_blocks_per_cu=int(b))
            try:
                batch.reset(solvers)
                batch.run(solvers)  # warm
                t0 = torch.cuda.Event(enable_timing=True)
                t1 = torch.cuda.Event(enable_timing=True)
                t0.record(stream)
                for _ in range(reps):
                    batch.reset(solvers)
                    batch.run(solvers)
                t1.record(stream)
                t1.synchronize()
                times[int(b)] = float(t0.elapsed_time(t1)) / reps
            finally:
                batch.close()
    finally:
        for s in solvers:
            s.close()
    best_b = min(times, key=times.get) if times else 0
    return {"lane_max_degree": per_graph, "move_blocks_per_cu": best_b, "groups": chosen,
            "batch_ms": times}


def load_cache(path: str) -> Dict[str, Dict]:
    if os.path.exists(path):
        with open(path) as f:
            return {k: dict(v) for k, v in json.load(f).items()}
    return {}


def save_cache(cache: Dict[str, Dict], path: str) -> None:
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
