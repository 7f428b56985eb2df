"""Seeded synthetic graph inputs (CSR) for the LPA library, its tests and
its benchmark.

This module is input preparation only: it holds none of the label
propagation arithmetic.  The heavy generators are C (``graphgen.c``, built
into ``libgraphgen.so``); this file marshals their output into numpy arrays
and names the standard workloads:

* ``sbm1``    planted partition, n = 10,000 in 50 blocks of 200, p_in = 0.05,
              expected inter-block degree 1.0, unit weights;
* ``rmat(s)`` R-MAT scale s, edge factor 16, (a, b, c, d) =
              (0.57, 0.19, 0.19, 0.05), symmetrised, self-loops and
              duplicates dropped, no id permutation;
* ``grid``    R x C lattice with 5% edge deletions and 1% rewires;
* ``batch``   many planted-partition graphs of log-uniform size;
* weights either all 1.0 (``w = None``) or uniform in (0, 1] drawn per
  undirected edge so the graph stays symmetric.

The paper evaluates on SuiteSparse graphs that are not available here; these
generators stand in for them (R-MAT for web / social graphs, the rewired grid
for road networks).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")


class _GG(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.POINTER(ctypes.c_int32)),
                ("col", ctypes.POINTER(ctypes.c_int32))]


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.gg_sbm.argtypes = [ctypes.c_int32, i32p, ctypes.c_double, ctypes.c_double,
                             ctypes.c_uint64, ctypes.POINTER(_GG)]
        L.gg_rmat.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, ctypes.c_uint64, ctypes.POINTER(_GG)]
        L.gg_grid.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                              ctypes.c_uint64, ctypes.POINTER(_GG)]
        L.gg_free.argtypes = [ctypes.POINTER(_GG)]
        L.gg_free.restype = None
        L.gg_weights_uniform.argtypes = [ctypes.c_int32, i32p, i32p, ctypes.c_uint64,
                                         ctypes.POINTER(ctypes.c_float)]
        L.gg_weights_uniform.restype = None
        L.gg_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]
        L.gg_uniform.restype = ctypes.c_double
        _lib = L
    return _lib


@dataclass
class Graph:
    """Symmetric CSR graph; ``w is None`` means every weight is 1.0."""
    row_ptr: np.ndarray
    col: np.ndarray
    w: Optional[np.ndarray] = None
    name: str = ""

    @property
    def n(self) -> int:
        return len(self.row_ptr) - 1

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def _take(g: _GG, name: str) -> Graph:
    n, nnz = g.n, g.nnz
    rp = np.ctypeslib.as_array(g.row_ptr, shape=(n + 1,)).copy()
    col = (np.ctypeslib.as_array(g.col, shape=(nnz,)).copy() if nnz > 0
           else np.zeros(0, np.int32))
    _L().gg_free(ctypes.byref(g))
    return Graph(rp, col, None, name)


def uniform(seed: int, a: int, b: int) -> float:
    """Counter-based uniform draw in [0, 1) (the generators' own stream)."""
    return float(_L().gg_uniform(seed & (2**64 - 1), a & (2**64 - 1), b & (2**64 - 1)))


def sbm(block_sizes, p_in: float, p_out: float, seed: int, name: str = "sbm") -> Graph:
    sizes = np.asarray(block_sizes, dtype=np.int64)
    start = np.zeros(len(sizes) + 1, np.int32)
    start[1:] = np.cumsum(sizes)
    g = _GG()
    rc = _L().gg_sbm(len(sizes), start.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                     p_in, p_out, seed, ctypes.byref(g))
    if rc != 0:
        raise RuntimeError(f"gg_sbm failed ({rc})")
    return _take(g, name)


def sbm1(seed: int = 1) -> Graph:
    """Planted partition: 50 blocks of 200, p_in 0.05, inter-degree 1.0."""
    n, b = 10_000, 200
    return sbm([b] * (n // b), 0.05, 1.0 / (n - b), seed, name=f"sbm1-s{seed}")


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, seed: Optional[int] = None) -> Graph:
    seed = scale if seed is None else seed
    g = _GG()
    rc = _L().gg_rmat(scale, edge_factor, a, b, c, seed, ctypes.byref(g))
    if rc != 0:
        raise RuntimeError(f"gg_rmat failed ({rc})")
    return _take(g, f"rmat{scale}-ef{edge_factor}-s{seed}")


def grid(rows: int = 4096, cols: int = 4096, p_del: float = 0.05, p_rw: float = 0.01,
         seed: int = 4096) -> Graph:
    g = _GG()
    rc = _L().gg_grid(rows, cols, p_del, p_rw, seed, ctypes.byref(g))
    if rc != 0:
        raise RuntimeError(f"gg_grid failed ({rc})")
    return _take(g, f"grid{rows}x{cols}-s{seed}")


def weights_uniform(g: Graph, seed: int) -> np.ndarray:
    """fp32 weights in (0, 1], exact multiples of 2^-24, symmetric."""
    w = np.empty(g.nnz, np.float32)
    i32p = ctypes.POINTER(ctypes.c_int32)
    _L().gg_weights_uniform(g.n, g.row_ptr.ctypes.data_as(i32p), g.col.ctypes.data_as(i32p),
                            seed, w.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    return w


def with_uniform_weights(g: Graph, seed: int) -> Graph:
    return Graph(g.row_ptr, g.col, weights_uniform(g, seed), g.name + "-wU")


def permuted(g: Graph, seed: int) -> Graph:
    """The same graph with vertex ids relabelled by a seeded random
    permutation (rows re-sorted, weights kept on their edges): the
    locality-free copy of a generator whose ids carry structure."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(g.n).astype(np.int64)  # old id -> new id
    src = np.repeat(perm, np.diff(g.row_ptr))
    dst = perm[g.col.astype(np.int64)]
    order = np.argsort(src * g.n + dst, kind="stable")
    rp = np.zeros(g.n + 1, np.int64)
    np.add.at(rp, perm + 1, np.diff(g.row_ptr))
    rp = np.cumsum(rp).astype(np.int32)
    col = dst[order].astype(np.int32)
    w = g.w[order] if g.w is not None else None
    return Graph(rp, col, w, g.name + "-perm")


def from_edges(n: int, edges, name: str = "edges") -> Graph:
    """Tiny helper: symmetric CSR from an undirected edge list (Python)."""
    adj = [set() for _ in range(n)]
    for u, v in edges:
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    rp = np.zeros(n + 1, np.int32)
    for i in range(n):
        rp[i + 1] = rp[i] + len(adj[i])
    col = np.array([j for i in range(n) for j in sorted(adj[i])], dtype=np.int32)
    return Graph(rp, col, None, name)


def two_cliques(s: int) -> Graph:
    """Two s-cliques {0..s-1} and {s..2s-1} joined by the edge (s-1, s)."""
    edges = [(u, v) for u in range(s) for v in range(u + 1, s)]
    edges += [(s + u, s + v) for u in range(s) for v in range(u + 1, s)]
    edges.append((s - 1, s))
    return from_edges(2 * s, edges, name=f"two-cliques-{s}")


@dataclass
class BatchSpec:
    n: int
    blocks: int


def batch_specs(count: int = 512, seed: int = 512, n_lo: float = 1e3, n_hi: float = 2e5,
                b_lo: float = 8, b_hi: float = 200) -> List[BatchSpec]:
    """Sizes for the many-graph workload: n log-uniform in [n_lo, n_hi],
    block count log-uniform in [b_lo, b_hi] clipped to n // 16 (so a mean
    intra-block degree of 12 stays feasible)."""
    out = []
    for g in range(count):
        n = int(math.exp(math.log(n_lo) + uniform(seed, g, 0) * (math.log(n_hi) - math.log(n_lo))))
        b = int(math.exp(math.log(b_lo) + uniform(seed, g, 1) * (math.log(b_hi) - math.log(b_lo))))
        b = max(1, min(b, n // 16))
        out.append(BatchSpec(n, b))
    return out


def batch_graph(spec: BatchSpec, seed: int, index: int,
                intra_degree: float = 12.0, inter_degree: float = 2.0) -> Graph:
    """One planted-partition graph of the batch: near-equal blocks,
    p_in = intra/(s_b - 1), p_out = inter/(n - s_b)."""
    n, B = spec.n, spec.blocks
    sizes = [n // B + (1 if i < n % B else 0) for i in range(B)]
    sb = n / B
    p_in = min(1.0, intra_degree / max(sb - 1.0, 1.0))
    p_out = min(1.0, inter_degree / max(n - sb, 1.0)) if B > 1 else 0.0
    gseed = int(uniform(seed, index, 2) * 2**62)
    return sbm(sizes, p_in, p_out, gseed, name=f"batch{seed}-{index}")


def batch(count: int = 512, seed: int = 512, **kw) -> List[Graph]:
    return [batch_graph(s, seed, i) for i, s in enumerate(batch_specs(count, seed, **kw))]


# ------------------------------------------------------------------ ring + hubs
# A graph of closed form, so that one far beyond 2^31 CSR entries can be
# built directly in device memory and any of its rows recomputed on the host:
#   * lane vertices j = 0 .. L-1: neighbours (j + o) mod L for o = -r .. -1,
#     1 .. r (in that order), then the hub L + (j mod H);
#   * hubs L + t, t = 0 .. H-1: neighbours t, t + H, t + 2H, ... < L;
#   * weight of edge {i, j}: a hash of (min, max, seed), an exact multiple of
#     2^-24 in (0, 1], so both directions carry the same weight.
# nnz = L (2r + 2); vertex ids and offsets are int64 in every formula.

def _ring_weight(lo, hi, seed: int, xp):
    x = lo * 0x9E3779 + hi * 0x85EBCA + (seed & 0xFFFFFF) * 0x27D4EB
    x = x ^ (x >> 15)
    x = (x & 0xFFFFFF) * 0xC2B2AE
    x = x ^ (x >> 16)
    u = (x & 0xFFFFFF) + 1
    return u.astype(xp.float32) * np.float32(2.0 ** -24) if xp is np else \
        u.to(xp.float32) * (2.0 ** -24)


def ring_hubs_offsets(L: int, H: int, r: int) -> np.ndarray:
    """int64 row offsets [n + 1] of the ring + hubs graph (n = L + H)."""
    if not (0 < H <= L and L > 2 * r + 1 and r >= 1):
        raise ValueError("need 0 < H <= L and L > 2r + 1")
    rp = np.zeros(L + H + 1, np.int64)
    rp[1:L + 1] = np.arange(1, L + 1, dtype=np.int64) * (2 * r + 1)
    t = np.arange(H, dtype=np.int64)
    hub_deg = (L - t + H - 1) // H
    rp[L + 1:] = rp[L] + np.cumsum(hub_deg)
    return rp


def ring_hubs_rows(L: int, H: int, r: int, seed: int, vertices):
    """Rows of the given vertices as a compact CSR (row_ptr int64 over the
    list, col int32, w float32), recomputed from the closed form."""
    vs = np.asarray(vertices, np.int64)
    offs = np.concatenate([np.arange(-r, 0), np.arange(1, r + 1)]).astype(np.int64)
    cols, ws, lens = [], [], []
    for v in vs:
        if v < L:
            c = np.concatenate([(v + offs) % L, [L + v % H]]).astype(np.int64)
        else:
            c = np.arange(v - L, L, H, dtype=np.int64)
        lo, hi = np.minimum(c, v), np.maximum(c, v)
        cols.append(c.astype(np.int32))
        ws.append(_ring_weight(lo, hi, seed, np))
        lens.append(len(c))
    rp = np.zeros(len(vs) + 1, np.int64)
    rp[1:] = np.cumsum(lens)
    col = np.concatenate(cols) if cols else np.zeros(0, np.int32)
    w = np.concatenate(ws) if ws else np.zeros(0, np.float32)
    return rp, col, w


def ring_hubs_device(L: int, H: int, r: int, seed: int, device, chunk: int = 1 << 22):
    """The whole ring + hubs graph built with torch on `device`:
    (row_ptr int64 [n + 1], col int32 [nnz], w float32 [nnz])."""
    import torch

    rp_np = ring_hubs_offsets(L, H, r)
    nnz = int(rp_np[-1])
    rp = torch.from_numpy(rp_np).to(device)
    col = torch.empty(nnz, dtype=torch.int32, device=device)
    w = torch.empty(nnz, dtype=torch.float32, device=device)
    D = 2 * r + 1
    offs = torch.cat([torch.arange(-r, 0), torch.arange(1, r + 1)]).to(device=device,
                                                                        dtype=torch.int64)
    for j0 in range(0, L, chunk):
        j1 = min(L, j0 + chunk)
        j = torch.arange(j0, j1, dtype=torch.int64, device=device)
        c = torch.empty((j1 - j0, D), dtype=torch.int64, device=device)
        c[:, :2 * r] = torch.remainder(j[:, None] + offs[None, :], L)
        c[:, 2 * r] = L + torch.remainder(j, H)
        jj = j[:, None].expand(-1, D)
        x = _ring_weight(torch.minimum(c, jj), torch.maximum(c, jj), seed, torch)
        col[j0 * D:j1 * D] = c.reshape(-1).to(torch.int32)
        w[j0 * D:j1 * D] = x.reshape(-1)
        del c, jj, x
    for t in range(H):
        b, e = int(rp_np[L + t]), int(rp_np[L + t + 1])
        c = torch.arange(t, L, H, dtype=torch.int64, device=device)
        hub = torch.full_like(c, L + t)
        col[b:e] = c.to(torch.int32)
        w[b:e] = _ring_weight(c, hub, seed, torch)
    return rp, col, w
