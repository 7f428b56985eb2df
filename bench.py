#!/usr/bin/env python3
"""Benchmark of the label-propagation hot path on one MI355X.

Default workload: R-MAT scale 24, edge factor 16 (a, b, c, d = 0.57, 0.19,
0.19, 0.05; symmetrised, self-loops and duplicates dropped; ~16.8M vertices,
~0.52B CSR entries) with fp32 weights uniform in (0, 1], k = 8 sketch slots,
asynchronous mode, tol 0.05, at most 20 iterations, pick-less every 8.

One step = one full solve of that graph from iteration 0: lpa_reset +
lpa_run (every iteration until convergence: neighbourhood scans, sketches,
label updates, pruning flags, changed counters, convergence tests).  The
graph is generated on the host, copied to HBM and binned by degree
(lpa_init) before the timed region.

value = CSR entries scanned over the timed steps / timed wall time, in
GTEPS (1e9 edges per second).  roofline: the move kernel, with 12 bytes
per scanned entry (column index 4 + weight 4 + gathered label 4) divided by
the kernel time measured with HIP events on the library's stream, against
the 8 TB/s HBM peak.  cpu_baseline: the CPU oracle (CSR-order sketches, all
host threads) choosing labels for a random vertex sample of the same graph
at iteration 0.
"""
import argparse
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LPA edges/sec per iteration (GTEPS) + % HBM roofline; batched graphs/s, p99"
HBM_PEAK_GBPS = 8000.0
BYTES_PER_EDGE = 12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def traffic_from_profiles(kernel: str, workload: str, src_digest: str):
    """HBM bytes per launch of `kernel` measured with rocprofv3 FETCH_SIZE and
    WRITE_SIZE counters (each scaled by the same counter's reading for a
    device copy of known size), if a summary in profiles/ was taken on this
    kernel source, kernel and workload; else None."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    for name in sorted(os.listdir(pdir)):
        if not name.endswith(".md"):
            continue
        text = open(os.path.join(pdir, name)).read()
        m = {k: v.strip() for k, v in re.findall(r"^- (\w+): (.+)$", text, re.M)}
        if (m.get("traffic_kernel") == kernel and m.get("traffic_workload") == workload
                and m.get("source_digest") == src_digest and "traffic_bytes_per_launch" in m):
            return float(m["traffic_bytes_per_launch"])
    return None


def source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in ("move.hip", "wave.h", "lpa_internal.h"):
        with open(os.path.join(ROOT, "paper_2411_19901_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(g, k, seconds, rng_seed=0, exact_run=False):
    """Oracle label choice (iteration 0, CSR order; k slots, or k=-1 for the
    vote of Algorithm 3) on a random vertex sample sized for about `seconds`
    of work on all host threads, plus the same on one thread for a sample a
    quarter as long.  exact_run: also the oracle's whole Jacobi run with the
    exact rule of Eq. 3 on the full graph (all host threads), with the
    modularity of its labels: the quality reference of the async mode."""
    import numpy as np
    import oracle

    deg = g.degrees()
    verts_all = np.nonzero(deg > 0)[0].astype(np.int32)
    rng = np.random.default_rng(rng_seed)
    C = np.arange(g.n, dtype=np.int32)
    nt = oracle.max_threads()

    def timed(sample, threads):
        t = time.perf_counter()
        oracle.lpa_choose(g.row_ptr, g.col, g.w, k, True, C, sample, nthreads=threads)
        return max(time.perf_counter() - t, 1e-6)

    def sized(rate, secs):
        frac = min(1.0, rate * secs / max(1, g.nnz))
        m = max(1000, int(frac * len(verts_all)))
        return np.sort(rng.choice(verts_all, size=min(m, len(verts_all)), replace=False))

    # calibrate on a small sample, then size the measured ones
    probe = rng.choice(verts_all, size=min(len(verts_all), 20000), replace=False)
    rate1 = deg[probe].sum() / timed(probe, 1)
    rate = deg[probe].sum() / timed(probe, nt)
    sample = sized(rate, seconds)
    edges = int(deg[sample].sum())
    dt = timed(sample, nt)
    one = sized(rate1, seconds / 4)
    edges1 = int(deg[one].sum())
    dt1 = timed(one, 1)
    what = f"k={k}" if k > 0 else "vote of Algorithm 3"
    # the exact rule of Eq. 3 (dense per-thread accumulator), same sample size
    ex = sized(rate, seconds / 4)
    edges_x = int(deg[ex].sum())
    tx = time.perf_counter()
    oracle.lpa_choose(g.row_ptr, g.col, g.w, 0, True, C, ex)
    dtx = max(time.perf_counter() - tx, 1e-6)
    res_exact = None
    if exact_run:
        tx = time.perf_counter()
        lab, it, _, sc = oracle.lpa_run(g.row_ptr, g.col, g.w, k=0)
        dt_run = max(time.perf_counter() - tx, 1e-6)
        res_exact = {"q": round(oracle.modularity(g.row_ptr, g.col, g.w, lab), 6),
                     "iterations": int(it), "seconds": round(dt_run, 2),
                     "GTEPS": round(int(sc.sum()) / dt_run / 1e9, 4),
                     "communities": int(len(np.unique(lab))),
                     "what": "whole Jacobi run with the exact argmax of Eq. 3 (tol 0.05, "
                             "max 20 iterations, pick-less every 8), full graph"}
    out = {"value": round(edges / dt / 1e9, 4), "unit": "GTEPS", "cores": int(nt),
            "kind": "oracle",
            "sample": f"{len(sample)} uniformly sampled non-isolated vertices ({edges} CSR entries, "
                      f"{100.0 * edges / g.nnz:.1f}% of the graph), one iteration-0 label choice each, "
                      f"{what}, {dt:.1f} s on {nt} threads",
            "single_core": {"value": round(edges1 / dt1 / 1e9, 4), "unit": "GTEPS", "cores": 1,
                            "sample": f"{len(one)} vertices ({edges1} CSR entries), {dt1:.1f} s"},
            "exact_rule": {"value": round(edges_x / dtx / 1e9, 4), "unit": "GTEPS", "cores": int(nt),
                           "sample": f"{len(ex)} vertices ({edges_x} CSR entries), exact argmax "
                                     f"of Eq. 3, {dtx:.1f} s"}}
    if res_exact is not None:
        out["exact_rule_run"] = res_exact
    return out


def timed_solves(solver, steps, warmup, tag=""):
    """Warm-up solves, then `steps` timed solves (lpa_reset + lpa_run each)
    with the move kernel's HIP events on; returns the whole-job and kernel
    figures of the timed region."""
    import torch

    for i in range(warmup):
        solver.reset()
        it = solver.run()
        log(f"[bench]{tag} warmup {i}: {it} iterations")
    edges_total, kernel_ms, launches, iters = 0, 0.0, 0, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        solver.reset()
        it = solver.run()
        _, sc = solver.trace()
        ms = solver.move_ms()
        iters.append(it)
        edges_total += int(sc.sum())
        kernel_ms += float(ms.sum())
        launches += len(ms)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    log(f"[bench]{tag} timed {steps} steps in {elapsed:.3f}s; iterations {iters}")
    return {"edges": edges_total, "elapsed": elapsed, "kernel_ms": kernel_ms,
            "launches": launches, "iters": iters}


def build_graph(args):
    from paper_2411_19901_amd import inputs
    t = time.perf_counter()
    if args.graph == "rmat":
        g = inputs.rmat(args.scale, 16, seed=args.scale)
        name = f"rmat{args.scale}-ef16"
    elif args.graph == "grid":
        g = inputs.grid(4096, 4096, 0.05, 0.01, seed=4096)
        name = "grid4096-del5-rw1"
    elif args.graph == "sbm1":
        g = inputs.sbm1(1)
        name = "sbm1"
    else:
        raise SystemExit(f"unknown graph {args.graph}")
    if args.weights == "uniform":
        g = inputs.with_uniform_weights(g, args.scale if args.graph == "rmat" else 7)
        name += "-wU(0,1]"
    else:
        name += "-w1"
    if getattr(args, "permute", False):
        g = inputs.permuted(g, 1000 + args.scale)
        name += "-perm"
    log(f"[bench] generated {name}: n={g.n} nnz={g.nnz} in {time.perf_counter() - t:.1f}s")
    return g, name


def bench_batch(args, cpu_sample: int = 0):
    """512 planted-partition graphs (sizes log-uniform 1e3..2e5) solved in det
    mode: one batched launch sequence vs one lpa_run per graph, identical
    labels required.  cpu_sample > 0: the cpu_baseline leg solves that many of
    the graphs with the CPU oracle (timed) and compares their labels."""
    import hashlib

    import numpy as np
    import torch
    from paper_2411_19901_amd import inputs, lpa

    dev = torch.device("cuda:0")
    t = time.perf_counter()
    specs = inputs.batch_specs(args.batch_graphs, 512)
    gs = [inputs.batch_graph(sp, 512, i) for i, sp in enumerate(specs)]
    gen_s = time.perf_counter() - t
    nv, ne = sum(g.n for g in gs), sum(g.nnz for g in gs)
    log(f"[bench] batch of {len(gs)} graphs: {nv} vertices, {ne} entries, generated in {gen_s:.1f}s")
    stream = torch.cuda.current_stream(dev)
    t = time.perf_counter()
    tensors = [(torch.from_numpy(g.row_ptr).to(dev), torch.from_numpy(g.col).to(dev), None)
               for g in gs]
    solvers = [lpa.LPA(rp, col, w, k=args.k, tol=args.tol, max_iter=args.max_iter,
                       mode=args.mode, stream=stream) for rp, col, w in tensors]
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t
    batch = lpa.Batch(len(solvers), k=args.k, mode=args.mode, stream=stream,
                      capture=args.capture)
    tuned = None
    if args.autotune:
        # per-graph lane thresholds (one tuning per shape group) and the
        # launch's workgroup cap, chosen untimed; a second set of handles
        from paper_2411_19901_amd import tune
        t = time.perf_counter()
        tuned = tune.tune_batch(tensors, k=args.k, mode=args.mode)
        tune_s = time.perf_counter() - t
        log(f"[bench] batch autotune in {tune_s:.1f}s: groups {tuned['groups']}, "
            f"workgroups {tuned['move_blocks_per_cu']} ({tuned['batch_ms']})")
        t_solvers = [lpa.LPA(rp, col, w, k=args.k, tol=args.tol, max_iter=args.max_iter,
                             mode=args.mode, stream=stream, lane_max_degree=S)
                     for (rp, col, w), S in zip(tensors, tuned["lane_max_degree"])]
        t_batch = lpa.Batch(len(t_solvers), k=args.k, mode=args.mode, stream=stream,
                            capture=args.capture,
                            move_blocks_per_cu=tuned["move_blocks_per_cu"])

    def solo():
        for s in solvers:
            s.reset()
            s.run()

    def batched():
        batch.reset(solvers)
        batch.run(solvers)

    def batched_tuned():
        t_batch.reset(t_solvers)
        t_batch.run(t_solvers)

    timings = {}
    legs = [("solo", solo, solvers), ("batched", batched, solvers)]
    if tuned is not None:
        legs.append(("tuned", batched_tuned, t_solvers))
    for name, fn, which in legs:
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        timings[name] = (time.perf_counter() - t0) / args.steps
        h = hashlib.sha256()
        for s in which:
            h.update(s.labels(device=False).tobytes())
        timings[name + "_digest"] = h.hexdigest()[:16]
        timings[name + "_iters"] = [s.iterations() for s in which]
    same = (timings["solo_digest"] == timings["batched_digest"]
            and timings["solo_iters"] == timings["batched_iters"])
    if tuned is not None:
        same = (same and timings["tuned_digest"] == timings["solo_digest"]
                and timings["tuned_iters"] == timings["solo_iters"])
    scanned = sum(int(s.trace()[1].sum()) for s in solvers)
    res = {
        "metric": "batched graphs/s", "value": round(len(gs) / timings["batched"], 2),
        "unit": "graphs/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(timings["batched"] * 1e3, 3), "higher_is_better": True,
        "scaling": "strong", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"sbm-batch{len(gs)}-{args.mode}-k{args.k}", "graphs": len(gs),
                   "vertices": nv, "nnz": ne, "k": args.k, "mode": args.mode,
                   "captured": bool(args.capture),
                   "step": "lpa_batch_reset + lpa_batch_run over all of them (solo: lpa_reset + "
                           "lpa_run per graph)"},
        "solo_graphs_per_s": round(len(gs) / timings["solo"], 2),
        "solo_ms_per_step": round(timings["solo"] * 1e3, 3),
        "speedup_vs_solo": round(timings["solo"] / timings["batched"], 3),
        "identical_labels_and_iterations": bool(same),
        "GTEPS_batched": round(scanned / timings["batched"] / 1e9, 3),
        "init_s": round(init_s, 2), "gen_s": round(gen_s, 1),
        "max_iterations": max(timings["batched_iters"]),
    }
    if tuned is not None:
        # the headline is the tuned launch; the default shape beside it
        res["value"] = round(len(gs) / timings["tuned"], 2)
        res["ms_per_step"] = round(timings["tuned"] * 1e3, 3)
        res["speedup_vs_solo"] = round(timings["solo"] / timings["tuned"], 3)
        res["default_shape_graphs_per_s"] = round(len(gs) / timings["batched"], 2)
        res["autotune"] = {"move_blocks_per_cu": tuned["move_blocks_per_cu"],
                           "lane_max_degree_by_group": tuned["groups"],
                           "batch_ms_by_blocks": {str(b): round(v, 3)
                                                  for b, v in tuned["batch_ms"].items()},
                           "seconds": round(tune_s, 2)}
        res["config"]["autotuned"] = True
        t_batch.close()
        for s in t_solvers:
            s.close()
    if cpu_sample > 0:
        res["cpu_baseline"] = batch_cpu_baseline(gs, solvers, args, cpu_sample)
    batch.close()
    for s in solvers:
        s.close()
    return res


def batch_cpu_baseline(gs, solvers, args, count):
    """The oracle's whole run (all host threads) on every (512 / count)-th
    graph of the batch: graphs/s on the host, and whether its labels and
    iteration counts equal the batched GPU run's."""
    import numpy as np
    import oracle

    idx = list(range(0, len(gs), max(1, len(gs) // count)))[:count]
    t = time.perf_counter()
    same = True
    for i in idx:
        g = gs[i]
        ref, it, _, _ = oracle.lpa_run(g.row_ptr, g.col, None, k=args.k, tol=args.tol,
                                       max_iter=args.max_iter)
        same = same and bool(np.array_equal(ref, solvers[i].labels(device=False))
                             and it == solvers[i].iterations())
    dt = time.perf_counter() - t
    return {"value": round(len(idx) / dt, 2), "unit": "graphs/s", "cores": int(oracle.max_threads()),
            "kind": "oracle",
            "sample": f"{len(idx)} of the {len(gs)} graphs (every {len(gs) // len(idx)}th), whole "
                      f"det run each, {dt:.1f} s",
            "labels_equal_gpu_batched": same}


def bench_serve(args):
    """Poisson stream of mixed requests (70% planted-partition graphs of
    1e3..1e5 vertices, 30% R-MAT scale 14..max, weights uniform (0, 1]) served
    with continuous batching vs one request at a time in arrival order."""
    import numpy as np
    import torch
    from paper_2411_19901_amd import inputs, lpa
    from paper_2411_19901_amd.serve import Backend, Server, poisson_arrivals

    dev = torch.device("cuda:0")
    rng_u = lambda i, j: inputs.uniform(5, i, j)  # noqa: E731
    t = time.perf_counter()
    gs = []
    for i in range(args.requests):
        if rng_u(i, 0) < 0.7:
            n = int(math.exp(math.log(1e3) + rng_u(i, 1) * (math.log(1e5) - math.log(1e3))))
            b = max(1, min(int(math.exp(math.log(8) + rng_u(i, 2) * (math.log(200) - math.log(8)))),
                           n // 16))
            g = inputs.batch_graph(inputs.BatchSpec(n, b), 5, i)
        else:
            g = inputs.rmat(14 + int(rng_u(i, 3) * (args.serve_max_scale - 13)), 16, seed=1000 + i)
        gs.append(inputs.with_uniform_weights(g, i))
    gen_s = time.perf_counter() - t
    log(f"[bench] {len(gs)} requests generated in {gen_s:.1f}s "
        f"({sum(g.nnz for g in gs)} entries)")
    be = Backend(k=args.k, mode=args.mode, tol=args.tol, max_iter=args.max_iter,
                 capacity=args.serve_slots)
    overlap = not args.serve_no_overlap
    # sequential service: one request at a time, each solved alone
    seq_labels, seq_ms = [], []
    for _ in range(args.warmup):
        s = be.admit(Server(be).submit(gs[0].row_ptr, gs[0].col, gs[0].w))
        s.run()
        s.close()
    for g in gs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        srv1 = Server(be, max_resident=1, hbm_reserve=0)
        srv1.submit(g.row_ptr, g.col, g.w, arrival=0.0)
        srv1.run_until_idle()
        seq_ms.append((time.perf_counter() - t0) * 1e3)
        seq_labels.append(srv1.completed[0].labels)
    mu_seq = 1e3 / np.mean(seq_ms)  # requests per second, sequential
    loads = [float(x) for x in args.serve_loads.split(",")]
    per_load = []
    same = True
    for li, load in enumerate(loads):
        rate = load * mu_seq
        # sequential latency under the same Poisson arrivals (FIFO queue)
        arr = poisson_arrivals(len(gs), rate, seed=5 + li)
        fin, clock = [], 0.0
        for a, ms in zip(arr, seq_ms):
            clock = max(clock, a) + ms / 1e3
            fin.append(clock)
        seq_lat = np.array(fin) - arr
        seq_span = fin[-1] - arr[0]
        # continuous batching
        srv = Server(be, max_resident=args.serve_slots, hbm_reserve=1 << 30,
                     overlap_admission=overlap)
        t0 = srv.clock()
        for g, a in zip(gs, arr):
            srv.submit(g.row_ptr, g.col, g.w, arrival=t0 + float(a))
        srv.run_until_idle()
        srv.close()
        span = max(r.finished for r in srv.completed) - (t0 + arr[0])
        by_id = {r.rid: r for r in srv.completed}
        same = same and all(np.array_equal(by_id[i].labels, seq_labels[i]) for i in range(len(gs)))
        st = srv.latency_stats()
        per_load.append({
            "load_vs_sequential": load, "arrival_rate_per_s": round(rate, 2),
            "graphs_per_s": round(len(gs) / span, 2), "span_ms": round(span * 1e3, 3),
            "p50_ms": round(st["p50_s"] * 1e3, 3), "p99_ms": round(st["p99_s"] * 1e3, 3),
            "ticks": srv.ticks, "memory_waits": srv.waits_for_memory,
            "sequential": {"graphs_per_s": round(len(gs) / seq_span, 2),
                           "p50_ms": round(float(np.percentile(seq_lat, 50)) * 1e3, 3),
                           "p99_ms": round(float(np.percentile(seq_lat, 99)) * 1e3, 3)}})
        log(f"[bench] load {load}: {per_load[-1]}")
    head = max(per_load, key=lambda r: r["load_vs_sequential"])
    res = {
        "metric": "served graphs/s (p50/p99 latency)", "value": head["graphs_per_s"],
        "unit": "graphs/s", "n_gpus": 1, "steps": 1, "warmup": args.warmup,
        "ms_per_step": head["span_ms"], "higher_is_better": True, "scaling": "strong",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"serve-mix{len(gs)}-{args.mode}-k{args.k}", "requests": len(gs),
                   "arrival_rate_per_s": head["arrival_rate_per_s"],
                   "load_vs_sequential": head["load_vs_sequential"],
                   "slots": args.serve_slots, "rmat_max_scale": args.serve_max_scale,
                   "overlapped_admission": overlap},
        "p50_ms": head["p50_ms"], "p99_ms": head["p99_ms"],
        "sequential_graphs_per_s_capacity": round(mu_seq, 2),
        "mean_service_ms": round(float(np.mean(seq_ms)), 3),
        "loads": per_load,
        "identical_to_alone": bool(same), "gen_s": round(gen_s, 1),
    }
    be.close()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--graph", default="rmat", choices=["rmat", "grid", "sbm1", "ring"],
                    help="ring: the closed-form ring-plus-hubs graph of 2.23e9 CSR entries "
                         "(L = 36M lane vertices of degree 61, 64 hubs), built in device "
                         "memory with int64 row offsets")
    ap.add_argument("--scale", type=int, default=24)
    ap.add_argument("--weights", default="uniform", choices=["uniform", "unit"])
    ap.add_argument("--k", type=int, default=8)
    ap.add_argument("--permute", action="store_true",
                    help="relabel the vertices by a seeded random permutation (R-MAT ids carry "
                         "locality; this is the locality-free copy)")
    ap.add_argument("--host-csr", action="store_true",
                    help="keep row_ptr / col / weights in pinned host memory (the kernels read "
                         "them over the host link; only the O(|V|) state is in device memory)")
    ap.add_argument("--autotune", action="store_true",
                    help="pick lane_max_degree by timing candidates on the graph (untimed)")
    ap.add_argument("--capture", action="store_true",
                    help="batch workload: replay the iterations from a captured hipGraph")
    ap.add_argument("--hub-shared", action="store_true",
                    help="one shared LDS sketch per high-degree vertex instead of merged "
                         "partial sketches (async ablation)")
    ap.add_argument("--stream-csr", action="store_true",
                    help="keep the CSR in pinned host memory and stream it to the device in "
                         "slices every iteration (LPA_STREAM_CSR, det mode)")
    ap.add_argument("--stream-chunk-kib", type=int, default=0,
                    help="slice size for --stream-csr in KiB of column indices (0 = 256 MiB)")
    ap.add_argument("--offsets64", action="store_true",
                    help="hand the row offsets over as int64 (64-bit CSR positions)")
    ap.add_argument("--shared-vars", action="store_true",
                    help="det hub path with LDS shared variables instead of wavefront votes "
                         "(LPA_SHARED_VARS)")
    ap.add_argument("--rescan", action="store_true",
                    help="double scan: re-weight the sketch's labels exactly in a second pass")
    ap.add_argument("--rule", default="mg", choices=["mg", "bm_paper"],
                    help="per-vertex rule: k-slot Misra-Gries sketch, or the vote of "
                         "Algorithm 3 (forces k=1)")
    ap.add_argument("--mode", default="async", choices=["async", "det"])
    ap.add_argument("--ranked", action="store_true",
                    help="ranked layout: labels and flags by degree-order position, column "
                         "indices rewritten as positions (LPA_RANKED_LAYOUT, +4 B per entry)")
    ap.add_argument("--no-other-layout", action="store_true",
                    help="leave out the measurement of the other state layout")
    ap.add_argument("--max-iter", type=int, default=20)
    ap.add_argument("--tol", type=float, default=0.05)
    ap.add_argument("--lane-max-degree", type=int, default=0)
    ap.add_argument("--check-every", type=int, default=-1,
                    help="lpa_config.check_every of the solve (-1: 1 above 5e7 entries, else 0)")
    ap.add_argument("--move-blocks-per-cu", type=int, default=0,
                    help="cap on resident move-kernel workgroups per CU (0 = all that fit)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="graph", choices=["graph", "batch", "serve"],
                    help="graph: one large graph (default); batch: many graphs per launch; "
                         "serve: Poisson request stream with continuous batching")
    ap.add_argument("--batch-graphs", type=int, default=512)
    ap.add_argument("--requests", type=int, default=200)
    ap.add_argument("--serve-loads", default="0.5,0.9,1.5",
                    help="arrival rates as multiples of the sequential service rate; the "
                         "headline value is the heaviest")
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--serve-max-scale", type=int, default=20)
    ap.add_argument("--serve-no-overlap", action="store_true",
                    help="admit requests inside the tick loop (no admission thread and stream)")
    ap.add_argument("--no-batch", action="store_true",
                    help="graph workload: leave out the batched sub-measurement")
    ap.add_argument("--no-serve", action="store_true",
                    help="graph workload: leave out the serving sub-measurement")
    ap.add_argument("--no-quality", action="store_true",
                    help="graph workload: leave out the det-mode quality run")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES (for scaling the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy // 4
        src = torch.arange(n, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 4 * n, "launches": 3}))
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "path is not built", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2411_19901_amd import lpa

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    lpa.load()  # fail loudly if the HIP library is missing
    if args.workload == "batch":
        if args.mode == "async" and "--mode" not in sys.argv:
            args.mode = "det"
        print(json.dumps(bench_batch(args, 0 if args.no_cpu_baseline else 8)), flush=True)
        return
    if args.workload == "serve":
        if "--mode" not in sys.argv:
            args.mode = "det"
        print(json.dumps(bench_serve(args)), flush=True)
        return
    dev = torch.device("cuda:0")
    if args.graph == "ring":
        from types import SimpleNamespace
        from paper_2411_19901_amd import inputs
        L, H, r = 36_000_000, 64, 30
        t = time.perf_counter()
        rp, col, w = inputs.ring_hubs_device(L, H, r, 2024, dev)
        torch.cuda.synchronize()
        g = SimpleNamespace(n=L + H, nnz=int(rp[-1]))
        gname = f"ring{L // 1_000_000}M-h{H}-r{r}-wU(0,1]"
        h2d_s = 0.0
        args.offsets64 = True
        args.no_cpu_baseline = True  # the graph exists only in device memory
        log(f"[bench] built {gname} on the device: n={g.n} nnz={g.nnz} "
            f"in {time.perf_counter() - t:.1f}s")
    else:
        g, gname = build_graph(args)
    if args.rule == "bm_paper":
        args.k = 1
    rule_tag = ((f"k{args.k}" if args.rule == "mg" else "bm-paper") + ("-rescan" if args.rescan else "")
                + ("-hubshared" if args.hub_shared else "")
                + ("-sharedvars" if args.shared_vars else ""))
    workload = (f"{gname}-{args.mode}-{rule_tag}" + ("-off64" if args.offsets64 else "")
                + ("-ranked" if args.ranked else ""))

    if args.graph != "ring":
        t = time.perf_counter()
        if args.host_csr or args.stream_csr:
            place = lambda a: torch.from_numpy(a).pin_memory()  # noqa: E731
            workload += "-stream" if args.stream_csr else "-hostcsr"
        else:
            place = lambda a: torch.from_numpy(a).to(dev)  # noqa: E731
        rp = place(g.row_ptr.astype(np.int64) if args.offsets64 else g.row_ptr)
        col = place(g.col)
        w = place(g.w) if g.w is not None else None
        torch.cuda.synchronize()
        h2d_s = time.perf_counter() - t
    stream = torch.cuda.current_stream(dev)
    tuned = None
    if args.autotune:
        from paper_2411_19901_amd import tune
        t = time.perf_counter()
        tuned = tune.tune(rp, col, w, k=args.k, mode=args.mode, rule=args.rule)
        tuned["seconds"] = round(time.perf_counter() - t, 2)
        tuned["table"] = {str(k_): round(v, 4) for k_, v in tuned["table"].items()}
        args.lane_max_degree = tuned["lane_max_degree"]
        args.move_blocks_per_cu = tuned["move_blocks_per_cu"]
        log(f"[bench] autotuned lane_max_degree = {args.lane_max_degree}, move_blocks_per_cu = "
            f"{args.move_blocks_per_cu} ({tuned['table']})")
    free0, _ = torch.cuda.mem_get_info(dev)
    t = time.perf_counter()
    # large graphs read the stop flag after every iteration (a host round
    # trip of a few microseconds) rather than enqueue every remaining
    # iteration of max_iter, whose launches cost more once converged
    check_every = args.check_every if args.check_every >= 0 else (1 if g.nnz > 50_000_000 else 0)

    def make_solver(ranked):
        return lpa.LPA(rp, col, w, k=args.k, tol=args.tol, max_iter=args.max_iter,
                       mode=args.mode, lane_max_degree=args.lane_max_degree, rule=args.rule,
                       rescan=args.rescan, hub_shared=args.hub_shared,
                       shared_vars=args.shared_vars, stream_csr=args.stream_csr,
                       stream_chunk_kib=args.stream_chunk_kib, ranked=ranked,
                       move_blocks_per_cu=args.move_blocks_per_cu,
                       check_every=check_every, stream=stream)

    solver = make_solver(args.ranked)
    torch.cuda.synchronize()
    init_ms = (time.perf_counter() - t) * 1e3
    free1, _ = torch.cuda.mem_get_info(dev)
    core_bytes, _ = solver.memory()
    solver.profile(True)
    log(f"[bench] lpa_init {init_ms:.1f} ms; library bytes/vertex {core_bytes / g.n:.2f}")

    tm = timed_solves(solver, args.steps, args.warmup)
    edges_total, elapsed, kernel_ms, launches, iters = (tm["edges"], tm["elapsed"],
                                                        tm["kernel_ms"], tm["launches"],
                                                        tm["iters"])
    kernel_bytes = BYTES_PER_EDGE * edges_total

    floor_ms = solver.memory_floor_ms(3)
    labels = solver.labels(device=True)
    q = solver.modularity()  # the first call allocates the community totals
    mod_ms = None
    for _ in range(3):  # warm calls: k_modularity, the totals pass, four doubles back
        tq = time.perf_counter()
        q = solver.modularity()
        t_q = (time.perf_counter() - tq) * 1e3
        mod_ms = t_q if mod_ms is None else min(mod_ms, t_q)
    dn, sc = solver.trace()
    ms = solver.move_ms()

    achieved = kernel_bytes / (kernel_ms * 1e-3) / 1e9 if kernel_ms > 0 else 0.0
    digest = source_digest()
    kk = args.k if args.rule == "mg" else 0  # kernel template: 0 = the vote of Algorithm 3
    wide = "true" if args.offsets64 else "false"
    if args.shared_vars:
        kname = f"lpa::k_move_sv<{kk}, {wide}>"
    else:
        kname = (f"lpa::k_move{'_rescan' if args.rescan else ''}"
                 f"<{kk}, {'true' if args.mode == 'async' else 'false'}, {wide}>")
    traffic = traffic_from_profiles(kname,
                                    workload, digest)
    result = {
        "metric": METRIC,
        "value": round(edges_total / elapsed / 1e9, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "n": g.n, "nnz": g.nnz, "k": args.k, "rule": args.rule,
                   "lane_max_degree": args.lane_max_degree or (1024 if args.mode == "async"
                                                                else 4096),
                   "rescan": args.rescan, "offsets": 64 if args.offsets64 else 32,
                   "ranked_layout": bool(args.ranked),
                   "move_blocks_per_cu": args.move_blocks_per_cu,
                   "mode": args.mode,
                   "tol": args.tol, "max_iter": args.max_iter, "rho": 8,
                   "step": "lpa_reset + lpa_run (all iterations to convergence)"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic,
                     "kernel": kname,
                     "bytes_per_edge": BYTES_PER_EDGE, "launches": launches,
                     "avg_launch_ms": round(kernel_ms / max(launches, 1), 4),
                     "source_digest": digest},
        "scan_memory_floor": {
            "ms": round(floor_ms, 4),
            "GBps": round(BYTES_PER_EDGE * g.nnz / (floor_ms * 1e-3) / 1e9, 1) if floor_ms > 0 else None,
            "what": "stream col+w and gather every neighbour label once, no sketch (lpa_memory_floor)",
            "kernel_frac_of_floor": round((BYTES_PER_EDGE * g.nnz / (floor_ms * 1e-3) / 1e9) and
                                          achieved / (BYTES_PER_EDGE * g.nnz / (floor_ms * 1e-3) / 1e9), 4)
            if floor_ms > 0 else None},
        "iterations": iters[-1],
        "iter0": {"scanned": int(sc[0]) if len(sc) else 0,
                  "move_ms": round(float(ms[0]), 4) if len(ms) else None,
                  "GBps": round(BYTES_PER_EDGE * int(sc[0]) / (float(ms[0]) * 1e-3) / 1e9, 1)
                  if len(ms) and ms[0] > 0 else None},
        "trace": {"changed": dn.tolist(), "scanned": sc.tolist(),
                  "move_ms": [round(float(x), 4) for x in ms]},
        "modularity": round(q, 6),
        "modularity_ms": round(mod_ms, 3),
        "init_ms": round(init_ms, 2),
        "h2d_s": round(h2d_s, 3),
        "bytes_per_vertex": round(core_bytes / g.n, 3),
        # per-vertex hashtables of the earlier GPU method: 16 B per CSR entry
        "hashtable_method_bytes_per_vertex": round(16 * g.nnz / g.n, 1),
        "hipmeminfo_bytes_per_vertex": round((free0 - free1) / g.n, 3),
        "gpu": torch.cuda.get_device_name(dev),
    }
    if tuned is not None:
        result["autotune"] = {"lane_max_degree": tuned["lane_max_degree"],
                              "move_blocks_per_cu": tuned["move_blocks_per_cu"],
                              "ns_per_entry": tuned["table"], "seconds": tuned["seconds"]}
    del labels
    solver.close()
    if (not args.no_other_layout and args.graph != "ring"
            and not (args.stream_csr or args.host_csr)):
        # the same measurement with the other state layout
        other = make_solver(not args.ranked)
        other.profile(True)
        tmo = timed_solves(other, args.steps, 1, tag=" [other layout]")
        fl = other.memory_floor_ms(3)
        ach = (BYTES_PER_EDGE * tmo["edges"] / (tmo["kernel_ms"] * 1e-3) / 1e9
               if tmo["kernel_ms"] > 0 else 0.0)
        cb, _ = other.memory()
        result["other_layout"] = {
            "ranked": not args.ranked, "value": round(tmo["edges"] / tmo["elapsed"] / 1e9, 3),
            "unit": "GTEPS", "ms_per_step": round(tmo["elapsed"] * 1e3 / args.steps, 3),
            "avg_launch_ms": round(tmo["kernel_ms"] / max(tmo["launches"], 1), 4),
            "achieved_GBps": round(ach, 1), "frac": round(ach / HBM_PEAK_GBPS, 4),
            "scan_memory_floor_ms": round(fl, 4), "iterations": tmo["iters"][-1],
            "modularity": round(other.modularity(), 6), "bytes_per_vertex": round(cb / g.n, 3),
            "traffic": traffic_from_profiles(
                kname, (workload[:-len("-ranked")] if args.ranked else workload + "-ranked"),
                digest)}
        other.close()
    quality = (not args.no_quality and args.mode == "async" and args.rule == "mg"
               and not (args.host_csr or args.stream_csr or args.hub_shared))
    if quality:
        # the same graph in det mode: Jacobi updates, every sketch fed in CSR
        # order (the labels the CPU definition of the method gives)
        log("[bench] det-mode run of the same graph for the quality comparison")
        det = lpa.LPA(rp, col, w, k=args.k, tol=args.tol, max_iter=args.max_iter, mode="det",
                      rescan=args.rescan, check_every=1, stream=stream)
        torch.cuda.synchronize()
        t = time.perf_counter()
        it_det = det.run()
        torch.cuda.synchronize()
        det_s = time.perf_counter() - t
        _, sc_det = det.trace()
        result["quality"] = {
            "q_async": round(q, 6), "async_iterations": iters[-1],
            "q_det": round(det.modularity(), 6), "det_iterations": it_det,
            "det_solve_ms": round(det_s * 1e3, 2),
            "det_GTEPS": round(int(sc_det.sum()) / det_s / 1e9, 3),
            "q_exact_oracle": None,
            "note": "q_det: det mode on the GPU (labels bit-identical to the Misra-Gries oracle); "
                    "q_exact_oracle: the exact rule of Eq. 3, from cpu_baseline.exact_rule_run"}
        det.close()
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a vertex sample")
        result["cpu_baseline"] = cpu_baseline(g, args.k if args.rule == "mg" else -1,
                                              args.cpu_seconds, exact_run=quality)
        if quality:
            result["quality"]["q_exact_oracle"] = result["cpu_baseline"]["exact_rule_run"]["q"]
    del rp, col, w
    torch.cuda.empty_cache()
    import copy
    if not args.no_batch and args.graph == "rmat" and args.scale == 24:
        log("[bench] batched workload (512 planted-partition graphs, det, captured)")
        ba = copy.copy(args)
        ba.mode, ba.capture, ba.k, ba.autotune = "det", True, 8, True
        ba.steps, ba.warmup = min(args.steps, 5), 1
        result["batch"] = bench_batch(ba, 0 if args.no_cpu_baseline else 8)
        torch.cuda.empty_cache()
    if not args.no_serve and args.graph == "rmat" and args.scale == 24:
        log("[bench] serving workload (Poisson mix, continuous batching)")
        sa = copy.copy(args)
        sa.mode, sa.k, sa.warmup = "det", 8, 1
        result["serve"] = bench_serve(sa)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
