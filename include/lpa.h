/*
 * lpa.h — C ABI of the MI355X (gfx950) label-propagation library
 * (liblpa.so): memory-efficient community detection with a k-slot weighted
 * Misra-Gries sketch per vertex, after arXiv 2411.19901.
 *
 * The method (paper Section 4; Algorithm 1 lpa / lpaMove; Algorithm 2
 * sketchAccumulate): every label starts as the vertex id; in each iteration
 * every unprocessed vertex streams its CSR neighbour list, keeps a k-slot
 * weighted Misra-Gries sketch of the neighbours' labels (Section 4.1) and
 * adopts the heaviest sketch label (Section 4.4, single scan).  Every rho
 * iterations from the first a vertex may only move to a lower label
 * (pick-less, Section 4.5).  Changed vertices mark their neighbours
 * unprocessed; the run stops when a non-pick-less iteration changes fewer
 * than tol * N labels, or after max_iter iterations (Algorithm 1, lpa).
 *
 * Modes:
 *   LPA_MODE_DET    synchronous (Jacobi) updates; every sketch is fed in CSR
 *                   order.  Labels are bit-identical to the sequential CPU
 *                   definition of the algorithm, independent of launch
 *                   geometry, bin thresholds and scheduling.
 *   LPA_MODE_ASYNC  labels and flags are updated in place while the
 *                   iteration runs (as the paper's GPU implementation
 *                   does); high-degree vertices use partial sketches that
 *                   are merged (Section 4.3).  Results depend on scheduling.
 *
 * Readings of points the paper leaves open (shared with the CPU
 * definition): the sketch decrement subtracts
 * d = min(w, smallest slot) and inserts the residue w - d (identical to the
 * paper's rule on unit weights); k = 1 is the same rule with one slot;
 * ties go to the lowest label; an empty sketch keeps the label; a vertex
 * blocked by pick-less still counts as processed; N = |V| and the
 * convergence test is strict.
 *
 * Conventions for every call:
 *   - Every function returns an lpa_status code; no call aborts or throws.
 *   - Device pointers are HIP device (or managed) pointers on the device
 *     current at lpa_init.  Graph arrays are BORROWED: the caller owns them,
 *     they must stay valid and unmodified until lpa_free.
 *   - Work is enqueued on the handle's stream.  Calls that return host
 *     values synchronise that stream first.
 *   - A handle is not re-entrant; separate handles may be used from
 *     separate threads on separate streams.
 *   - After a HIP runtime error the handle is poisoned: every later call
 *     except lpa_free / lpa_last_error returns LPA_ERR_HIP.
 *   - All device memory the library needs is allocated in lpa_init (plus
 *     an fp64 scratch on the first lpa_modularity call); iterations
 *     allocate nothing.
 */
#ifndef LPA_H
#define LPA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lpa_status {
  LPA_OK = 0,
  LPA_ERR_ARG = 1,         /* null pointer, bad k / tol / max_iter / rho / size */
  LPA_ERR_GRAPH = 2,       /* invalid CSR, weights or labels (see LPA_VALIDATE) */
  LPA_ERR_UNSUPPORTED = 3, /* k not one of 1, 2, 4, 8, 16, 32; unknown mode */
  LPA_ERR_NOMEM = 4,       /* device allocation failed */
  LPA_ERR_HIP = 5,         /* HIP runtime error; the handle is now poisoned */
  LPA_ERR_STATE = 6        /* handle in the wrong state for this call */
} lpa_status;

/* mode (low byte) and option flags for lpa_config.flags */
#define LPA_MODE_DET 0u
#define LPA_MODE_ASYNC 1u
#define LPA_MODE_MASK 0xFFu
/* Check the CSR on the device in lpa_init: row_ptr[0] == 0, nondecreasing,
 * row_ptr[n] == nnz, 0 <= col < n, weights finite and > 0.  Without it an
 * invalid graph is undefined behaviour (out-of-range reads).  Symmetry is
 * expected but never checked. */
#define LPA_VALIDATE 0x100u
/* Replace the sketch by the paper's one-candidate weighted Boyer-Moore vote
 * (Section 4.7, Algorithm 3, nu-BM-LPA): the candidate starts as the
 * vertex's own label with weight 0; a neighbour pair (c, w) adds w when c is
 * the candidate, subtracts w when the candidate's weight is larger than w,
 * and otherwise becomes the candidate with weight w.  The final candidate is
 * the choice (pick-less and pruning as for the sketch).  Requires k == 1
 * (LPA_ERR_ARG otherwise).  LPA_MODE_DET feeds every vertex in CSR order
 * (bit-identical to the CPU definition); LPA_MODE_ASYNC splits high-degree
 * vertices into segments whose candidates are combined by the largest
 * weight, ties to the lowest label (the paper's pair-max reduction). */
#define LPA_RULE_BM_PAPER 0x200u
/* Double scan (Section 4.4 and Algorithm 4, "rescan"): after the single
 * scan the labels of the sketch's non-empty slots are the candidates; a
 * second pass over the row sums each candidate's exact weight and the
 * heaviest candidate is chosen (ties to the lowest label; no candidate
 * keeps the label).  In LPA_MODE_DET the second pass adds in CSR order
 * (bit-identical to the CPU definition); in LPA_MODE_ASYNC high-degree
 * vertices sum their segments' weights in any order.  Sketch rule only
 * (LPA_ERR_ARG together with LPA_RULE_BM_PAPER).  Reads every processed row
 * twice. */
#define LPA_RESCAN 0x400u
/* Ablation of the partial sketches of Section 4.3 (LPA_MODE_ASYNC, sketch
 * rule, no LPA_RESCAN; LPA_ERR_ARG otherwise): every vertex of degree above
 * lane_max_degree is processed by one workgroup whose threads all update
 * a single shared sketch in LDS with atomics, as in the shared mode of
 * Algorithm 5 (add to a matching slot, claim a free slot by
 * compare-and-swap with retries, otherwise decrement every slot), instead
 * of per-segment sketches merged afterwards.  Updates race, so results are
 * approximate and depend on scheduling. */
#define LPA_HUB_SHARED 0x800u
/* Run iterations from a captured hipGraph: when check_every is 0, the
 * remaining iterations of an lpa_run / lpa_batch_run (all their kernels)
 * are captured once on a private stream of the handle or batch and the
 * graph is replayed on the caller's stream; it is captured again only when
 * the launch shape (graphs, work items, iteration count) changes.  Results
 * are identical to launching the kernels one by one.  Ignored while
 * per-iteration profiling (lpa_profile) is on. */
#define LPA_CAPTURE 0x1000u
/* Ablation of the wavefront votes of Section 4.1 (LPA_MODE_DET, sketch
 * rule, no LPA_RESCAN; LPA_ERR_ARG otherwise): in the one-wavefront-per-
 * vertex path for vertices above lane_max_degree, whose lanes hold one
 * sketch slot each, the lanes find the slot of a label, a free slot and the
 * smallest slot through shared variables in LDS written with plain stores
 * and atomic minimums (the shared-variable protocol of Algorithm 5) instead
 * of wavefront votes.  Results are identical; only the speed differs. */
#define LPA_SHARED_VARS 0x2000u
/* Stream the graph from host memory (not with LPA_HUB_SHARED: LPA_ERR_ARG):
 * col_idx and the weights must be pinned host memory (LPA_PTR_HOST; the
 * row offsets may be host or device memory and are copied to the device
 * once).  lpa_init cuts the vertices into consecutive id ranges whose rows
 * fill at most stream_chunk_kib KiB of column indices (a range is one
 * vertex when that vertex alone is larger) and bins each range by degree
 * (LPA_MODE_ASYNC: and splits each range's hubs into segments of their own).
 * Every iteration then copies the ranges' rows into four device buffers in
 * turn with DMA on a stream of the handle's own; each range's move kernel
 * starts once its copy has landed, on one of four compute streams (the
 * caller's and three of the handle's), so copies and up to four ranges'
 * kernels overlap.  In LPA_MODE_DET the synchronous update makes the
 * labels independent of the cut and of that overlap: results are identical
 * to the unstreamed run; LPA_MODE_ASYNC runs the ranges in place like its
 * wavefronts.  Device memory: the library state, a second degree order (4 B
 * per vertex), the row offsets, each range's hub segments (async) and the
 * four buffers; not the graph.  LPA_VALIDATE in lpa_init and lpa_modularity
 * read the host arrays directly over the link (once per call).  lpa_run checks convergence after every
 * iteration; LPA_CAPTURE and lpa_batch_* do not apply (batches refuse such
 * handles with LPA_ERR_ARG). */
#define LPA_STREAM_CSR 0x4000u
/* Ranked layout of the device state (not with LPA_STREAM_CSR: LPA_ERR_ARG):
 * lpa_init lists the vertices in decreasing-degree order (the order of its
 * degree binning; isolated vertices last) and keeps each vertex's label
 * and unprocessed flag at its position in that order instead of at its id,
 * with a copy of col_idx rewritten as positions (int32[nnz], owned by the
 * handle; +4 bytes per CSR entry of device memory, part of
 * lpa_workspace_bytes).  The label values are still vertex ids, every
 * sketch still sees its row in CSR order, and the rows are still read from
 * the caller's row offsets and weights, so LPA_MODE_DET results are
 * bit-identical to the default layout.  What changes is locality: the
 * labels of the high-degree vertices, which most CSR entries name, sit
 * together at the front of the label array, so the per-entry label reads
 * of the neighbourhood scans hit the caches far more often, and a
 * wavefront's own labels and flags are read contiguously.  Labels, flags
 * and checkpoints cross the ABI indexed by vertex id as usual. */
#define LPA_RANKED_LAYOUT 0x8000u

/* Undirected graph as symmetric CSR (paper Section 3: w_ij = w_ji).  Row
 * offsets are given either as int32 (row_ptr, graphs of fewer than 2^31 - 1
 * entries) or as int64 (row_ptr64, any size that memory holds, up to
 * 2^62 entries): exactly one of the two is set when n > 0, otherwise
 * lpa_init returns LPA_ERR_ARG.  With either width every vertex has fewer
 * than 2^31 entries (checked under LPA_VALIDATE).  The arrays may be in
 * device memory or in pinned host memory (lpa_pointer_location). */
typedef struct lpa_graph {
  int32_t n;               /* number of vertices, 0 <= n < 2^31 - 1 */
  int64_t nnz;             /* number of CSR entries (directed) */
  const int32_t *row_ptr;  /* int32[n+1], or NULL when row_ptr64 is set */
  const int32_t *col_idx;  /* int32[nnz], neighbour ids */
  const int64_t *row_ptr64; /* int64[n+1], or NULL when row_ptr is set */
} lpa_graph;

typedef struct lpa_config {
  uint32_t flags;          /* LPA_MODE_DET or LPA_MODE_ASYNC,
                              | LPA_VALIDATE, | LPA_RULE_BM_PAPER, | LPA_RESCAN,
                              | LPA_HUB_SHARED, | LPA_CAPTURE, | LPA_SHARED_VARS,
                              | LPA_STREAM_CSR, | LPA_RANKED_LAYOUT */
  int32_t rho;             /* pick-less period; 0 disables pick-less; default 8 */
  void *stream;            /* hipStream_t for all work; NULL = null stream */
  int32_t lane_max_degree; /* vertices with degree <= this run one lane per
                              vertex, higher degrees cooperatively;
                              0 = default for the mode (async 1024, det
                              4096).  Never changes
                              LPA_MODE_DET results. */
  int32_t check_every;     /* lpa_run / lpa_batch_run read the convergence
                              state on the host every this many iterations
                              and stop launching once every graph finished;
                              0 = enqueue all remaining iterations (finished
                              graphs exit on the device), synchronise once */
  void *workspace;         /* optional device memory for every array of the
                              handle (256-byte aligned, at least
                              lpa_workspace_bytes, which covers the largest
                              possible number of async hub segments); NULL =
                              lpa_init allocates one block itself and, in
                              LPA_MODE_ASYNC, the partial sketches of the
                              segments it planned in a second one.  Borrowed
                              like the graph. */
  size_t workspace_bytes;
  int32_t stream_chunk_kib; /* LPA_STREAM_CSR: rows copied per slice, in
                              KiB of column indices (the weights double
                              it); 0 = 262144 (256 MiB).  Ignored
                              otherwise. */
  int32_t move_blocks_per_cu; /* launch at most this many workgroups of the
                              move kernel per compute unit (0 = as many as
                              are resident at once; 1..64).  Fewer
                              resident wavefronts trade latency hiding for
                              cache share; the autotuner picks it.  Never
                              changes LPA_MODE_DET results. */
  int32_t reserved[2];     /* must be zero */
} lpa_config;

typedef struct lpa_handle lpa_handle;
typedef struct lpa_batch lpa_batch;

/* Fill *cfg with the defaults (det mode, rho 8, null stream, validation on). */
void lpa_config_default(lpa_config *cfg);

/* Where the library's kernels would read an array from (values of
 * *location): LPA_PTR_DEVICE device or managed memory of the current device;
 * LPA_PTR_HOST pinned host memory mapped into the device's address space
 * (hipHostMalloc), read over the host link at the same address;
 * LPA_PTR_UNUSABLE anything else (pageable host memory, another device's
 * memory, NULL).  The graph arrays of lpa_init and the labels of
 * lpa_modularity may be device or mapped host memory; anything else is
 * refused with LPA_ERR_ARG before a kernel could touch it.  A CSR kept in
 * pinned host memory leaves only the O(|V|) state of the method in device
 * memory (Section 6 names keeping the input graph outside device memory as
 * the way to larger graphs); every iteration then streams it over the
 * link.
 * Synchronises nothing; no device work. */
#define LPA_PTR_UNUSABLE 0
#define LPA_PTR_DEVICE 1
#define LPA_PTR_HOST 2
int lpa_pointer_location(const void *ptr, int *location);

/* Create a handle for graph g (its arrays: device or mapped pinned host
 * memory, see lpa_pointer_location; LPA_ERR_ARG otherwise).
 *   weights  device fp32[nnz] edge weights, symmetric, finite, > 0;
 *            NULL = every weight 1.0 (borrowed like the graph)
 *   k        sketch slots: 1 (weighted Boyer-Moore), 2, 4, 8, 16 or 32
 *   tol      tau in [0, 1]: stop when dN / N < tol in a non-pick-less iteration
 *   max_iter maximum iterations, >= 0
 *   seed     recorded only; no mode draws random numbers
 *   cfg      NULL = lpa_config_default
 * Allocates the label, flag, bin and counter arrays on the current device,
 * bins the vertices by degree (the degree-dependent assignment of threads to
 * vertices of Section 4.2), and sets up the start of Algorithm 1 (lpa):
 * every label is the vertex id and every vertex is unprocessed.
 * On success *out receives the handle; on failure *out is NULL. */
int lpa_init(const lpa_graph *g, const float *weights, int k, double tol,
             int max_iter, uint64_t seed, const lpa_config *cfg,
             lpa_handle **out);

/* Device bytes lpa_init needs for a graph of n vertices and nnz entries
 * with these parameters (cfg NULL = defaults); the size of a caller
 * workspace (lpa_config.workspace).  The size does not depend on the
 * width of the row offsets.  LPA_ERR_ARG for nnz < 0 or nnz >= 2^62;
 * LPA_ERR_UNSUPPORTED when LPA_MODE_ASYNC would split the hubs into 2^30
 * or more segments (nnz / lane_max_degree too large: raise the threshold). */
int lpa_workspace_bytes(int32_t n, int64_t nnz, int k, int max_iter,
                        const lpa_config *cfg, size_t *bytes);

/* Move the handle to another stream: synchronises the current one, then
 * enqueues all later work of the handle on `stream` (NULL = null stream).
 * Lets a caller build a handle on a stream of its own (lpa_init copies and
 * bins there) while other handles keep computing, then join it to the
 * stream of a batch.  LPA_ERR_ARG for a handle with LPA_STREAM_CSR. */
int lpa_set_stream(lpa_handle *h, void *stream);

/* Return the handle to iteration 0 (labels = ids, all vertices unprocessed,
 * traces cleared) without re-binning.  Enqueued; does not synchronise. */
int lpa_reset(lpa_handle *h);

/* Run one iteration (Algorithm 1, one lpaMove plus its convergence test)
 * and synchronise.  *changed = dN of that iteration; *done = 1 once the
 * run has finished (converged or max_iter reached).  A call on a finished
 * handle does nothing and reports changed = 0, done = 1.  Either output
 * pointer may be NULL. */
int lpa_step(lpa_handle *h, int64_t *changed, int *done);

/* The main loop of Algorithm 1 (lpa; Section 4.6): run iterations (one
 * lpaMove each, pick-less every rho iterations from the first, Section 4.5)
 * until a non-pick-less iteration changes fewer than tol * N labels or
 * max_iter iterations have run, then synchronise.
 * *iterations (may be NULL) = total iterations run since init / reset. */
int lpa_run(lpa_handle *h, int *iterations);

/* Batched launches.  A batch runs iterations of many handles (one graph
 * each) with one set of kernel launches per iteration: every graph keeps its
 * own iteration count, pick-less schedule, pruning flags, counters and
 * convergence test, so each handle ends exactly as lpa_run would leave it
 * (bit-identical labels in LPA_MODE_DET).  The handles passed to one call
 * must share k, mode, device and stream with the batch, appear once, and
 * number at most `capacity`; the set may change between calls (continuous
 * batching).  Graphs with int32 and int64 row offsets may be mixed (the
 * launch then computes CSR positions in 64 bits for all of them).  A call
 * whose graphs together have 2^31 or more work items (hub segments plus
 * wavefronts of lane vertices) returns LPA_ERR_UNSUPPORTED; split it.
 * The batch owns only its launch tables.
 *   cfg: mode flags, stream and check_every are used (NULL = defaults). */
int lpa_batch_create(int capacity, int k, const lpa_config *cfg, lpa_batch **out);

/* One iteration of every unfinished handle in hs[0..count); synchronises.
 * *changed = sum of their dN; *all_done = 1 when every handle has finished.
 * Either output may be NULL. */
int lpa_batch_step(lpa_batch *b, lpa_handle *const *hs, int count, int64_t *changed,
                   int *all_done);

/* Iterate every handle in hs[0..count) until each has converged or reached
 * max_iter; synchronises.  *iterations = the largest iteration count. */
int lpa_batch_run(lpa_batch *b, lpa_handle *const *hs, int count, int *iterations);

/* lpa_reset of every handle in hs[0..count) with one kernel launch
 * (labels to vertex ids, all vertices unprocessed, counters cleared), for
 * handles that fit the batch as in lpa_batch_run; does not synchronise. */
int lpa_batch_reset(lpa_batch *b, lpa_handle *const *hs, int count);

/* Release the batch (not its handles).  NULL is accepted. */
int lpa_batch_free(lpa_batch *b);

/* Progress of h as of its last synchronising call (no device access):
 * *iteration = iterations run, *finished = 1 once converged or at max_iter.
 * Either pointer may be NULL. */
int lpa_progress(const lpa_handle *h, int *iteration, int *finished);

/* Modularity Q of Eq. 1, community-sum form, accumulated in fp64.
 * labels: device (or mapped pinned host) int32[n] with values in [0, n),
 * or NULL for the handle's current labels; LPA_ERR_ARG for other memory.  Returns LPA_ERR_GRAPH (and leaves *q unset) if a label
 * is out of range.  Synchronises. */
int lpa_modularity(lpa_handle *h, const int32_t *labels, double *q);

/* lpa_modularity for callers that cannot allocate device memory (code
 * under stream capture, serving loops, harnesses that forbid hipMalloc):
 * the same result (|dQ| <= 1e-9 against lpa_modularity: fp64 sums in another
 * order), but the per-community totals live in a static device array of
 * the library instead of a per-handle allocation, so the call allocates
 * nothing, ever.  Limit: n <= 2^21 vertices (LPA_ERR_UNSUPPORTED above; the
 * array holds 2^21 + 32 doubles, 16 MiB per device the library runs on, kept
 * until the process ends).  The handle's device must be current
 * (LPA_ERR_ARG otherwise).  Every call on one device shares that array:
 * calls that overlap on one GPU (other streams or threads) race and give
 * wrong results; serialise them.  Other arguments, checks and errors as in
 * lpa_modularity.  Synchronises. */
int lpa_modularity_noalloc(lpa_handle *h, const int32_t *labels, double *q);

/* Copy the current labels (int32[n]) to out, a host pointer if out_is_host
 * is nonzero, else a device pointer.  Synchronises. */
int lpa_get_labels(lpa_handle *h, int32_t *out, int out_is_host);

/* Per-iteration counters of the current run: changed[i] = dN and
 * scanned[i] = CSR entries read by the neighbourhood scans of iteration i,
 * for i < *count = iterations run (at most capacity are written; either
 * array may be NULL).  Synchronises. */
int lpa_get_trace(lpa_handle *h, int64_t *changed, int64_t *scanned,
                  int capacity, int *count);

/* Checkpoint: copy out labels int32[n] and the unprocessed flags uint8[n]
 * that the next iteration will read, plus the next iteration index
 * (flags of degree-0 vertices are unspecified).  Host pointers if is_host.
 * Synchronises. */
int lpa_get_state(lpa_handle *h, int32_t *labels, uint8_t *unprocessed,
                  int *iteration, int is_host);

/* Restore a checkpoint into a handle built on the same graph and
 * parameters: labels (values in [0, n), checked -> LPA_ERR_GRAPH),
 * unprocessed flags (nonzero = unprocessed) and the next iteration index in
 * [0, max_iter].  Traces of earlier iterations read as zero.  In
 * LPA_MODE_DET the continued run is bit-identical to an uninterrupted one.
 * Synchronises. */
int lpa_set_state(lpa_handle *h, const int32_t *labels,
                  const uint8_t *unprocessed, int iteration, int is_host);

/* Device bytes allocated by the handle: core = everything the iterations
 * use (labels, flags, bins, counters; excludes the caller's graph and
 * weights), eval = fp64 modularity scratch (0 before the first
 * lpa_modularity). Either pointer may be NULL. */
int lpa_memory(const lpa_handle *h, size_t *core_bytes, size_t *eval_bytes);

/* Kernel timing: when enabled, HIP events are recorded on the handle's
 * stream immediately before and after the move kernel k_move (the
 * neighbourhood scans, sketches and label updates; in LPA_MODE_ASYNC the
 * hub flag snapshot before it and the hub merge after it are outside) of
 * every iteration.  Enabling it creates
 * the events; it is off by default. */
int lpa_profile(lpa_handle *h, int enable);

/* Duration in milliseconds of the move kernel of each iteration of the
 * current run (move_ms[i] for i < *count = iterations run; at most
 * capacity written).  An iteration whose kernel was not timed (run before
 * profiling was enabled, skipped by lpa_set_state, or run through
 * lpa_batch_step / lpa_batch_run) reads -1.  LPA_ERR_STATE when profiling
 * is off.  Synchronises. */
int lpa_get_profile(lpa_handle *h, float *move_ms, int capacity, int *count);

/* Memory-pattern floor of one full scan of this graph: time (ms, best of
 * `reps` >= 1 launches) of a kernel that performs only the scan's memory
 * accesses (streams col_idx and the weights, gathers the label of every
 * neighbour) and none of the sketch work.  It bounds from below what the
 * move kernel can reach on this graph and GPU.  Does not change any state;
 * synchronises. */
int lpa_memory_floor(lpa_handle *h, int reps, float *ms);

/* Release the handle and its device memory (synchronises its stream first).
 * NULL is accepted. */
int lpa_free(lpa_handle *h);

/* Static description of a status code. */
const char *lpa_error_string(int code);
/* Description of the last error on h ("" when none); valid until the next
 * call on h. */
const char *lpa_last_error(const lpa_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* LPA_H */
