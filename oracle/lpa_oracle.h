/*
 * CPU oracle for memory-efficient label propagation (weighted Misra-Gries
 * sketch LPA, arXiv 2411.19901).
 *
 * TEST INFRASTRUCTURE ONLY. Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load or call this library. The product
 * (the HIP library under paper_2411_19901_amd/) shares no code with it and
 * never links it.
 *
 * Conventions shared with the product only through the paper:
 *   - undirected graph stored as symmetric CSR: row_ptr int32[n+1],
 *     col int32[nnz]; weights fp32[nnz] (NULL = every weight 1.0);
 *   - labels int32[n], initialised to the vertex id;
 *   - sketch keys int32, sketch values fp32 (Section 5.1.2, Configuration).
 */
#ifndef LPA_ORACLE_H
#define LPA_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* k-slot weighted Misra-Gries sketch (Section 4.1); slot s is empty iff
 * val[s] == 0. */
void orc_sketch_clear(int k, int32_t *key, float *val);
void orc_sketch_accumulate(int k, int32_t *key, float *val, int32_t c, float w);
int32_t orc_sketch_max_key(int k, const int32_t *key, const float *val,
                           int32_t keep);
/* clear, then feed len (label, weight) pairs in order; w NULL = unit. */
void orc_sketch_feed(int k, int64_t len, const int32_t *labels, const float *w,
                     int32_t *key, float *val);

/* The weighted Boyer-Moore vote exactly as Algorithm 3 (lpaMove scan loop)
 * states it: the candidate starts as (init, 0); a pair (c, w) adds w when c
 * is the candidate, else subtracts w when the candidate's weight exceeds w,
 * else replaces the candidate by (c, w).  Returns the final candidate and
 * stores its weight in *weight. */
int32_t orc_bm_paper_feed(int64_t len, const int32_t *labels, const float *w,
                          int32_t init, float *weight);

/* Value of k that selects the rule of Algorithm 3 (one candidate) in the
 * functions below. */
#define ORC_BM_PAPER (-1)

/* One synchronous (Jacobi) iteration of Algorithm 1's lpaMove.
 * k >= 1: k-slot sketch; k == 0: exact argmax of Eq. 3 (dense accumulator);
 * k == ORC_BM_PAPER: the vote of Algorithm 3.  rescan != 0 (k >= 1 only):
 * double scan, the sketch's live labels re-weighted exactly in a second
 * pass over the row (Section 4.4, Algorithm 4).
 * Reads C and act, writes C_next and act_next (act_next must be zeroed by
 * the caller).  Returns the number of changed vertices; *scanned receives
 * the number of CSR entries read by the neighbourhood scans. */
int64_t orc_lpa_move(int32_t n, const int32_t *row_ptr, const int32_t *col,
                     const float *w, int k, int rescan, int pickless, const int32_t *C,
                     const uint8_t *act, int32_t *C_next, uint8_t *act_next,
                     int nthreads, int64_t *scanned);

/* Whole driver (Algorithm 1, lpa). Returns the number of iterations run,
 * or -1 on bad arguments.  dN_trace / scanned_trace (may be NULL) receive
 * max_iter entries each. */
int orc_lpa_run(int32_t n, const int32_t *row_ptr, const int32_t *col,
                const float *w, int k, int rescan, double tol, int max_iter, int rho,
                int nthreads, int32_t *labels, int64_t *dN_trace,
                int64_t *scanned_trace);

/* The label each listed vertex would choose in one iteration, given C:
 * out[q] = chosen label of verts[q] (the current label when it keeps it). */
void orc_lpa_choose(int32_t n, const int32_t *row_ptr, const int32_t *col,
                    const float *w, int k, int rescan, int pickless, const int32_t *C,
                    int64_t nv, const int32_t *verts, int32_t *out,
                    int nthreads);

/* Partial sketches of a high-degree vertex v (Section 4.3; reading R9): its
 * row is cut into segments of seg_len entries, each fed in CSR order (v
 * itself skipped) into a k-slot sketch of its own.  Up to
 * ORC_MERGE_CHAINS segments, the partials' live slots are fed, segment by
 * segment and slot by slot, into one sketch.  Above that, partial q goes to
 * chain q mod ORC_MERGE_CHAINS (each chain fed in segment order), and the
 * chains are then combined in rounds at distances 32, 16, ..., 1: in each
 * round chain t is fed the live slots chain t ^ distance held at the start
 * of the round; the merged sketch is chain 0.  Writes it to key/val (k
 * entries) and returns the number of segments (-1: bad arguments). */
#define ORC_MERGE_CHAINS 64
int64_t orc_hub_merged_sketch(const int32_t *row_ptr, const int32_t *col,
                              const float *w, int k, int32_t seg_len,
                              const int32_t *C, int32_t v, int32_t *key,
                              float *val);

/* For each listed vertex, the label it holds after one iteration when it is
 * processed through its partial sketches: the merged sketch's heaviest
 * label (rescan: its live labels re-weighted exactly over the whole row),
 * adopted under the pick-less rule. */
void orc_hub_choose(int32_t n, const int32_t *row_ptr, const int32_t *col,
                    const float *w, int k, int rescan, int32_t seg_len,
                    int pickless, const int32_t *C, int64_t nv,
                    const int32_t *verts, int32_t *out, int nthreads);

/* Modularity Q of Eq. 1 (community-sum form) in fp64. */
double orc_modularity(int32_t n, const int32_t *row_ptr, const int32_t *col,
                      const float *w, const int32_t *C);

int orc_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
