/*
 * CPU oracle for memory-efficient label propagation (arXiv 2411.19901).
 *
 * TEST INFRASTRUCTURE ONLY: tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py are its only users.  It is a plain, slow,
 * sequential-per-vertex rendering of the paper's algorithm in deterministic
 * synchronous (Jacobi) form:
 *
 *   - every vertex reads the labels of the previous iteration and feeds its
 *     neighbours' (label, weight) pairs into its own k-slot sketch in CSR
 *     order (Section 4.1; Algorithm 1, lpaMove; Algorithm 2 non-shared);
 *   - it adopts the heaviest sketch label, ties to the lowest label, and
 *     keeps its label when the sketch ends empty;
 *   - pick-less mode every rho iterations from the first (Section 4.5);
 *   - changed vertices mark their neighbours unprocessed (Algorithm 1);
 *   - stop when not pick-less and dN/N < tau, or after max_iter.
 *
 * Readings of points the paper leaves open:
 *   R1 decrement: when no slot is free the paper subtracts w from every slot
 *      (Section 4.1, Algorithm 2).  On non-unit weights that drives slots
 *      negative, so they can never become empty again.  We use the
 *      textbook weighted Misra-Gries step: subtract d = min(w, smallest
 *      slot) from every slot and insert the residue w - d when positive.
 *      On unit weights this is the paper's rule exactly.
 *   R2 k == 1 is the same rule with one slot (weighted Boyer-Moore).
 *   R3 ties in sketchMaxKey go to the lowest label; an empty sketch keeps
 *      the current label (not counted as a change).
 *   R4 processing clears a vertex's unprocessed flag; only neighbours of
 *      changed vertices are marked for the next iteration; a vertex blocked
 *      by pick-less is still processed.
 *   R5 N in dN/N is |V| (isolated vertices included); the comparison is
 *      strict and evaluated in double.
 *   R7 a pair goes to the slot whose label it carries even when a decrement
 *      has emptied that slot (Algorithm 2 compares labels only); a new label
 *      takes the lowest free slot; a pair of weight 0 changes nothing.
 *   R9 the merge order of a high-degree vertex's partial sketches (Section
 *      4.3 leaves it open): see orc_hub_merged_sketch.
 *   The paper's own Boyer-Moore rule (Algorithm 3) is available as a second
 *   per-vertex rule (k == ORC_BM_PAPER), run by the same Jacobi driver.
 *   R14 double scan (Section 4.4; Algorithm 4 rescan): the candidates are the
 *      labels of the live slots (value > 0) after the single scan; a second
 *      pass over the row in CSR order sums each candidate's exact weight in
 *      fp32, and the heaviest candidate wins (ties to the lowest label; no
 *      candidate keeps the label).
 * fp32 arithmetic is plain IEEE single precision in program order (build
 * with -ffp-contract=off and without -ffast-math).  Modularity is fp64.
 */
#include "lpa_oracle.h"

#include <float.h>
#include <limits.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------- */
/* Weighted Misra-Gries sketch, k slots (Section 4.1; reading R1).         */
/* ---------------------------------------------------------------------- */

void orc_sketch_clear(int k, int32_t *key, float *val) {
  for (int s = 0; s < k; ++s) {
    key[s] = -1;
    val[s] = 0.0f;
  }
}

void orc_sketch_accumulate(int k, int32_t *key, float *val, int32_t c,
                           float w) {
  /* a pair of weight zero changes nothing (reading R11) */
  if (w == 0.0f) return;
  /* the slot whose label is c takes the weight, whatever its value: the
   * first test of Algorithm 2 looks at the slot's label only, so a label
   * whose slot was emptied by a decrement returns to that same slot */
  for (int s = 0; s < k; ++s) {
    if (key[s] == c) {
      val[s] = val[s] + w;
      return;
    }
  }
  /* otherwise the lowest free slot (value zero) takes the pair: the first
   * set bit of Algorithm 2's free-slot ballot */
  for (int s = 0; s < k; ++s) {
    if (val[s] == 0.0f) {
      key[s] = c;
      val[s] = w;
      return;
    }
  }
  /* all slots live: decrement every slot by d = min(w, smallest value) */
  float d = w;
  for (int s = 0; s < k; ++s)
    if (val[s] < d) d = val[s];
  for (int s = 0; s < k; ++s) val[s] = val[s] - d;
  /* what is left of w (if anything) goes into the lowest slot that just
   * emptied */
  float r = w - d;
  if (r > 0.0f) {
    for (int s = 0; s < k; ++s) {
      if (val[s] == 0.0f) {
        key[s] = c;
        val[s] = r;
        return;
      }
    }
  }
}

int32_t orc_sketch_max_key(int k, const int32_t *key, const float *val,
                           int32_t keep) {
  int found = 0;
  int32_t best = keep;
  float bv = 0.0f;
  for (int s = 0; s < k; ++s) {
    if (!(val[s] > 0.0f)) continue;
    if (!found || val[s] > bv || (val[s] == bv && key[s] < best)) {
      best = key[s];
      bv = val[s];
      found = 1;
    }
  }
  return best;
}

void orc_sketch_feed(int k, int64_t len, const int32_t *labels, const float *w,
                     int32_t *key, float *val) {
  orc_sketch_clear(k, key, val);
  for (int64_t t = 0; t < len; ++t)
    orc_sketch_accumulate(k, key, val, labels[t], w ? w[t] : 1.0f);
}

/* ---------------------------------------------------------------------- */
/* Weighted Boyer-Moore vote of Algorithm 3 (scan loop of its lpaMove).    */
/* ---------------------------------------------------------------------- */

static void bm_paper_step(int32_t *cand, float *wc, int32_t c, float w) {
  if (c == *cand) {
    *wc = *wc + w;
  } else if (*wc > w) {
    *wc = *wc - w;
  } else {
    *cand = c;
    *wc = w;
  }
}

int32_t orc_bm_paper_feed(int64_t len, const int32_t *labels, const float *w,
                          int32_t init, float *weight) {
  int32_t cand = init;
  float wc = 0.0f;
  for (int64_t t = 0; t < len; ++t)
    bm_paper_step(&cand, &wc, labels[t], w ? w[t] : 1.0f);
  if (weight) *weight = wc;
  return cand;
}

/* ---------------------------------------------------------------------- */
/* Per-vertex choice: the label c@ a vertex would adopt.                    */
/* ---------------------------------------------------------------------- */

/* Sketch path: neighbours fed in CSR order, the vertex itself skipped
 * (Algorithm 1, scan loop), then sketchMaxKey. */
static int32_t choose_sketch(int32_t i, const int32_t *row_ptr,
                             const int32_t *col, const float *w, int k,
                             const int32_t *C, int32_t *key, float *val) {
  orc_sketch_clear(k, key, val);
  for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
    int32_t j = col[e];
    if (j == i) continue;
    orc_sketch_accumulate(k, key, val, C[j], w ? w[e] : 1.0f);
  }
  return orc_sketch_max_key(k, key, val, C[i]);
}

/* Algorithm 3 path: the candidate starts as the vertex's own label with
 * weight 0 and sees the neighbours in CSR order, the vertex itself skipped;
 * the final candidate is the choice. */
static int32_t choose_bm_paper(int32_t i, const int32_t *row_ptr,
                               const int32_t *col, const float *w,
                               const int32_t *C) {
  int32_t cand = C[i];
  float wc = 0.0f;
  for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
    int32_t j = col[e];
    if (j == i) continue;
    bm_paper_step(&cand, &wc, C[j], w ? w[e] : 1.0f);
  }
  return cand;
}

/* Double scan (Section 4.4, Algorithm 4 rescan; reading R14): the single
 * scan's live sketch labels are the candidates; their exact weights are
 * summed in CSR order in fp32, then the heaviest wins (ties to the lowest
 * label, none keeps). */
static int32_t choose_rescan(int32_t i, const int32_t *row_ptr,
                             const int32_t *col, const float *w, int k,
                             const int32_t *C, int32_t *key, float *val) {
  orc_sketch_clear(k, key, val);
  for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
    int32_t j = col[e];
    if (j == i) continue;
    orc_sketch_accumulate(k, key, val, C[j], w ? w[e] : 1.0f);
  }
  /* candidates: distinct labels of the live slots, with fresh sums */
  int32_t cand[64];
  float sum[64];
  int nc = 0;
  for (int s = 0; s < k; ++s) {
    if (!(val[s] > 0.0f)) continue;
    int dup = 0;
    for (int q = 0; q < nc; ++q) dup |= cand[q] == key[s];
    if (!dup) {
      cand[nc] = key[s];
      sum[nc] = 0.0f;
      ++nc;
    }
  }
  for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
    int32_t j = col[e];
    if (j == i) continue;
    for (int q = 0; q < nc; ++q)
      if (cand[q] == C[j]) sum[q] = sum[q] + (w ? w[e] : 1.0f);
  }
  int32_t best = C[i];
  float bv = 0.0f;
  int found = 0;
  for (int q = 0; q < nc; ++q) {
    if (sum[q] > 0.0f && (!found || sum[q] > bv || (sum[q] == bv && cand[q] < best))) {
      best = cand[q];
      bv = sum[q];
      found = 1;
    }
  }
  return best;
}

/* Exact path (Eq. 3): K_{i->c} for every neighbouring label c, summed in
 * fp32 in CSR order into a dense per-thread array indexed by label (the
 * collision-free table of Section 2), then the argmax with ties to the
 * lowest label. */
static int32_t choose_exact(int32_t i, const int32_t *row_ptr,
                            const int32_t *col, const float *w,
                            const int32_t *C, float *acc, int32_t *touched) {
  int32_t nt = 0;
  for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
    int32_t j = col[e];
    if (j == i) continue;
    int32_t c = C[j];
    if (acc[c] == 0.0f) touched[nt++] = c;
    acc[c] = acc[c] + (w ? w[e] : 1.0f);
  }
  int32_t best = C[i];
  float bv = 0.0f;
  int found = 0;
  for (int32_t t = 0; t < nt; ++t) {
    int32_t c = touched[t];
    float v = acc[c];
    if (v > 0.0f && (!found || v > bv || (v == bv && c < best))) {
      best = c;
      bv = v;
      found = 1;
    }
    acc[c] = 0.0f;
  }
  return best;
}

static int resolve_threads(int nthreads) {
#ifdef _OPENMP
  return nthreads > 0 ? nthreads : omp_get_max_threads();
#else
  (void)nthreads;
  return 1;
#endif
}

int orc_max_threads(void) { return resolve_threads(0); }

/* ---------------------------------------------------------------------- */
/* One iteration (Algorithm 1, lpaMove) in Jacobi form.                     */
/* ---------------------------------------------------------------------- */

int64_t orc_lpa_move(int32_t n, const int32_t *row_ptr, const int32_t *col,
                     const float *w, int k, int rescan, int pickless, const int32_t *C,
                     const uint8_t *act, int32_t *C_next, uint8_t *act_next,
                     int nthreads, int64_t *scanned) {
  int64_t dN = 0, sc = 0;
  int nt = resolve_threads(nthreads);
  memcpy(C_next, C, (size_t)n * sizeof(int32_t));
#pragma omp parallel num_threads(nt) reduction(+ : dN, sc)
  {
    int32_t key[64];
    float val[64];
    float *acc = NULL;
    int32_t *touched = NULL;
    if (k == 0) {
      acc = (float *)calloc((size_t)n + 1, sizeof(float));
      touched = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    }
#pragma omp for schedule(dynamic, 256)
    for (int32_t i = 0; i < n; ++i) {
      if (!act[i]) continue; /* only unprocessed vertices */
      sc += row_ptr[i + 1] - row_ptr[i];
      int32_t c = (k == 0)   ? choose_exact(i, row_ptr, col, w, C, acc, touched)
                  : (k < 0) ? choose_bm_paper(i, row_ptr, col, w, C)
                  : rescan  ? choose_rescan(i, row_ptr, col, w, k, C, key, val)
                            : choose_sketch(i, row_ptr, col, w, k, C, key, val);
      if (c != C[i] && (!pickless || c < C[i])) {
        C_next[i] = c;
        dN += 1;
        /* mark every CSR neighbour unprocessed for the next iteration;
         * plain byte stores of the same value, so order cannot matter */
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
          act_next[col[e]] = 1;
      }
    }
    free(acc);
    free(touched);
  }
  if (scanned) *scanned = sc;
  return dN;
}

/* ---------------------------------------------------------------------- */
/* Driver (Algorithm 1, lpa).                                               */
/* ---------------------------------------------------------------------- */

int orc_lpa_run(int32_t n, const int32_t *row_ptr, const int32_t *col,
                const float *w, int k, int rescan, double tol, int max_iter, int rho,
                int nthreads, int32_t *labels, int64_t *dN_trace,
                int64_t *scanned_trace) {
  if (n < 0 || (k < 0 && k != ORC_BM_PAPER) || k > 64 || max_iter < 0 || rho < 0 ||
      (rescan && k <= 0))
    return -1;
  for (int32_t i = 0; i < n; ++i) labels[i] = i; /* unique initial labels */
  if (dN_trace)
    for (int l = 0; l < max_iter; ++l) dN_trace[l] = 0;
  if (scanned_trace)
    for (int l = 0; l < max_iter; ++l) scanned_trace[l] = 0;
  if (n == 0) return 0;

  int32_t *Cn = (int32_t *)malloc((size_t)n * sizeof(int32_t));
  uint8_t *act = (uint8_t *)malloc((size_t)n);
  uint8_t *actn = (uint8_t *)malloc((size_t)n);
  memset(act, 1, (size_t)n); /* every vertex starts unprocessed */
  int iters = max_iter;
  for (int l = 0; l < max_iter; ++l) {
    int pickless = (rho > 0) && (l % rho == 0);
    memset(actn, 0, (size_t)n);
    int64_t sc = 0;
    int64_t dN = orc_lpa_move(n, row_ptr, col, w, k, rescan, pickless, labels, act,
                              Cn, actn, nthreads, &sc);
    memcpy(labels, Cn, (size_t)n * sizeof(int32_t));
    uint8_t *t = act;
    act = actn;
    actn = t;
    if (dN_trace) dN_trace[l] = dN;
    if (scanned_trace) scanned_trace[l] = sc;
    if (!pickless && (double)dN / (double)n < tol) {
      iters = l + 1;
      break;
    }
  }
  free(Cn);
  free(act);
  free(actn);
  return iters;
}

void orc_lpa_choose(int32_t n, const int32_t *row_ptr, const int32_t *col,
                    const float *w, int k, int rescan, int pickless, const int32_t *C,
                    int64_t nv, const int32_t *verts, int32_t *out,
                    int nthreads) {
  int nt = resolve_threads(nthreads);
#pragma omp parallel num_threads(nt)
  {
    int32_t key[64];
    float val[64];
    float *acc = NULL;
    int32_t *touched = NULL;
    if (k == 0) {
      acc = (float *)calloc((size_t)n + 1, sizeof(float));
      touched = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
    }
#pragma omp for schedule(dynamic, 64)
    for (int64_t q = 0; q < nv; ++q) {
      int32_t i = verts[q];
      int32_t c = (k == 0)   ? choose_exact(i, row_ptr, col, w, C, acc, touched)
                  : (k < 0) ? choose_bm_paper(i, row_ptr, col, w, C)
                  : rescan  ? choose_rescan(i, row_ptr, col, w, k, C, key, val)
                            : choose_sketch(i, row_ptr, col, w, k, C, key, val);
      out[q] = (c != C[i] && (!pickless || c < C[i])) ? c : C[i];
    }
    free(acc);
    free(touched);
  }
}

/* ---------------------------------------------------------------------- */
/* Partial sketches of a high-degree vertex (Section 4.3; reading R9).     */
/* ---------------------------------------------------------------------- */

/* Feed the live slots of sketch (pk, pv) into (key, val), slot by slot. */
static void feed_live(int k, int32_t *key, float *val, const int32_t *pk,
                      const float *pv) {
  for (int s = 0; s < k; ++s)
    if (pv[s] > 0.0f) orc_sketch_accumulate(k, key, val, pk[s], pv[s]);
}

/* Sketch of segment q of vertex v's row: entries [b + q S, b + (q+1) S)
 * in CSR order, the vertex itself skipped. */
static void segment_sketch(const int32_t *row_ptr, const int32_t *col,
                           const float *w, int k, int32_t seg_len,
                           const int32_t *C, int32_t v, int64_t q,
                           int32_t *key, float *val) {
  int64_t b = (int64_t)row_ptr[v] + q * seg_len;
  int64_t e = b + seg_len;
  if (e > row_ptr[v + 1]) e = row_ptr[v + 1];
  orc_sketch_clear(k, key, val);
  for (int64_t t = b; t < e; ++t) {
    if (col[t] == v) continue;
    orc_sketch_accumulate(k, key, val, C[col[t]], w ? w[t] : 1.0f);
  }
}

int64_t orc_hub_merged_sketch(const int32_t *row_ptr, const int32_t *col,
                              const float *w, int k, int32_t seg_len,
                              const int32_t *C, int32_t v, int32_t *key,
                              float *val) {
  if (k < 1 || k > 64 || seg_len < 1) return -1;
  const int64_t deg = (int64_t)row_ptr[v + 1] - row_ptr[v];
  const int64_t np = (deg + seg_len - 1) / seg_len;
  int32_t pk[64];
  float pv[64];
  orc_sketch_clear(k, key, val);
  if (np <= ORC_MERGE_CHAINS) {
    /* every partial, in segment order, into one sketch */
    for (int64_t q = 0; q < np; ++q) {
      segment_sketch(row_ptr, col, w, k, seg_len, C, v, q, pk, pv);
      feed_live(k, key, val, pk, pv);
    }
    return np;
  }
  /* ORC_MERGE_CHAINS chains: chain t takes partials t, t + 64, t + 128, ...
   * in that order; then rounds at distance 32, 16, 8, 4, 2, 1, in each of
   * which every chain t absorbs what chain t ^ distance held at the start
   * of the round; the result is chain 0 */
  const int nc = ORC_MERGE_CHAINS;
  int32_t *ck = (int32_t *)malloc((size_t)nc * k * sizeof(int32_t));
  float *cw = (float *)malloc((size_t)nc * k * sizeof(float));
  int32_t *sk = (int32_t *)malloc((size_t)nc * k * sizeof(int32_t));
  float *sw = (float *)malloc((size_t)nc * k * sizeof(float));
  if (!ck || !cw || !sk || !sw) {
    free(ck);
    free(cw);
    free(sk);
    free(sw);
    return -1;
  }
  for (int t = 0; t < nc; ++t) orc_sketch_clear(k, ck + t * k, cw + t * k);
  for (int64_t q = 0; q < np; ++q) {
    const int t = (int)(q % nc);
    segment_sketch(row_ptr, col, w, k, seg_len, C, v, q, pk, pv);
    feed_live(k, ck + t * k, cw + t * k, pk, pv);
  }
  for (int dist = nc / 2; dist >= 1; dist /= 2) {
    memcpy(sk, ck, (size_t)nc * k * sizeof(int32_t));
    memcpy(sw, cw, (size_t)nc * k * sizeof(float));
    for (int t = 0; t < nc; ++t)
      feed_live(k, ck + t * k, cw + t * k, sk + (t ^ dist) * k, sw + (t ^ dist) * k);
  }
  memcpy(key, ck, (size_t)k * sizeof(int32_t));
  memcpy(val, cw, (size_t)k * sizeof(float));
  free(ck);
  free(cw);
  free(sk);
  free(sw);
  return np;
}

/* Choice of a high-degree vertex from its merged partial sketch: the
 * heaviest slot; with rescan, the merged sketch's live labels re-weighted
 * exactly over the whole row (fp32 sums in CSR order). */
static int32_t choose_hub(const int32_t *row_ptr, const int32_t *col,
                          const float *w, int k, int rescan, int32_t seg_len,
                          const int32_t *C, int32_t v) {
  int32_t key[64];
  float val[64];
  if (orc_hub_merged_sketch(row_ptr, col, w, k, seg_len, C, v, key, val) < 0)
    return C[v];
  if (!rescan) return orc_sketch_max_key(k, key, val, C[v]);
  float sum[64];
  for (int s = 0; s < k; ++s) sum[s] = 0.0f;
  for (int32_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
    if (col[e] == v) continue;
    for (int s = 0; s < k; ++s)
      if (val[s] > 0.0f && key[s] == C[col[e]]) sum[s] = sum[s] + (w ? w[e] : 1.0f);
  }
  int32_t best = C[v];
  float bv = 0.0f;
  int found = 0;
  for (int s = 0; s < k; ++s) {
    if (sum[s] > 0.0f && (!found || sum[s] > bv || (sum[s] == bv && key[s] < best))) {
      best = key[s];
      bv = sum[s];
      found = 1;
    }
  }
  return best;
}

void orc_hub_choose(int32_t n, const int32_t *row_ptr, const int32_t *col,
                    const float *w, int k, int rescan, int32_t seg_len,
                    int pickless, const int32_t *C, int64_t nv,
                    const int32_t *verts, int32_t *out, int nthreads) {
  (void)n;
  int nt = resolve_threads(nthreads);
#pragma omp parallel for num_threads(nt) schedule(dynamic, 4)
  for (int64_t q = 0; q < nv; ++q) {
    int32_t i = verts[q];
    int32_t c = choose_hub(row_ptr, col, w, k, rescan, seg_len, C, i);
    out[q] = (c != C[i] && (!pickless || c < C[i])) ? c : C[i];
  }
}

/* ---------------------------------------------------------------------- */
/* Modularity, Eq. 1 in its community-sum form, fp64, index order.          */
/* ---------------------------------------------------------------------- */

double orc_modularity(int32_t n, const int32_t *row_ptr, const int32_t *col,
                      const float *w, const int32_t *C) {
  double two_m = 0.0, sigma_in = 0.0;
  double *tot = (double *)calloc((size_t)n + 1, sizeof(double));
  for (int32_t i = 0; i < n; ++i) {
    double Ki = 0.0;
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      double we = w ? (double)w[e] : 1.0;
      Ki += we;
      if (C[col[e]] == C[i]) sigma_in += we; /* sigma_c, both directions */
    }
    two_m += Ki;
    tot[C[i]] += Ki; /* Sigma_c */
  }
  double q = 0.0;
  if (two_m > 0.0) {
    double sq = 0.0;
    for (int32_t c = 0; c < n; ++c) sq += (tot[c] / two_m) * (tot[c] / two_m);
    q = sigma_in / two_m - sq;
  }
  free(tot);
  return q;
}
