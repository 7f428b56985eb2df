/*
 * Seeded synthetic graph generators (input preparation only).
 *
 * Every generator here writes a symmetric CSR graph: row_ptr int32[n+1],
 * col int32[nnz], neighbour lists sorted ascending, no duplicates, no
 * self-loops.  They hold none of the label-propagation arithmetic; both the
 * CPU oracle and the GPU library consume what they produce.
 *
 * Randomness is counter based: every draw is splitmix64-style mixing of
 * (seed, stream, index), so results do not depend on thread count or
 * scheduling.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct gg_graph {
  int32_t n;
  int64_t nnz;
  int32_t *row_ptr;
  int32_t *col;
} gg_graph;

/* ------------------------------------------------------------------ */
/* counter-based random numbers                                         */
/* ------------------------------------------------------------------ */

static inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t gg_hash3(uint64_t seed, uint64_t a, uint64_t b) {
  return mix64(mix64(mix64(seed) ^ a) + 0x632BE59BD9B4E019ull * (b + 1));
}

/* uniform double in [0, 1) with 53 random bits */
static inline double u01(uint64_t h) { return (double)(h >> 11) * 0x1.0p-53; }

double gg_uniform(uint64_t seed, uint64_t a, uint64_t b) {
  return u01(gg_hash3(seed, a, b));
}

/* ------------------------------------------------------------------ */
/* CSR assembly                                                          */
/* ------------------------------------------------------------------ */

static void insertion_sort(int32_t *a, int64_t len) {
  for (int64_t i = 1; i < len; ++i) {
    int32_t x = a[i];
    int64_t j = i - 1;
    while (j >= 0 && a[j] > x) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = x;
  }
}

/* in-place quicksort of int32 (median of three, small parts by insertion) */
static void sort_row(int32_t *a, int64_t len) {
  while (len > 24) {
    int32_t x = a[0], y = a[len / 2], z = a[len - 1];
    int32_t p = x < y ? (y < z ? y : (x < z ? z : x)) : (x < z ? x : (y < z ? z : y));
    int64_t i = 0, j = len - 1;
    for (;;) {
      while (a[i] < p) ++i;
      while (a[j] > p) --j;
      if (i >= j) break;
      int32_t t = a[i];
      a[i] = a[j];
      a[j] = t;
      ++i;
      --j;
    }
    /* recurse into the smaller side, loop on the larger */
    int64_t left = j + 1;
    if (left < len - left) {
      sort_row(a, left);
      a += left;
      len -= left;
    } else {
      sort_row(a + left, len - left);
      len = left;
    }
  }
  insertion_sort(a, len);
}

/* tmp holds, for each vertex i, deg0[i] unsorted neighbour ids starting at
 * off[i].  Sort and dedupe every row, then pack into a fresh CSR.  Frees
 * tmp and off.  Returns 0, or -1 when nnz does not fit int32 offsets. */
static int pack_rows(int32_t n, int64_t *off, int32_t *tmp, gg_graph *g) {
  int64_t *newdeg = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t i = 0; i < n; ++i) {
    int32_t *a = tmp + off[i];
    int64_t len = off[i + 1] - off[i];
    sort_row(a, len);
    int64_t m = 0;
    for (int64_t t = 0; t < len; ++t)
      if (m == 0 || a[t] != a[m - 1]) a[m++] = a[t];
    newdeg[i] = m;
  }
  int64_t total = 0;
  for (int32_t i = 0; i < n; ++i) total += newdeg[i];
  if (total >= INT32_MAX) {
    free(newdeg);
    free(off);
    free(tmp);
    return -1;
  }
  g->n = n;
  g->nnz = total;
  g->row_ptr = (int32_t *)malloc(((size_t)n + 1) * sizeof(int32_t));
  g->col = (int32_t *)malloc((size_t)(total > 0 ? total : 1) * sizeof(int32_t));
  int64_t acc = 0;
  for (int32_t i = 0; i < n; ++i) {
    g->row_ptr[i] = (int32_t)acc;
    acc += newdeg[i];
  }
  g->row_ptr[n] = (int32_t)acc;
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t i = 0; i < n; ++i)
    memcpy(g->col + g->row_ptr[i], tmp + off[i], (size_t)newdeg[i] * sizeof(int32_t));
  free(newdeg);
  free(off);
  free(tmp);
  return 0;
}

/* Build from an undirected pair list (both directions are inserted). */
static int csr_from_pairs(int32_t n, int64_t m, const int32_t *pu,
                          const int32_t *pv, gg_graph *g) {
  int64_t *off = (int64_t *)calloc((size_t)n + 2, sizeof(int64_t));
  for (int64_t t = 0; t < m; ++t) {
    if (pu[t] == pv[t]) continue;
    off[pu[t] + 1]++;
    off[pv[t] + 1]++;
  }
  for (int32_t i = 0; i < n; ++i) off[i + 1] += off[i];
  int64_t tot = off[n];
  int32_t *tmp = (int32_t *)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(int32_t));
  int64_t *cur = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  memcpy(cur, off, ((size_t)n + 1) * sizeof(int64_t));
  for (int64_t t = 0; t < m; ++t) {
    if (pu[t] == pv[t]) continue;
    tmp[cur[pu[t]]++] = pv[t];
    tmp[cur[pv[t]]++] = pu[t];
  }
  free(cur);
  return pack_rows(n, off, tmp, g);
}

void gg_free(gg_graph *g) {
  if (!g) return;
  free(g->row_ptr);
  free(g->col);
  g->row_ptr = NULL;
  g->col = NULL;
}

/* ------------------------------------------------------------------ */
/* Stochastic block model (planted partition)                            */
/* ------------------------------------------------------------------ */

typedef struct {
  int64_t cap, m;
  int32_t *u, *v;
} pairbuf;

static void pb_push(pairbuf *b, int32_t u, int32_t v) {
  if (b->m == b->cap) {
    b->cap = b->cap ? 2 * b->cap : 1024;
    b->u = (int32_t *)realloc(b->u, (size_t)b->cap * sizeof(int32_t));
    b->v = (int32_t *)realloc(b->v, (size_t)b->cap * sizeof(int32_t));
  }
  b->u[b->m] = u;
  b->v[b->m] = v;
  b->m++;
}

/* Geometric gap to the next success of Bernoulli(p) trials. */
static inline int64_t geo_skip(double p, uint64_t h) {
  if (p >= 1.0) return 0;
  double U = 1.0 - u01(h); /* (0, 1] */
  double s = floor(log(U) / log1p(-p));
  if (s > 9.0e18) return INT64_MAX / 4;
  return (int64_t)s;
}

/* Blocks: nb blocks, block b holds vertices [start[b], start[b+1]).  Each
 * unordered pair is an edge with probability p_in inside a block and p_out
 * across blocks. */
int gg_sbm(int32_t nb, const int32_t *start, double p_in, double p_out,
           uint64_t seed, gg_graph *g) {
  int32_t n = start[nb];
  pairbuf pb = {0, 0, NULL, NULL};
  for (int32_t b1 = 0; b1 < nb; ++b1) {
    for (int32_t b2 = b1; b2 < nb; ++b2) {
      double p = (b1 == b2) ? p_in : p_out;
      if (p <= 0.0) continue;
      int64_t s1 = start[b1 + 1] - start[b1], s2 = start[b2 + 1] - start[b2];
      int64_t P = (b1 == b2) ? s1 * (s1 - 1) / 2 : s1 * s2;
      uint64_t stream = (uint64_t)b1 * (uint64_t)nb + (uint64_t)b2;
      int64_t t = -1, draw = 0;
      /* row cursor for the triangular enumeration of a diagonal block */
      int64_t r = 0, rbase = 0;
      for (;;) {
        t += 1 + geo_skip(p, gg_hash3(seed, stream, (uint64_t)draw++));
        if (t >= P) break;
        int32_t u, v;
        if (b1 == b2) {
          while (t >= rbase + (s1 - 1 - r)) {
            rbase += s1 - 1 - r;
            ++r;
          }
          u = start[b1] + (int32_t)r;
          v = start[b1] + (int32_t)(r + 1 + (t - rbase));
        } else {
          u = start[b1] + (int32_t)(t / s2);
          v = start[b2] + (int32_t)(t % s2);
        }
        pb_push(&pb, u, v);
      }
    }
  }
  int rc = csr_from_pairs(n, pb.m, pb.u, pb.v, g);
  free(pb.u);
  free(pb.v);
  return rc;
}

/* ------------------------------------------------------------------ */
/* R-MAT (recursive matrix) graphs                                        */
/* ------------------------------------------------------------------ */

/* One counter hash per sampled edge seeds a splitmix64 stream; each level
 * consumes 32 bits compared against 32-bit fixed-point thresholds. */
static inline void rmat_edge(int scale, uint32_t ta, uint32_t tab, uint32_t tabc,
                             uint64_t seed, uint64_t e, int32_t *pu, int32_t *pv) {
  uint32_t u = 0, v = 0;
  uint64_t state = gg_hash3(seed, e, 0x5241544dull), bits = 0;
  for (int lv = 0; lv < scale; ++lv) {
    if ((lv & 1) == 0) {
      state += 0x9E3779B97F4A7C15ull;
      bits = mix64(state);
    }
    uint32_t r = (lv & 1) ? (uint32_t)(bits >> 32) : (uint32_t)bits;
    uint32_t ub = r >= tab, vb = (r >= ta && r < tab) || r >= tabc;
    u = (u << 1) | ub;
    v = (v << 1) | vb;
  }
  *pu = (int32_t)u;
  *pv = (int32_t)v;
}

static uint32_t fixed32(double p) {
  double x = p * 4294967296.0;
  if (x >= 4294967295.0) return 0xFFFFFFFFu;
  if (x <= 0.0) return 0u;
  return (uint32_t)x;
}

/* 2^scale vertices, edge_factor * 2^scale sampled edges; self-loops and
 * duplicates dropped; symmetrised.  No vertex-id permutation. */
int gg_rmat(int scale, int edge_factor, double a, double b, double c,
            uint64_t seed, gg_graph *g) {
  if (scale < 1 || scale > 30) return -2;
  int32_t n = (int32_t)1 << scale;
  int64_t m = (int64_t)edge_factor << scale;
  const uint32_t ta = fixed32(a), tab = fixed32(a + b), tabc = fixed32(a + b + c);
  int64_t *off = (int64_t *)calloc((size_t)n + 2, sizeof(int64_t));
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    int32_t u, v;
    rmat_edge(scale, ta, tab, tabc, seed, (uint64_t)e, &u, &v);
    if (u == v) continue;
    __atomic_fetch_add(&off[u + 1], 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(&off[v + 1], 1, __ATOMIC_RELAXED);
  }
  for (int32_t i = 0; i < n; ++i) off[i + 1] += off[i];
  int64_t tot = off[n];
  int32_t *tmp = (int32_t *)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(int32_t));
  int64_t *cur = (int64_t *)malloc(((size_t)n + 1) * sizeof(int64_t));
  memcpy(cur, off, ((size_t)n + 1) * sizeof(int64_t));
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < m; ++e) {
    int32_t u, v;
    rmat_edge(scale, ta, tab, tabc, seed, (uint64_t)e, &u, &v);
    if (u == v) continue;
    tmp[__atomic_fetch_add(&cur[u], 1, __ATOMIC_RELAXED)] = v;
    tmp[__atomic_fetch_add(&cur[v], 1, __ATOMIC_RELAXED)] = u;
  }
  free(cur);
  return pack_rows(n, off, tmp, g);
}

/* ------------------------------------------------------------------ */
/* Road-like grid: R x Cc lattice, edges deleted with p_del, survivors   */
/* rewired with p_rw (larger-id endpoint replaced by a uniform vertex).  */
/* ------------------------------------------------------------------ */

int gg_grid(int32_t R, int32_t Cc, double p_del, double p_rw, uint64_t seed,
            gg_graph *g) {
  int64_t n64 = (int64_t)R * Cc;
  if (n64 <= 0 || n64 >= INT32_MAX) return -2;
  int32_t n = (int32_t)n64;
  int64_t H = (int64_t)R * (Cc - 1), V = (int64_t)(R - 1) * Cc;
  int64_t m = H + V;
  int32_t *pu = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  int32_t *pv = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
#pragma omp parallel for schedule(static)
  for (int64_t eid = 0; eid < m; ++eid) {
    int32_t u, v;
    if (eid < H) {
      int64_t r = eid / (Cc - 1), c = eid % (Cc - 1);
      u = (int32_t)(r * Cc + c);
      v = u + 1;
    } else {
      int64_t t = eid - H, r = t / Cc, c = t % Cc;
      u = (int32_t)(r * Cc + c);
      v = u + Cc;
    }
    if (u01(gg_hash3(seed, (uint64_t)eid, 0)) < p_del) {
      pu[eid] = 0;
      pv[eid] = 0; /* marked as self-loop: dropped */
      continue;
    }
    if (u01(gg_hash3(seed, (uint64_t)eid, 1)) < p_rw) {
      int32_t keep = u < v ? u : v;
      uint64_t draw = 2;
      int32_t nv;
      do {
        nv = (int32_t)(gg_hash3(seed, (uint64_t)eid, draw++) % (uint64_t)n);
      } while (nv == keep);
      u = keep;
      v = nv;
    }
    pu[eid] = u;
    pv[eid] = v;
  }
  int rc = csr_from_pairs(n, m, pu, pv, g);
  free(pu);
  free(pv);
  return rc;
}

/* ------------------------------------------------------------------ */
/* Edge weights                                                           */
/* ------------------------------------------------------------------ */

/* w = (u + 1) * 2^-24 with u uniform in [0, 2^24), drawn from the
 * unordered endpoint pair so that w_ij == w_ji; every value is exact in
 * fp32 and lies in (0, 1]. */
void gg_weights_uniform(int32_t n, const int32_t *row_ptr, const int32_t *col,
                        uint64_t seed, float *w) {
#pragma omp parallel for schedule(dynamic, 4096)
  for (int32_t i = 0; i < n; ++i) {
    for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      int32_t j = col[e];
      uint64_t lo = (uint64_t)(i < j ? i : j), hi = (uint64_t)(i < j ? j : i);
      uint64_t u = gg_hash3(seed, lo, hi) >> 40;
      w[e] = (float)(u + 1) * 0x1.0p-24f;
    }
  }
}
