// C-ABI runtime of liblpa.so: handle, device state, auxiliary kernels and
// the iteration driver (paper Algorithm 1, lpa).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

#include "lpa_internal.h"

using namespace lpa;

// ===========================================================================
// Auxiliary kernels
// ===========================================================================
namespace {

constexpr int kAuxBlock = 256;

__global__ void k_fill_i32_iota(int32_t *C, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) C[i] = i;
}

__global__ void k_fill_u8(uint8_t *p, size_t count, uint8_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

__global__ void k_normalize_u8(uint8_t *p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    p[i] = p[i] ? 1 : 0;
}

// bad |= 1: row_ptr; 2: col out of range; 4: weight not finite or <= 0
__global__ void k_validate(int n, int64_t nnz, const int32_t *rp, const int32_t *col,
                           const float *w, int *bad) {
  const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  int b = 0;
  if (tid == 0 && (rp[0] != 0 || (int64_t)rp[n] != nnz)) b |= 1;
  for (size_t i = tid; i < (size_t)n; i += stride)
    if (rp[i] > rp[i + 1]) b |= 1;
  for (size_t e = tid; e < (size_t)nnz; e += stride) {
    const int j = col[e];
    if (j < 0 || j >= n) b |= 2;
    if (w) {
      const float x = w[e];
      if (!(x > 0.0f) || !isfinite(x)) b |= 4;
    }
  }
  if (b) atomicOr(bad, b);
}

__global__ void k_check_labels(const int32_t *lab, int n, int *bad) {
  int b = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int c = lab[i];
    if (c < 0 || c >= n) b = 8;
  }
  if (b) atomicOr(bad, b);
}

// --- degree binning: histogram -> exclusive scan -> scatter ---------------
__global__ void k_bin_hist(int n, const int32_t *rp, int lane_max, int ncls, unsigned *hist) {
  extern __shared__ unsigned sh[];
  for (int c = threadIdx.x; c < ncls; c += blockDim.x) sh[c] = 0;
  __syncthreads();
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
    const int d = rp[v + 1] - rp[v];
    if (d > 0) atomicAdd(&sh[degree_class(d, lane_max)], 1u);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < ncls; c += blockDim.x)
    if (sh[c]) atomicAdd(&hist[c], sh[c]);
}

// hist becomes exclusive offsets; totals[0] = hubs, totals[1] = lane vertices
__global__ void k_bin_scan(int ncls, unsigned *hist, int *totals) {
  if (threadIdx.x != 0) return;
  unsigned acc = 0, hubs = 0;
  for (int c = 0; c < ncls; ++c) {
    const unsigned x = hist[c];
    hist[c] = acc;
    acc += x;
    if (c < kHubClasses) hubs += x;
  }
  totals[0] = (int)hubs;
  totals[1] = (int)(acc - hubs);
}

constexpr int kScatterItems = 16;
__global__ void k_bin_scatter(int n, const int32_t *rp, int lane_max, int ncls, unsigned *cursor,
                              int32_t *order) {
  extern __shared__ unsigned sh[];  // [ncls] local counts, then [ncls] bases
  unsigned *cnt = sh;
  unsigned *base = sh + ncls;
  for (int c = threadIdx.x; c < ncls; c += blockDim.x) cnt[c] = 0;
  __syncthreads();
  const int v0 = blockIdx.x * blockDim.x * kScatterItems;
  int cls[kScatterItems];
  unsigned rank[kScatterItems];
#pragma unroll
  for (int t = 0; t < kScatterItems; ++t) {
    const int v = v0 + t * blockDim.x + threadIdx.x;
    cls[t] = -1;
    if (v < n) {
      const int d = rp[v + 1] - rp[v];
      if (d > 0) {
        cls[t] = degree_class(d, lane_max);
        rank[t] = atomicAdd(&cnt[cls[t]], 1u);
      }
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < ncls; c += blockDim.x)
    base[c] = cnt[c] ? atomicAdd(&cursor[c], cnt[c]) : 0u;
  __syncthreads();
#pragma unroll
  for (int t = 0; t < kScatterItems; ++t) {
    const int v = v0 + t * blockDim.x + threadIdx.x;
    if (cls[t] >= 0) order[base[cls[t]] + rank[t]] = v;
  }
}

// --- iteration epilogue ------------------------------------------------------
// Async hub segments: pbase[h] = sum over earlier hubs of ceil(deg / S);
// pbase[n_hubs] (also written to *total) = number of segments.  One block.
__global__ void k_hub_plan(const int32_t *order, int n_hubs, const int32_t *rp, int S,
                           int32_t *pbase, int *total) {
  __shared__ long long part[1024];
  const int t = threadIdx.x, nt = blockDim.x;
  const int per = (n_hubs + nt - 1) / nt;
  const int h0 = t * per, h1 = min(n_hubs, h0 + per);
  long long s = 0;
  for (int h = h0; h < h1; ++h) {
    const int v = order[h];
    s += (rp[v + 1] - rp[v] + S - 1) / S;
  }
  part[t] = s;
  __syncthreads();
  if (t == 0) {
    long long acc = 0;
    for (int i = 0; i < nt; ++i) {
      const long long x = part[i];
      part[i] = acc;
      acc += x;
    }
    pbase[n_hubs] = (int32_t)acc;
    *total = (int)acc;
  }
  __syncthreads();
  long long acc = part[t];
  for (int h = h0; h < h1; ++h) {
    pbase[h] = (int32_t)acc;
    const int v = order[h];
    acc += (rp[v + 1] - rp[v] + S - 1) / S;
  }
}

__global__ void k_fill_seg_hub(const int32_t *pbase, int n_hubs, int32_t *seg_hub) {
  for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < n_hubs; h += gridDim.x * blockDim.x)
    for (int q = pbase[h]; q < pbase[h + 1]; ++q) seg_hub[q] = h;
}

// ctl[0] = done, ctl[1] = iterations run
__global__ void k_finish(const unsigned long long *dN, int iter, int n, double tol, int rho,
                         int max_iter, int *ctl) {
  if (threadIdx.x != 0 || ctl[0]) return;
  const bool pl = rho > 0 && iter % rho == 0;
  ctl[1] = iter + 1;
  const double frac = (double)dN[iter] / (double)n;
  if ((!pl && frac < tol) || iter + 1 >= max_iter) ctl[0] = 1;
}

__global__ void k_clear_err(int *ctl) {
  if (threadIdx.x == 0) ctl[2] = 0;
}

__global__ void k_set_ctl(int *ctl, int done, int iters) {
  if (threadIdx.x == 0) {
    ctl[0] = done;
    ctl[1] = iters;
    ctl[2] = 0;
  }
}

// --- modularity (Eq. 1, community-sum form), fp64 --------------------------
__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// acc[0] += K_i (sum = 2m), acc[1] += intra-community weight, tot[C_i] += K_i
__global__ void k_mod_lane(const int32_t *order, int first, int count, const int32_t *rp,
                           const int32_t *col, const float *w, const int32_t *lab, int n,
                           double *tot, double *acc, int *bad) {
  double k_sum = 0.0, in_sum = 0.0;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < count; t += gridDim.x * blockDim.x) {
    const int i = order[first + t];
    const int ci = lab[i];
    if (ci < 0 || ci >= n) {
      atomicOr(bad, 8);
      continue;
    }
    double ki = 0.0, in = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; ++e) {
      const double x = w ? (double)w[e] : 1.0;
      ki += x;
      if (lab[col[e]] == ci) in += x;
    }
    atomicAdd(&tot[ci], ki);
    k_sum += ki;
    in_sum += in;
  }
  k_sum = wave_sum_d(k_sum);
  in_sum = wave_sum_d(in_sum);
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&acc[0], k_sum);
    atomicAdd(&acc[1], in_sum);
  }
}

__global__ void k_mod_hub(const int32_t *order, int count, const int32_t *rp, const int32_t *col,
                          const float *w, const int32_t *lab, int n, double *tot, double *acc,
                          int *bad) {
  const int lane = threadIdx.x & 63;
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int nw = (gridDim.x * blockDim.x) >> 6;
  double k_sum = 0.0, in_sum = 0.0;  // lane partial sums over this wave's hubs
  for (int t = wid; t < count; t += nw) {
    const int i = order[t];
    const int ci = lab[i];
    if (ci < 0 || ci >= n) {
      if (lane == 0) atomicOr(bad, 8);
      continue;
    }
    double ki = 0.0;
    for (int e = rp[i] + lane; e < rp[i + 1]; e += 64) {
      const double x = w ? (double)w[e] : 1.0;
      ki += x;
      if (lab[col[e]] == ci) in_sum += x;
    }
    k_sum += ki;
    ki = wave_sum_d(ki);
    if (lane == 0) atomicAdd(&tot[ci], ki);
  }
  k_sum = wave_sum_d(k_sum);
  in_sum = wave_sum_d(in_sum);
  if (lane == 0) {
    atomicAdd(&acc[0], k_sum);
    atomicAdd(&acc[1], in_sum);
  }
}

// acc[2] += sum_c tot[c]^2; clears tot for the next call
__global__ void k_mod_sq(double *tot, int n, double *acc) {
  double s = 0.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    const double x = tot[c];
    s += x * x;
    tot[c] = 0.0;
  }
  s = wave_sum_d(s);
  if ((threadIdx.x & 63) == 0) atomicAdd(&acc[2], s);
}

// Only the memory accesses of one full scan: stream col and w, gather
// C[col]; the sum is written only if it takes an impossible value.
__global__ void k_scan_floor(const int32_t *col, const float *w, const int32_t *C, int64_t nnz,
                             unsigned long long *sink) {
  unsigned long long acc = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int j = __builtin_nontemporal_load(col + e);
    const float x = w ? __builtin_nontemporal_load(w + e) : 1.0f;
    acc += (unsigned)C[j] + (x > 2.0f ? 1u : 0u);
  }
  if (acc == ~0ull) *sink = acc;
}

__global__ void k_zero_d(double *p, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    p[i] = 0.0;
}

int grid_for(size_t count, int block = kAuxBlock, int cap = 4096) {
  size_t g = (count + block - 1) / block;
  if (g < 1) g = 1;
  if (g > (size_t)cap) g = cap;
  return (int)g;
}

}  // namespace

// ===========================================================================
// Handle
// ===========================================================================
struct lpa_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  int32_t n = 0;
  int64_t nnz = 0;
  const int32_t *row_ptr = nullptr;
  const int32_t *col = nullptr;
  const float *w = nullptr;
  int k = 8;
  double tol = 0.05;
  int max_iter = 20;
  int rho = 8;
  uint32_t flags = 0;
  bool async_mode = false;
  uint64_t seed = 0;
  int lane_max = 0;
  int check_every = 0;
  std::vector<hipEvent_t> ev_beg, ev_end;  // per-iteration move timing

  int32_t *C[2] = {nullptr, nullptr};    // det: labels of even / odd iterations; async: C[0]
  uint8_t *act[2] = {nullptr, nullptr};   // det: flags of even / odd iterations; async: act[0]
  int32_t *order = nullptr;
  int32_t *hub_pbase = nullptr;  // async: [n_hubs + 1]
  int32_t *seg_hub = nullptr;    // async: [n_seg]
  uint8_t *hub_act = nullptr;    // async: [n_hubs]
  int32_t *part_key = nullptr;   // async: [n_seg * k]
  float *part_val = nullptr;     // async: [n_seg * k]
  int n_seg = 0;
  int grid_merge = 1;
  unsigned long long *dN = nullptr;       // [max(1, max_iter)]
  unsigned long long *scanned = nullptr;  // [max(1, max_iter)]
  int *ctl = nullptr;                     // [0] done, [1] iterations, [2] error bits, [3..] totals
  double *mod_tot = nullptr;
  double *mod_acc = nullptr;

  int n_hubs = 0, n_lane = 0;
  int grid_move = 1;
  int iter = 0;  // next iteration index (host view)
  bool finished = false;
  size_t core_bytes = 0, eval_bytes = 0;
  bool poisoned = false;
  std::string err;
  std::vector<void *> allocs;
};

namespace {

int set_err(lpa_handle *h, int code, const std::string &msg) {
  if (h) h->err = msg;
  return code;
}

int fail_hip(lpa_handle *h, hipError_t e, const char *what) {
  if (h) {
    h->poisoned = true;
    h->err = std::string(what) + ": " + hipGetErrorString(e);
  }
  return LPA_ERR_HIP;
}

#define HIP_TRY(h, expr)                                 \
  do {                                                   \
    hipError_t _e = (expr);                              \
    if (_e != hipSuccess) return fail_hip((h), _e, #expr); \
  } while (0)

#define LAUNCH_TRY(h, what)                              \
  do {                                                   \
    hipError_t _e = hipGetLastError();                   \
    if (_e != hipSuccess) return fail_hip((h), _e, what); \
  } while (0)

template <typename T>
int dev_alloc(lpa_handle *h, T **p, size_t count, bool core = true) {
  void *q = nullptr;
  const size_t bytes = (count ? count : 1) * sizeof(T);
  hipError_t e = hipMalloc(&q, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_err(h, LPA_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  h->allocs.push_back(q);
  if (core)
    h->core_bytes += bytes;
  else
    h->eval_bytes += bytes;
  *p = (T *)q;
  return LPA_OK;
}

bool k_supported(int k) { return k == 1 || k == 2 || k == 4 || k == 8 || k == 16 || k == 32; }

// labels after the iterations run so far
int32_t *cur_labels(const lpa_handle *h) { return h->async_mode ? h->C[0] : h->C[h->iter & 1]; }

int check_ready(lpa_handle *h) {
  if (!h) return LPA_ERR_ARG;
  if (h->poisoned) return LPA_ERR_HIP;
  return LPA_OK;
}

// Longest run of CSR entries one lane scans (measured on R-MAT scale 24).
int default_lane_max(bool async_mode) { return async_mode ? 2048 : 1024; }

// Enqueue iteration state for iteration 0.
int enqueue_reset(lpa_handle *h) {
  const int n = h->n;
  const size_t T = (size_t)(h->max_iter > 0 ? h->max_iter : 1);
  if (n > 0) {
    hipLaunchKernelGGL(k_fill_i32_iota, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream, h->C[0], n);
    if (h->C[1])
      hipLaunchKernelGGL(k_fill_i32_iota, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream, h->C[1],
                         n);
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream, h->act[0],
                       (size_t)n, (uint8_t)1);
    if (h->act[1])
      hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream, h->act[1],
                         (size_t)n, (uint8_t)0);
  }
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(T)), dim3(kAuxBlock), 0, h->stream, h->dN, T);
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(T)), dim3(kAuxBlock), 0, h->stream, h->scanned, T);
  const bool done0 = (n == 0 || h->max_iter == 0);
  hipLaunchKernelGGL(k_set_ctl, dim3(1), dim3(64), 0, h->stream, h->ctl, done0 ? 1 : 0, 0);
  LAUNCH_TRY(h, "reset kernels");
  h->iter = 0;
  h->finished = done0;
  return LPA_OK;
}

// Enqueue iteration l (move, apply, convergence test).
int enqueue_iteration(lpa_handle *h, int l) {
  MoveArgs a;
  a.n = h->n;
  a.row_ptr = h->row_ptr;
  a.col = h->col;
  a.w = h->w;
  if (h->async_mode) {
    a.C = a.Cn = h->C[0];
    a.act_cur = a.act_next = h->act[0];
  } else {
    a.C = h->C[l & 1];
    a.Cn = h->C[(l + 1) & 1];
    a.act_cur = h->act[l & 1];
    a.act_next = h->act[(l + 1) & 1];
  }
  a.order = h->order;
  a.n_hubs = h->n_hubs;
  a.n_lane = h->n_lane;
  a.seg_len = h->lane_max;
  a.n_seg = h->async_mode ? h->n_seg : 0;
  a.seg_hub = h->seg_hub;
  a.hub_pbase = h->hub_pbase;
  a.hub_act = h->hub_act;
  a.part_key = h->part_key;
  a.part_val = h->part_val;
  a.iter = l;
  a.pickless = (h->rho > 0 && l % h->rho == 0) ? 1 : 0;
  a.dN = h->dN;
  a.scanned = h->scanned;
  a.done = h->ctl;
  const bool prof = !h->ev_beg.empty();
  hipEvent_t eb = prof ? h->ev_beg[l] : nullptr, ee = prof ? h->ev_end[l] : nullptr;
  if (h->n_hubs + h->n_lane > 0) {
    hipError_t e = launch_move(h->k, h->async_mode, a, h->grid_move, h->grid_merge, h->stream, eb, ee);
    if (e != hipSuccess) return fail_hip(h, e, "move kernel launch");
  } else if (prof) {
    HIP_TRY(h, hipEventRecord(eb, h->stream));
    HIP_TRY(h, hipEventRecord(ee, h->stream));
  }
  hipLaunchKernelGGL(k_finish, dim3(1), dim3(64), 0, h->stream, (const unsigned long long *)h->dN,
                     l, h->n, h->tol, h->rho, h->max_iter, h->ctl);
  LAUNCH_TRY(h, "iteration kernels");
  return LPA_OK;
}

int read_ctl(lpa_handle *h, int *done, int *iters) {
  int host[2] = {0, 0};
  HIP_TRY(h, hipMemcpyAsync(host, h->ctl, sizeof(host), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  *done = host[0];
  *iters = host[1];
  return LPA_OK;
}

}  // namespace

// ===========================================================================
// Public API
// ===========================================================================
extern "C" {

void lpa_config_default(lpa_config *cfg) {
  if (!cfg) return;
  memset(cfg, 0, sizeof(*cfg));
  cfg->flags = LPA_MODE_DET | LPA_VALIDATE;
  cfg->rho = 8;
}

const char *lpa_error_string(int code) {
  switch (code) {
    case LPA_OK: return "ok";
    case LPA_ERR_ARG: return "invalid argument";
    case LPA_ERR_GRAPH: return "invalid graph, weights or labels";
    case LPA_ERR_UNSUPPORTED: return "unsupported parameter (k or mode)";
    case LPA_ERR_NOMEM: return "device allocation failed";
    case LPA_ERR_HIP: return "HIP runtime error (handle poisoned)";
    case LPA_ERR_STATE: return "handle in the wrong state for this call";
    default: return "unknown status";
  }
}

const char *lpa_last_error(const lpa_handle *h) { return h ? h->err.c_str() : ""; }

int lpa_free(lpa_handle *h) {
  if (!h) return LPA_OK;
  (void)hipStreamSynchronize(h->stream);
  for (hipEvent_t e : h->ev_beg) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->ev_end) (void)hipEventDestroy(e);
  for (void *p : h->allocs) (void)hipFree(p);
  delete h;
  return LPA_OK;
}

int lpa_init(const lpa_graph *g, const float *weights, int k, double tol, int max_iter,
             uint64_t seed, const lpa_config *cfg_in, lpa_handle **out) {
  if (!out) return LPA_ERR_ARG;
  *out = nullptr;
  if (!g) return LPA_ERR_ARG;
  lpa_config cfg;
  if (cfg_in)
    cfg = *cfg_in;
  else
    lpa_config_default(&cfg);
  for (int i = 0; i < 6; ++i)
    if (cfg.reserved[i] != 0) return LPA_ERR_ARG;
  if (cfg.check_every < 0) return LPA_ERR_ARG;
  if (g->n < 0 || g->n == INT32_MAX || g->nnz < 0 || g->nnz >= (int64_t)INT32_MAX) return LPA_ERR_ARG;
  if (g->n > 0 && !g->row_ptr) return LPA_ERR_ARG;
  if (g->nnz > 0 && !g->col_idx) return LPA_ERR_ARG;
  if (g->n == 0 && g->nnz != 0) return LPA_ERR_ARG;
  if (!(tol >= 0.0 && tol <= 1.0) || max_iter < 0 || cfg.rho < 0 || cfg.lane_max_degree < 0)
    return LPA_ERR_ARG;
  const uint32_t mode = cfg.flags & LPA_MODE_MASK;
  if (mode != LPA_MODE_DET && mode != LPA_MODE_ASYNC) return LPA_ERR_UNSUPPORTED;
  if ((cfg.flags & ~(LPA_MODE_MASK | LPA_VALIDATE)) != 0) return LPA_ERR_UNSUPPORTED;
  if (!k_supported(k)) return LPA_ERR_UNSUPPORTED;

  lpa_handle *h = new (std::nothrow) lpa_handle();
  if (!h) return LPA_ERR_NOMEM;
  h->stream = (hipStream_t)cfg.stream;
  h->n = g->n;
  h->nnz = g->nnz;
  h->row_ptr = g->row_ptr;
  h->col = g->col_idx;
  h->w = weights;
  h->k = k;
  h->tol = tol;
  h->max_iter = max_iter;
  h->rho = cfg.rho;
  h->flags = cfg.flags;
  h->async_mode = (mode == LPA_MODE_ASYNC);
  h->seed = seed;
  h->check_every = cfg.check_every;
  h->lane_max = cfg.lane_max_degree > 0 ? cfg.lane_max_degree : default_lane_max(h->async_mode);
  if (h->lane_max > 4096) h->lane_max = 4096;

  int rc = LPA_OK;
  auto bail = [&](int code) {
    std::string msg = h->err;
    lpa_free(h);
    (void)msg;
    return code;
  };
  if (hipGetDevice(&h->device) != hipSuccess) return bail(LPA_ERR_HIP);

  const int n = h->n;
  const size_t T = (size_t)(max_iter > 0 ? max_iter : 1);
  if ((rc = dev_alloc(h, &h->C[0], (size_t)n)) != LPA_OK) return bail(rc);
  if ((rc = dev_alloc(h, &h->act[0], (size_t)n)) != LPA_OK) return bail(rc);
  if (!h->async_mode) {
    if ((rc = dev_alloc(h, &h->C[1], (size_t)n)) != LPA_OK) return bail(rc);
    if ((rc = dev_alloc(h, &h->act[1], (size_t)n)) != LPA_OK) return bail(rc);
  }
  if ((rc = dev_alloc(h, &h->order, (size_t)n)) != LPA_OK) return bail(rc);
  if ((rc = dev_alloc(h, &h->dN, T)) != LPA_OK) return bail(rc);
  if ((rc = dev_alloc(h, &h->scanned, T)) != LPA_OK) return bail(rc);
  if ((rc = dev_alloc(h, &h->ctl, 8)) != LPA_OK) return bail(rc);

  hipLaunchKernelGGL(k_set_ctl, dim3(1), dim3(64), 0, h->stream, h->ctl, 0, 0);
  if (n > 0 && (cfg.flags & LPA_VALIDATE)) {
    hipLaunchKernelGGL(k_validate, dim3(grid_for(h->nnz > n ? (size_t)h->nnz : (size_t)n)),
                       dim3(kAuxBlock), 0, h->stream, n, h->nnz, h->row_ptr, h->col, h->w,
                       h->ctl + 2);
    int bad = 0;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&bad, h->ctl + 2, sizeof(int), hipMemcpyDeviceToHost, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
      return bail(LPA_ERR_HIP);
    if (bad) return bail(LPA_ERR_GRAPH);
  }

  // degree binning (once per graph)
  if (n > 0) {
    const int ncls = kHubClasses + h->lane_max + 1;
    unsigned *hist = nullptr;
    if (hipMalloc(&hist, ncls * sizeof(unsigned)) != hipSuccess) return bail(LPA_ERR_NOMEM);
    bool ok = hipMemsetAsync(hist, 0, ncls * sizeof(unsigned), h->stream) == hipSuccess;
    if (ok) {
      hipLaunchKernelGGL(k_bin_hist, dim3(grid_for(n, kAuxBlock, 2048)), dim3(kAuxBlock),
                         ncls * sizeof(unsigned), h->stream, n, h->row_ptr, h->lane_max, ncls,
                         hist);
      hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(64), 0, h->stream, ncls, hist, h->ctl + 3);
      const int per_block = kAuxBlock * kScatterItems;
      hipLaunchKernelGGL(k_bin_scatter, dim3((n + per_block - 1) / per_block), dim3(kAuxBlock),
                         2 * ncls * sizeof(unsigned), h->stream, n, h->row_ptr, h->lane_max, ncls,
                         hist, h->order);
      ok = hipGetLastError() == hipSuccess;
    }
    int totals[2] = {0, 0};
    if (ok)
      ok = hipMemcpyAsync(totals, h->ctl + 3, sizeof(totals), hipMemcpyDeviceToHost, h->stream) ==
               hipSuccess &&
           hipStreamSynchronize(h->stream) == hipSuccess;
    (void)hipFree(hist);
    if (!ok) return bail(LPA_ERR_HIP);
    h->n_hubs = totals[0];
    h->n_lane = totals[1];
  }

  // async: split every hub into segments of lane_max entries
  if (h->async_mode && h->n_hubs > 0) {
    if ((rc = dev_alloc(h, &h->hub_pbase, (size_t)h->n_hubs + 1)) != LPA_OK) return bail(rc);
    if ((rc = dev_alloc(h, &h->hub_act, (size_t)h->n_hubs)) != LPA_OK) return bail(rc);
    hipLaunchKernelGGL(k_hub_plan, dim3(1), dim3(1024), 0, h->stream, (const int32_t *)h->order,
                       h->n_hubs, h->row_ptr, h->lane_max, h->hub_pbase, h->ctl + 5);
    int nseg = 0;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&nseg, h->ctl + 5, sizeof(int), hipMemcpyDeviceToHost, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
      return bail(LPA_ERR_HIP);
    h->n_seg = nseg;
    if ((rc = dev_alloc(h, &h->seg_hub, (size_t)nseg)) != LPA_OK) return bail(rc);
    if ((rc = dev_alloc(h, &h->part_key, (size_t)nseg * k)) != LPA_OK) return bail(rc);
    if ((rc = dev_alloc(h, &h->part_val, (size_t)nseg * k)) != LPA_OK) return bail(rc);
    hipLaunchKernelGGL(k_fill_seg_hub, dim3(grid_for(h->n_hubs)), dim3(kAuxBlock), 0, h->stream,
                       (const int32_t *)h->hub_pbase, h->n_hubs, h->seg_hub);
    if (hipGetLastError() != hipSuccess) return bail(LPA_ERR_HIP);
  }

  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess)
    return bail(LPA_ERR_HIP);
  const int waves_per_block = kBlock / kWave;
  int grid = cus * move_blocks_per_cu(k, h->async_mode);
  const int units = (h->async_mode ? h->n_seg : 0) + h->n_lane;
  const int items = (h->async_mode ? 0 : h->n_hubs) + (units + kWave - 1) / kWave;
  const int need = (items + waves_per_block - 1) / waves_per_block;
  if (grid > need) grid = need;
  h->grid_move = grid > 0 ? grid : 1;
  const int merge_items = (h->n_hubs + kWave - 1) / kWave;
  int mg = (merge_items + waves_per_block - 1) / waves_per_block;
  if (mg > cus * 4) mg = cus * 4;
  h->grid_merge = mg > 0 ? mg : 1;

  if ((rc = enqueue_reset(h)) != LPA_OK) return bail(rc);
  if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(LPA_ERR_HIP);
  *out = h;
  return LPA_OK;
}

int lpa_reset(lpa_handle *h) {
  int rc = check_ready(h);
  if (rc) return rc;
  return enqueue_reset(h);
}

int lpa_step(lpa_handle *h, int64_t *changed, int *done) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (h->finished) {
    if (changed) *changed = 0;
    if (done) *done = 1;
    return LPA_OK;
  }
  const int l = h->iter;
  if ((rc = enqueue_iteration(h, l)) != LPA_OK) return rc;
  unsigned long long d = 0;
  HIP_TRY(h, hipMemcpyAsync(&d, h->dN + l, sizeof(d), hipMemcpyDeviceToHost, h->stream));
  int dn = 0, it = 0;
  if ((rc = read_ctl(h, &dn, &it)) != LPA_OK) return rc;
  h->iter = l + 1;
  h->finished = dn != 0;
  if (changed) *changed = (int64_t)d;
  if (done) *done = h->finished ? 1 : 0;
  return LPA_OK;
}

int lpa_run(lpa_handle *h, int *iterations) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!h->finished) {
    int dn = 0, it = 0;
    for (int l = h->iter; l < h->max_iter; ++l) {
      if ((rc = enqueue_iteration(h, l)) != LPA_OK) return rc;
      if (h->check_every > 0 && (l + 1 - h->iter) % h->check_every == 0 && l + 1 < h->max_iter) {
        if ((rc = read_ctl(h, &dn, &it)) != LPA_OK) return rc;
        if (dn) break;
      }
    }
    if ((rc = read_ctl(h, &dn, &it)) != LPA_OK) return rc;
    h->iter = it > h->iter ? it : h->iter;
    h->finished = true;
  }
  if (iterations) *iterations = h->iter;
  return LPA_OK;
}

int lpa_get_labels(lpa_handle *h, int32_t *out, int out_is_host) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!out && h->n > 0) return LPA_ERR_ARG;
  if (h->n > 0)
    HIP_TRY(h, hipMemcpyAsync(out, cur_labels(h), (size_t)h->n * sizeof(int32_t),
                              out_is_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                              h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return LPA_OK;
}

int lpa_get_trace(lpa_handle *h, int64_t *changed, int64_t *scanned, int capacity, int *count) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (capacity < 0) return LPA_ERR_ARG;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  const int cnt = h->iter;
  const int m = cnt < capacity ? cnt : capacity;
  if (m > 0) {
    std::vector<unsigned long long> tmp((size_t)m);
    if (changed) {
      HIP_TRY(h, hipMemcpy(tmp.data(), h->dN, m * sizeof(unsigned long long), hipMemcpyDeviceToHost));
      for (int i = 0; i < m; ++i) changed[i] = (int64_t)tmp[i];
    }
    if (scanned) {
      HIP_TRY(h, hipMemcpy(tmp.data(), h->scanned, m * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost));
      for (int i = 0; i < m; ++i) scanned[i] = (int64_t)tmp[i];
    }
  }
  if (count) *count = cnt;
  return LPA_OK;
}

int lpa_modularity(lpa_handle *h, const int32_t *labels, double *q) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!q) return LPA_ERR_ARG;
  const int n = h->n;
  if (n == 0) {
    *q = 0.0;
    return LPA_OK;
  }
  if (!h->mod_tot) {
    if ((rc = dev_alloc(h, &h->mod_tot, (size_t)n, false)) != LPA_OK) return rc;
    if ((rc = dev_alloc(h, &h->mod_acc, 4, false)) != LPA_OK) return rc;
    hipLaunchKernelGGL(k_zero_d, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream, h->mod_tot, n);
  }
  const int32_t *lab = labels ? labels : cur_labels(h);
  hipLaunchKernelGGL(k_zero_d, dim3(1), dim3(64), 0, h->stream, h->mod_acc, 4);
  hipLaunchKernelGGL(k_clear_err, dim3(1), dim3(64), 0, h->stream, h->ctl);
  if (h->n_hubs > 0)
    hipLaunchKernelGGL(k_mod_hub, dim3(grid_for((size_t)h->n_hubs * 64, kAuxBlock, 2048)),
                       dim3(kAuxBlock), 0, h->stream, (const int32_t *)h->order, h->n_hubs,
                       h->row_ptr, h->col, h->w, lab, n, h->mod_tot, h->mod_acc, h->ctl + 2);
  if (h->n_lane > 0)
    hipLaunchKernelGGL(k_mod_lane, dim3(grid_for(h->n_lane, kAuxBlock, 4096)), dim3(kAuxBlock), 0,
                       h->stream, (const int32_t *)h->order, h->n_hubs, h->n_lane, h->row_ptr,
                       h->col, h->w, lab, n, h->mod_tot, h->mod_acc, h->ctl + 2);
  hipLaunchKernelGGL(k_mod_sq, dim3(grid_for(n, kAuxBlock, 4096)), dim3(kAuxBlock), 0, h->stream,
                     h->mod_tot, n, h->mod_acc);
  LAUNCH_TRY(h, "modularity kernels");
  double acc[4] = {0, 0, 0, 0};
  int bad = 0;
  HIP_TRY(h, hipMemcpyAsync(acc, h->mod_acc, sizeof(acc), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipMemcpyAsync(&bad, h->ctl + 2, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  if (bad) {
    // labels of vertices with degree 0 are not visited above; out of range
    // labels among the others were skipped, so tot may hold stale sums
    hipLaunchKernelGGL(k_zero_d, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream, h->mod_tot, n);
    hipLaunchKernelGGL(k_clear_err, dim3(1), dim3(64), 0, h->stream, h->ctl);
    LAUNCH_TRY(h, "modularity reset");
    return set_err(h, LPA_ERR_GRAPH, "label out of range [0, n)");
  }
  const double two_m = acc[0];
  *q = two_m > 0.0 ? acc[1] / two_m - acc[2] / (two_m * two_m) : 0.0;
  return LPA_OK;
}

int lpa_get_state(lpa_handle *h, int32_t *labels, uint8_t *unprocessed, int *iteration,
                  int is_host) {
  int rc = check_ready(h);
  if (rc) return rc;
  const int n = h->n;
  const hipMemcpyKind kind = is_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice;
  if (n > 0 && labels)
    HIP_TRY(h, hipMemcpyAsync(labels, cur_labels(h), (size_t)n * sizeof(int32_t), kind, h->stream));
  if (n > 0 && unprocessed) {
    const uint8_t *src = h->async_mode ? h->act[0] : h->act[h->iter & 1];
    HIP_TRY(h, hipMemcpyAsync(unprocessed, src, (size_t)n, kind, h->stream));
  }
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  if (iteration) *iteration = h->iter;
  return LPA_OK;
}

int lpa_set_state(lpa_handle *h, const int32_t *labels, const uint8_t *unprocessed, int iteration,
                  int is_host) {
  int rc = check_ready(h);
  if (rc) return rc;
  const int n = h->n;
  if (iteration < 0 || iteration > h->max_iter) return LPA_ERR_ARG;
  if (n > 0 && (!labels || !unprocessed)) return LPA_ERR_ARG;
  if (n > 0) {
    if (is_host) {
      for (int i = 0; i < n; ++i)
        if (labels[i] < 0 || labels[i] >= n)
          return set_err(h, LPA_ERR_GRAPH, "label out of range [0, n)");
    } else {
      hipLaunchKernelGGL(k_clear_err, dim3(1), dim3(64), 0, h->stream, h->ctl);
      hipLaunchKernelGGL(k_check_labels, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream, labels,
                         n, h->ctl + 2);
      LAUNCH_TRY(h, "label check");
      int bad = 0;
      HIP_TRY(h, hipMemcpyAsync(&bad, h->ctl + 2, sizeof(int), hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(h, hipStreamSynchronize(h->stream));
      if (bad) return set_err(h, LPA_ERR_GRAPH, "label out of range [0, n)");
    }
  }
  // counters of every iteration start from zero again
  if ((rc = enqueue_reset(h)) != LPA_OK) return rc;
  if (n > 0) {
    const hipMemcpyKind kind = is_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
    uint8_t *cur = h->async_mode ? h->act[0] : h->act[iteration & 1];
    HIP_TRY(h, hipMemcpyAsync(h->C[0], labels, (size_t)n * sizeof(int32_t), kind, h->stream));
    if (h->C[1])  // both buffers: vertices of degree 0 are never rewritten
      HIP_TRY(h, hipMemcpyAsync(h->C[1], labels, (size_t)n * sizeof(int32_t), kind, h->stream));
    HIP_TRY(h, hipMemcpyAsync(cur, unprocessed, (size_t)n, kind, h->stream));
    hipLaunchKernelGGL(k_normalize_u8, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream, cur, n);
    if (!h->async_mode)
      hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream,
                         h->act[(iteration + 1) & 1], (size_t)n, (uint8_t)0);
    LAUNCH_TRY(h, "state restore");
  }
  const bool fin = (n == 0 || iteration >= h->max_iter);
  hipLaunchKernelGGL(k_set_ctl, dim3(1), dim3(64), 0, h->stream, h->ctl, fin ? 1 : 0, iteration);
  LAUNCH_TRY(h, "state restore");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->iter = iteration;
  h->finished = fin;
  return LPA_OK;
}

int lpa_profile(lpa_handle *h, int enable) {
  int rc = check_ready(h);
  if (rc) return rc;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  for (hipEvent_t e : h->ev_beg) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->ev_end) (void)hipEventDestroy(e);
  h->ev_beg.clear();
  h->ev_end.clear();
  if (enable) {
    const int T = h->max_iter > 0 ? h->max_iter : 1;
    h->ev_beg.resize(T);
    h->ev_end.resize(T);
    for (int i = 0; i < T; ++i) {
      HIP_TRY(h, hipEventCreate(&h->ev_beg[i]));
      HIP_TRY(h, hipEventCreate(&h->ev_end[i]));
    }
  }
  return LPA_OK;
}

int lpa_get_profile(lpa_handle *h, float *move_ms, int capacity, int *count) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (h->ev_beg.empty()) return set_err(h, LPA_ERR_STATE, "profiling is off");
  if (capacity < 0) return LPA_ERR_ARG;
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  const int cnt = h->iter;
  for (int i = 0; i < cnt && i < capacity && move_ms; ++i)
    HIP_TRY(h, hipEventElapsedTime(&move_ms[i], h->ev_beg[i], h->ev_end[i]));
  if (count) *count = cnt;
  return LPA_OK;
}

int lpa_memory_floor(lpa_handle *h, int reps, float *ms) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!ms || reps < 1) return LPA_ERR_ARG;
  *ms = 0.0f;
  if (h->nnz == 0) return LPA_OK;
  hipEvent_t b = nullptr, e = nullptr;
  HIP_TRY(h, hipEventCreate(&b));
  HIP_TRY(h, hipEventCreate(&e));
  float best = -1.0f;
  for (int r = 0; r < reps + 1; ++r) {  // the first launch warms the caches
    HIP_TRY(h, hipEventRecord(b, h->stream));
    hipLaunchKernelGGL(k_scan_floor, dim3(4096), dim3(kAuxBlock), 0, h->stream, h->col, h->w,
                       (const int32_t *)cur_labels(h), h->nnz, (unsigned long long *)(h->ctl + 6));
    HIP_TRY(h, hipGetLastError());
    HIP_TRY(h, hipEventRecord(e, h->stream));
    HIP_TRY(h, hipEventSynchronize(e));
    float t = 0.0f;
    HIP_TRY(h, hipEventElapsedTime(&t, b, e));
    if (r > 0 && (best < 0.0f || t < best)) best = t;
  }
  (void)hipEventDestroy(b);
  (void)hipEventDestroy(e);
  *ms = best;
  return LPA_OK;
}

int lpa_memory(const lpa_handle *h, size_t *core_bytes, size_t *eval_bytes) {
  if (!h) return LPA_ERR_ARG;
  if (core_bytes) *core_bytes = h->core_bytes;
  if (eval_bytes) *eval_bytes = h->eval_bytes;
  return LPA_OK;
}

}  // extern "C"
