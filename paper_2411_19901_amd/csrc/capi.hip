// C-ABI runtime of liblpa.so: handle, device state, auxiliary kernels and
// the iteration driver (paper Algorithm 1, lpa).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <array>
#include <string>
#include <vector>

#include "lpa_internal.h"

using namespace lpa;

// ===========================================================================
// Auxiliary kernels
// ===========================================================================
namespace {

constexpr int kAuxBlock = 256;
constexpr int kPrefixArrays = 4;  // per-graph prefix sums kept for a batched launch

__global__ void k_fill_i32_iota(int32_t *C, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) C[i] = i;
}

// Ranked layout: labels start as the ids of the vertices at each position.
__global__ void k_copy_i32(const int32_t *src, int32_t *dst, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// pos[order[p]] = p: the degree-order position of every vertex.
__global__ void k_positions(const int32_t *order, int n, int32_t *pos) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x)
    pos[order[p]] = p;
}

// Column indices rewritten as positions: colr[e] = pos[col[e]].
__global__ void k_remap_cols(const int32_t *col, int64_t nnz, const int32_t *pos, int32_t *colr) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nnz;
       e += (int64_t)gridDim.x * blockDim.x)
    colr[e] = pos[col[e]];
}

// Vertex-indexed data to and from a ranked state array:
// out[order[p]] = st[p] and st[p] = in[order[p]].
template <class T>
__global__ void k_unrank(const int32_t *order, const T *st, int n, T *out) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x)
    out[order[p]] = st[p];
}
template <class T>
__global__ void k_rank(const int32_t *order, const T *in, int n, T *st) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x)
    st[p] = in[order[p]];
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
__global__ void k_validate(int n, int64_t nnz, RowPtr rp, const int32_t *col, const float *w,
                           int *bad) {
  const size_t tid = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  int b = 0;
  if (tid == 0 && (rp[0] != 0 || rp[n] != nnz)) b |= 1;
  for (size_t i = tid; i < (size_t)n; i += stride) {
    const long long d = rp[i + 1] - rp[i];
    if (d < 0 || d > (long long)INT32_MAX) b |= 1;
  }
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
// Stable degree binning (once per graph, or once per id range of a streamed
// graph): vertices v0 .. v0 + n - 1 ordered by degree class (decreasing
// degree), increasing id within a class; isolated vertices come last.
// Block b owns the ids v0 + [b * kBinIds, (b + 1) * kBinIds).
//   1. k_bin_count: counts[c * nblk + b] = vertices of class c in block b;
//   2. k_scan_*: exclusive prefix sum over counts in (class, block) order,
//      which is each block's first position for each class;
//   3. k_bin_place: every block walks its ids in order and writes each
//      vertex at its class's next position.
// Largest graph: 2^62 CSR entries; async hub segments (work items of one
// iteration) below 2^30 so that per-launch sums stay within int32.
constexpr int64_t kMaxEntries = (int64_t)1 << 62;
constexpr int64_t kMaxSegs = (int64_t)1 << 30;
constexpr int kBinIds = 4096;
constexpr int kScanChunk = 4096;  // entries per block of the prefix sum

__global__ void k_bin_count(int v0, int n, RowPtr rp, int lane_max, int nblk, unsigned *counts) {
  __shared__ unsigned cnt[kBinClasses];
  for (int c = threadIdx.x; c < kBinClasses; c += blockDim.x) cnt[c] = 0;
  __syncthreads();
  const int b0 = blockIdx.x * kBinIds;
  for (int u = b0 + threadIdx.x; u < b0 + kBinIds && u < n; u += blockDim.x) {
    const int v = v0 + u;
    const int d = (int)(rp[v + 1] - rp[v]);
    atomicAdd(&cnt[degree_class(d, lane_max)], 1u);
  }
  __syncthreads();
  for (int c = threadIdx.x; c < kBinClasses; c += blockDim.x)
    counts[(size_t)c * nblk + blockIdx.x] = cnt[c];
}

// In-place exclusive scan of each kScanChunk-entry chunk; chunk totals to
// sums[chunk].  256 threads, 16 consecutive entries per thread.
__global__ void k_scan_chunks(unsigned *x, size_t count, unsigned *sums) {
  __shared__ unsigned part[256];
  const size_t base = (size_t)blockIdx.x * kScanChunk + (size_t)threadIdx.x * 16;
  unsigned loc[16];
  unsigned t = 0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    loc[i] = base + i < count ? x[base + i] : 0u;
    t += loc[i];
  }
  part[threadIdx.x] = t;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive scan of the 256 thread totals
    const unsigned y = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += y;
    __syncthreads();
  }
  unsigned run = part[threadIdx.x] - t;  // exclusive
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    if (base + i < count) x[base + i] = run;
    run += loc[i];
  }
  if (threadIdx.x == 255) sums[blockIdx.x] = part[255];
}

// Exclusive scan of the chunk totals (one block, sequential in the first
// thread: there are at most a few hundred thousand chunks and it runs once
// per graph); writes the number of hubs and of lane vertices.
__global__ void k_scan_sums(unsigned *sums, int nchunks, const unsigned *x, int nblk,
                            int *totals) {
  if (threadIdx.x != 0) return;
  unsigned acc = 0;
  for (int c = 0; c < nchunks; ++c) {
    const unsigned y = sums[c];
    sums[c] = acc;
    acc += y;
  }
  // first position of class kHubClasses (block 0) = number of hubs; first
  // position of the isolated class = hubs + lane vertices; from the first
  // position of kShortClass on, the lane vertices are short
  const size_t i = (size_t)kHubClasses * nblk;
  const unsigned hubs = x[i] + sums[i / kScanChunk];
  const size_t j = (size_t)kClasses * nblk;
  const unsigned placed = x[j] + sums[j / kScanChunk];
  const size_t q = (size_t)kShortClass * nblk;
  const unsigned short_first = x[q] + sums[q / kScanChunk];
  totals[0] = (int)hubs;
  totals[1] = (int)(placed - hubs);
  totals[3] = (int)(placed - (short_first > hubs ? short_first : hubs));
}

__global__ void k_scan_add(unsigned *x, size_t count, const unsigned *sums) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) x[i] += sums[i / kScanChunk];
}

// Place every vertex of block b at its class's next position, in id order.
// 256 threads walk the block's ids 256 at a time; the four wavefronts take
// turns so that lower ids are placed first.
__global__ __launch_bounds__(256) void k_bin_place(int v0, int n, RowPtr rp, int lane_max, int nblk,
                                                   const unsigned *offsets, int32_t *order) {
  __shared__ unsigned next[kBinClasses];
  for (int c = threadIdx.x; c < kBinClasses; c += blockDim.x) next[c] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const unsigned long long below = (1ull << lane) - 1ull;
  const int b0 = blockIdx.x * kBinIds;
  for (int r = 0; r < kBinIds; r += 256) {
    const int u = b0 + r + (int)threadIdx.x;
    const int v = v0 + u;
    int cls = -1;
    if (u < n) cls = degree_class((int)(rp[v + 1] - rp[v]), lane_max);
    for (int w = 0; w < 4; ++w) {
      if (wid == w) {
        unsigned long long rest = __ballot(cls >= 0);
        while (rest) {
          const int src = __ffsll((long long)rest) - 1;
          const int c = __shfl(cls, src);
          const unsigned long long m = __ballot(cls == c);
          rest &= ~m;
          const unsigned start = next[c];
          if (cls == c) {
            const unsigned rank = (unsigned)__popcll(m & below);
            order[offsets[(size_t)c * nblk + blockIdx.x] + start + rank] = v;
          }
          if (lane == src) next[c] = start + (unsigned)__popcll(m);
          __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
          __builtin_amdgcn_wave_barrier();
        }
      }
      __syncthreads();
    }
  }
}

// --- iteration epilogue ------------------------------------------------------
// Async hub segments: pbase[h] = sum over earlier hubs of ceil(deg / S);
// pbase[n_hubs] (also written to *total) = number of segments.  One block.
__global__ void k_hub_plan(const int32_t *order, int n_hubs, RowPtr rp, int S,
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
    // a total beyond int32 (possible only for an unvalidated invalid
    // graph) is reported as INT32_MAX, which exceeds every segment bound
    pbase[n_hubs] = (int32_t)(acc < INT32_MAX ? acc : INT32_MAX);
    *total = (int)(acc < INT32_MAX ? acc : INT32_MAX);
  }
  __syncthreads();
  long long acc = part[t];
  for (int h = h0; h < h1; ++h) {
    pbase[h] = (int32_t)(acc < INT32_MAX ? acc : INT32_MAX);
    const int v = order[h];
    acc += (rp[v + 1] - rp[v] + S - 1) / S;
  }
}

__global__ void k_fill_seg_hub(const int32_t *pbase, int n_hubs, int32_t *seg_hub) {
  for (int h = blockIdx.x * blockDim.x + threadIdx.x; h < n_hubs; h += gridDim.x * blockDim.x)
    for (int q = pbase[h]; q < pbase[h + 1]; ++q) seg_hub[q] = h;
}

__global__ void k_status_set(GraphStatus *st, int iter, int done, int fresh) {
  if (threadIdx.x == 0) {
    st->iter = iter;
    st->done = done;
    st->err = 0;
    st->fresh = fresh;
  }
}

// *bad = 1 if some hub row (order[0, n_hubs)) does not strictly increase:
// one wavefront per hub compares every entry with the next.
__global__ void k_check_hub_rows(const int32_t *order, int n_hubs, RowPtr rp, const int32_t *col,
                                 int *bad) {
  const int lane = threadIdx.x & 63;
  const int wave = (blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const int nwaves = gridDim.x * blockDim.x / 64;
  int b = 0;
  for (int h = wave; h < n_hubs; h += nwaves) {
    const int v = order[h];
    const int64_t rb = rp[v], re = rp[v + 1];
    for (int64_t e = rb + lane; e + 1 < re; e += 64) b |= col[e] >= col[e + 1] ? 1 : 0;
  }
  if (__ballot(b != 0) != 0ull && lane == 0) atomicOr(bad, 1);
}

// lpa_reset of every graph of a table: blockIdx.y (strided) picks the graph,
// the x blocks stride over its vertices; block x = 0 also clears the
// per-iteration counters and the status.
__global__ void k_batch_reset(const GraphDesc *d, int G) {
  for (int g = blockIdx.y; g < G; g += gridDim.y) {
    const GraphDesc &gd = d[g];
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < gd.n; i += gridDim.x * blockDim.x) {
      const int c = gd.ranked ? gd.order[i] : i;  // the id of the vertex whose label this is
      gd.C[0][i] = c;
      if (gd.C[1] != gd.C[0]) gd.C[1][i] = c;
      gd.act[0][i] = 1;
      if (gd.act[1] != gd.act[0]) gd.act[1][i] = 0;
    }
    if (blockIdx.x == 0) {
      const int T = gd.max_iter > 0 ? gd.max_iter : 1;
      for (int t = threadIdx.x; t < T; t += blockDim.x) {
        gd.dN[t] = 0;
        gd.scanned[t] = 0;
      }
      if (threadIdx.x == 0) {
        gd.st->iter = 0;
        gd.st->done = (gd.n == 0 || gd.max_iter == 0) ? 1 : 0;
        gd.st->err = 0;
        gd.st->fresh = 1;
      }
    }
  }
}

__global__ void k_status_clear_err(GraphStatus *st) {
  if (threadIdx.x == 0) st->err = 0;
}

__global__ void k_zero_i32(int32_t *p, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    p[i] = 0;
}

// --- modularity (Eq. 1, community-sum form), fp64 --------------------------
__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// Sum of squares of the community totals (then cleared for the next call).
// One atomic per workgroup: atomics on the one accumulator serialise, so
// the workgroup sums its wavefronts' parts first (and the launch is capped
// at kModSqBlocks workgroups).
constexpr int kModSqBlocks = 1024;
__global__ __launch_bounds__(kAuxBlock) void k_mod_sq(double *tot, int n, double *acc) {
  __shared__ double part[kAuxBlock / 64];
  double s = 0.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    const double x = tot[c];
    s += x * x;
    tot[c] = 0.0;
  }
  s = wave_sum_d(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kAuxBlock / 64; ++w) t += part[w];
    atomicAdd(&acc[2], t);
  }
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
// Handles and batches
// ===========================================================================
struct lpa_batch {
  int capacity = 0;
  int k = 8;  // kernel selector: sketch slots, 0 = the vote of Algorithm 3
  bool rescan = false;      // double scan (LPA_RESCAN)
  bool hub_shared = false;  // one shared sketch per hub (LPA_HUB_SHARED)
  bool shared_vars = false;  // LDS shared variables in the det hub path (LPA_SHARED_VARS)
  bool capture = false;     // replay iterations from a captured hipGraph (LPA_CAPTURE)
  hipStream_t cap_stream = nullptr;  // private stream the iterations are captured on
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  long long graph_key[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  bool async_mode = false;
  hipStream_t stream = nullptr;
  int device = 0;
  int check_every = 0;
  int cus = 1;
  int grid_cap[2] = {1, 1};  // resident k_move workgroups: int32 / int64 positions
  int blocks_cap = 0;        // lpa_config.move_blocks_per_cu (0: as many as fit)
  bool wide = false;         // a loaded graph has int64 row offsets
  void *dblock = nullptr;  // device: descriptors, prefixes, finished counter, status
  GraphDesc *d_desc = nullptr;
  int32_t *d_prefix = nullptr;  // items, hubs, merge items, hub segments: [cap+1] each
  int32_t *d_finished = nullptr;
  int32_t *d_status = nullptr;  // [3 * cap]: iter, done, dN of the last launched iteration
  void *hblock = nullptr;  // pinned host mirror of the same layout
  GraphDesc *h_desc = nullptr;
  int32_t *h_prefix = nullptr;
  int32_t *h_finished = nullptr;
  int32_t *h_status = nullptr;
  size_t block_bytes = 0;
  size_t off_prefix = 0, off_finished = 0, off_status = 0;
  std::vector<lpa_handle *> loaded;
  int total_items = 0, total_hubs = 0, total_merge = 0, total_segs = 0, unfinished = 0;
  bool poisoned = false;
  std::string err;
};

struct lpa_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  int32_t n = 0;
  int64_t nnz = 0;
  RowPtr row_ptr{nullptr, nullptr};
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

  void *block = nullptr;  // every device array of the handle
  bool owns_block = false;
  void *part_block = nullptr;  // async partial sketches, sized once the segments are planned
  GraphDesc desc{};       // host copy of the static descriptor
  GraphStatus *st = nullptr;
  uint32_t *hist = nullptr;  // binning scratch
  int32_t seg_cap = 0, hub_cap = 0;
  int32_t n_segs = 0;  // hub segments planned (det mode too, for modularity)
  double *mod_tot = nullptr;
  int mod_grid = 0;  // k_modularity workgroups (resident on every CU)
  double *mod_acc = nullptr;
  std::vector<void *> eval_allocs;
  // LPA_RANKED_LAYOUT: neighbour positions (desc.col points here) and a
  // transfer buffer for host copies of ranked state
  int32_t *colr = nullptr;
  void *tmp = nullptr;

  int iter = 0;  // iterations run (host mirror of st->iter)
  bool finished = false;
  size_t core_bytes = 0, eval_bytes = 0;
  bool poisoned = false;
  std::string err;
  std::vector<hipEvent_t> ev_beg, ev_end;
  std::vector<uint8_t> ev_rec;  // 1: the events of iteration i were recorded in this run
  lpa_batch *self = nullptr;  // batch of one used by lpa_step / lpa_run

  // LPA_STREAM_CSR: the graph stays in pinned host memory; every iteration
  // copies the rows of one id range after another into kBufs device
  // buffers in turn; range p runs on compute stream p % kBufs (stream 0 is
  // the handle's), so the move kernels of up to kBufs ranges overlap
  struct Streamed {
    static constexpr int kBufs = 4;
    bool on = false;
    hipStream_t copy = nullptr;        // DMA stream (default priority)
    hipStream_t cs[kBufs] = {};        // compute streams; cs[0] = the handle's
    hipEvent_t copied[kBufs] = {}, done[kBufs] = {};
    hipEvent_t start = nullptr;        // the previous iteration's stop test is done
    const int32_t *host_col = nullptr;
    const float *host_w = nullptr;
    void *dev = nullptr;  // row offsets, second order, descriptors, prefixes, buffers
    size_t dev_bytes = 0;
    int32_t *col_buf[kBufs] = {};
    float *w_buf[kBufs] = {};
    std::vector<int32_t> first;          // [ranges + 1] first vertex of each range
    std::vector<int64_t> base, entries;  // per range: first CSR entry, entries
    int32_t *order = nullptr;            // device [n]: vertices of each range by degree
    std::vector<int32_t> items;          // per range: move work items
    GraphDesc *desc = nullptr;           // device [ranges]
    int32_t *prefix = nullptr;  // device [ranges][8]: {0, items, 0, hubs, 0, merge items, 0, segments}
    // LPA_MODE_ASYNC: each range's hub segments (bounds from its entries)
    std::vector<int32_t> hub_cap, seg_cap, hubs, segs;
    std::vector<std::array<size_t, 6>> o_hub;  // offsets in dev: pbase, flags, segment hubs,
                                               // partial keys, partial values, candidates
    int grid_cap = 1, cus = 1;
  } sm;
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

int fail_hip_b(lpa_batch *b, hipError_t e, const char *what) {
  if (b) {
    b->poisoned = true;
    b->err = std::string(what) + ": " + hipGetErrorString(e);
  }
  return LPA_ERR_HIP;
}

#define HIP_TRY(h, expr)                                   \
  do {                                                     \
    hipError_t _e = (expr);                                \
    if (_e != hipSuccess) return fail_hip((h), _e, #expr); \
  } while (0)

#define LAUNCH_TRY(h, what)                                \
  do {                                                     \
    hipError_t _e = hipGetLastError();                     \
    if (_e != hipSuccess) return fail_hip((h), _e, what);  \
  } while (0)

#define HIP_TRY_B(b, expr)                                   \
  do {                                                       \
    hipError_t _e = (expr);                                  \
    if (_e != hipSuccess) return fail_hip_b((b), _e, #expr); \
  } while (0)

bool k_supported(int k) { return k == 1 || k == 2 || k == 4 || k == 8 || k == 16 || k == 32; }

// Where an array handed to the library lives, as the kernels will see it:
// device (or managed) memory of the current device, pinned host memory
// mapped into the device's address space (read over the host link at the
// same virtual address), or neither.  Classified before any kernel touches
// the array.
int pointer_location(const void *p) {
  if (!p) return LPA_PTR_UNUSABLE;
  hipPointerAttribute_t at;
  memset(&at, 0, sizeof(at));
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return LPA_PTR_UNUSABLE;
  }
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    return LPA_PTR_UNUSABLE;
  }
  switch (at.type) {
    case hipMemoryTypeDevice:
    case hipMemoryTypeUnified:
      return at.device == dev ? LPA_PTR_DEVICE : LPA_PTR_UNUSABLE;
    case hipMemoryTypeManaged:
      return LPA_PTR_DEVICE;
    case hipMemoryTypeHost:
      return (at.devicePointer == p) ? LPA_PTR_HOST : LPA_PTR_UNUSABLE;
    default:
      return LPA_PTR_UNUSABLE;
  }
}

// Check k against the rule flags: LPA_ERR_UNSUPPORTED for a k without
// kernels, LPA_ERR_ARG for the one-candidate vote with k != 1.
int check_k(int k, uint32_t flags) {
  if (!k_supported(k)) return LPA_ERR_UNSUPPORTED;
  if ((flags & LPA_RULE_BM_PAPER) && k != 1) return LPA_ERR_ARG;
  if ((flags & LPA_RULE_BM_PAPER) && (flags & LPA_RESCAN)) return LPA_ERR_ARG;
  if ((flags & LPA_HUB_SHARED) &&
      ((flags & LPA_MODE_MASK) != LPA_MODE_ASYNC || (flags & (LPA_RULE_BM_PAPER | LPA_RESCAN))))
    return LPA_ERR_ARG;
  if ((flags & LPA_SHARED_VARS) &&
      ((flags & LPA_MODE_MASK) != LPA_MODE_DET || (flags & (LPA_RULE_BM_PAPER | LPA_RESCAN))))
    return LPA_ERR_ARG;
  if ((flags & LPA_STREAM_CSR) && (flags & (LPA_HUB_SHARED | LPA_RANKED_LAYOUT)))
    return LPA_ERR_ARG;
  return LPA_OK;
}

// Kernel selector: k slots, or 0 for the vote of Algorithm 3.
int kernel_k(int k, uint32_t flags) { return (flags & LPA_RULE_BM_PAPER) ? 0 : k; }

int check_ready(lpa_handle *h) {
  if (!h) return LPA_ERR_ARG;
  if (h->poisoned) return LPA_ERR_HIP;
  return LPA_OK;
}

// Longest run of CSR entries one lane scans (measured on R-MAT scale 24).
// Lane threshold S when the caller leaves it 0: the autotuner's choice on
// R-MAT scale 22-24 (async 1024, det 4096); tune.py picks per graph.
int default_lane_max(bool async_mode) { return async_mode ? 1024 : 4096; }

// labels after the iterations run so far
int32_t *cur_labels(const lpa_handle *h) { return h->desc.C[h->iter & 1]; }
uint8_t *cur_flags(const lpa_handle *h) { return h->desc.act[h->iter & 1]; }

// --- one device block per handle -------------------------------------------
struct Layout {
  size_t st, dN, scanned, C0, C1, act0, act1, order, hist, hub_pbase, hub_act, seg_hub, pkey,
      pval, hcand, colr, tmp, total;
  int32_t hub_cap, seg_cap, ncls;
  bool too_many_segs;
};

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// bound_partials: reserve the partial sketches for the largest possible
// number of hub segments (a caller workspace); otherwise lpa_init sizes them
// once the segments are planned.
Layout plan_layout(int32_t n, int64_t nnz, int k, int max_iter, bool async_mode, int lane_max,
                   bool rescan, bool bound_partials, bool ranked) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + (bytes ? bytes : 1));
    return at;
  };
  const size_t T = (size_t)(max_iter > 0 ? max_iter : 1);
  L.ncls = kBinClasses;
  const size_t nblk = ((size_t)n + kBinIds - 1) / kBinIds;
  const size_t cells = (size_t)kBinClasses * (nblk ? nblk : 1);
  const size_t chunks = (cells + kScanChunk - 1) / kScanChunk;
  L.st = take(sizeof(GraphStatus));
  L.dN = take(T * 8);
  L.scanned = take(T * 8);
  // the binning's count matrix uses C0 before the labels are initialised
  L.C0 = take(std::max((size_t)n * 4, cells * 4));
  L.C1 = async_mode ? L.C0 : take((size_t)n * 4);
  L.act0 = take((size_t)n);
  L.act1 = async_mode ? L.act0 : take((size_t)n);
  L.order = take((size_t)n * 4);
  L.hist = take(chunks * 4);
  if (ranked) {  // LPA_RANKED_LAYOUT: column indices as positions, a transfer buffer
    L.colr = take((size_t)nnz * 4);
    L.tmp = take((size_t)n * 4);
  }
  // hubs have more than S entries each; a hub of degree d > S has
  // ceil(d / S) < 2 d / S segments.  Async mode scans the segments as work
  // items; both modes spread modularity's reads of a hub over them.
  const int64_t hubs = nnz / (lane_max + 1) + 1;
  const int64_t segs = 2 * (nnz / lane_max) + 2;
  if (segs >= kMaxSegs) {  // work items of one iteration must fit int32
    if (async_mode) {
      L.too_many_segs = true;
      return L;
    }
  } else {
    L.hub_cap = (int32_t)(hubs < n ? hubs : n);
    L.seg_cap = (int32_t)segs;
    L.hub_pbase = take(((size_t)L.hub_cap + 1) * 4);
    L.seg_hub = take((size_t)L.seg_cap * 4);
  }
  if (async_mode) {
    L.hub_act = take((size_t)L.hub_cap);
    L.pkey = take(bound_partials ? (size_t)L.seg_cap * k * 4 : 0);
    L.pval = take(bound_partials ? (size_t)L.seg_cap * k * 4 : 0);
    L.hcand = take(rescan ? (size_t)L.hub_cap * k * 4 : 0);  // double-scan candidates
  }
  L.total = off;
  return L;
}

// Enqueue iteration-0 state.
int enqueue_reset(lpa_handle *h) {
  const int n = h->n;
  const size_t T = (size_t)(h->max_iter > 0 ? h->max_iter : 1);
  if (n > 0) {
    for (int b = 0; b < 2; ++b) {
      if (b == 1 && h->desc.C[1] == h->desc.C[0]) break;
      if (h->desc.ranked)  // label at position p: the id of the vertex there
        hipLaunchKernelGGL(k_copy_i32, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream,
                           h->desc.order, h->desc.C[b], n);
      else
        hipLaunchKernelGGL(k_fill_i32_iota, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream,
                           h->desc.C[b], n);
    }
    hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream, h->desc.act[0],
                       (size_t)n, (uint8_t)1);
    if (h->desc.act[1] != h->desc.act[0])
      hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream,
                         h->desc.act[1], (size_t)n, (uint8_t)0);
  }
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(T)), dim3(kAuxBlock), 0, h->stream, h->desc.dN, T);
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(T)), dim3(kAuxBlock), 0, h->stream,
                     h->desc.scanned, T);
  const bool done0 = (n == 0 || h->max_iter == 0);
  hipLaunchKernelGGL(k_status_set, dim3(1), dim3(64), 0, h->stream, h->st, 0, done0 ? 1 : 0, 1);
  LAUNCH_TRY(h, "reset kernels");
  h->iter = 0;
  h->finished = done0;
  std::fill(h->ev_rec.begin(), h->ev_rec.end(), (uint8_t)0);
  return LPA_OK;
}

// Copy the n-item state array `st` (labels: elem 4, flags: elem 1) to the
// caller's vertex-indexed `out` (host or device), and back (state_in),
// reordering through the degree order when the handle's state is ranked
// (host data then passes through the transfer buffer).  Enqueued on the
// handle's stream.
int state_out(lpa_handle *h, const void *st, void *out, size_t elem, bool out_is_host) {
  const int n = h->n;
  if (!h->desc.ranked) {
    HIP_TRY(h, hipMemcpyAsync(out, st, (size_t)n * elem,
                              out_is_host ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                              h->stream));
    return LPA_OK;
  }
  void *dst = out_is_host ? h->tmp : out;
  if (elem == 4)
    hipLaunchKernelGGL(k_unrank<int32_t>, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream,
                       h->desc.order, (const int32_t *)st, n, (int32_t *)dst);
  else
    hipLaunchKernelGGL(k_unrank<uint8_t>, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream,
                       h->desc.order, (const uint8_t *)st, n, (uint8_t *)dst);
  LAUNCH_TRY(h, "state reorder");
  if (out_is_host)
    HIP_TRY(h, hipMemcpyAsync(out, h->tmp, (size_t)n * elem, hipMemcpyDeviceToHost, h->stream));
  return LPA_OK;
}

int state_in(lpa_handle *h, const void *in, void *st, size_t elem, bool in_is_host) {
  const int n = h->n;
  if (!h->desc.ranked) {
    HIP_TRY(h, hipMemcpyAsync(st, in, (size_t)n * elem,
                              in_is_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice,
                              h->stream));
    return LPA_OK;
  }
  const void *src = in;
  if (in_is_host) {
    HIP_TRY(h, hipMemcpyAsync(h->tmp, in, (size_t)n * elem, hipMemcpyHostToDevice, h->stream));
    src = h->tmp;
  }
  if (elem == 4)
    hipLaunchKernelGGL(k_rank<int32_t>, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream,
                       h->desc.order, (const int32_t *)src, n, (int32_t *)st);
  else
    hipLaunchKernelGGL(k_rank<uint8_t>, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream,
                       h->desc.order, (const uint8_t *)src, n, (uint8_t *)st);
  LAUNCH_TRY(h, "state reorder");
  return LPA_OK;
}

// --- batches -----------------------------------------------------------------
int batch_alloc(lpa_batch *b) {
  const size_t cap = (size_t)b->capacity;
  size_t off = 0;
  off = align_up(cap * sizeof(GraphDesc));
  b->off_prefix = off;
  off = align_up(off + kPrefixArrays * (cap + 1) * sizeof(int32_t));
  b->off_finished = off;
  off = align_up(off + sizeof(int32_t));
  b->off_status = off;
  off = align_up(off + 3 * cap * sizeof(int32_t));
  b->block_bytes = off;
  if (hipMalloc(&b->dblock, off) != hipSuccess) {
    (void)hipGetLastError();
    return LPA_ERR_NOMEM;
  }
  if (hipHostMalloc(&b->hblock, off, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return LPA_ERR_NOMEM;
  }
  char *d = (char *)b->dblock, *hh = (char *)b->hblock;
  b->d_desc = (GraphDesc *)d;
  b->h_desc = (GraphDesc *)hh;
  b->d_prefix = (int32_t *)(d + b->off_prefix);
  b->h_prefix = (int32_t *)(hh + b->off_prefix);
  b->d_finished = (int32_t *)(d + b->off_finished);
  b->h_finished = (int32_t *)(hh + b->off_finished);
  b->d_status = (int32_t *)(d + b->off_status);
  b->h_status = (int32_t *)(hh + b->off_status);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LPA_ERR_HIP;
  b->device = dev;
  if (hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return LPA_ERR_HIP;
  for (int wide = 0; wide < 2; ++wide) {
    int per_cu = move_blocks_per_cu(b->k, b->async_mode, b->rescan, b->shared_vars, wide != 0);
    if (b->blocks_cap > 0 && b->blocks_cap < per_cu) per_cu = b->blocks_cap;
    b->grid_cap[wide] = b->cus * per_cu;
  }
  if (b->capture && hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    return LPA_ERR_HIP;
  }
  return LPA_OK;
}

void batch_release(lpa_batch *b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->dblock) (void)hipFree(b->dblock);
  if (b->hblock) (void)hipHostFree(b->hblock);
  delete b;
}

int move_items(const lpa_handle *h) { return h->desc.items; }

// Upload the descriptor table for hs[0..count).
int batch_load(lpa_batch *b, lpa_handle *const *hs, int count) {
  if (count < 0 || count > b->capacity) return LPA_ERR_ARG;
  int32_t *pi = b->h_prefix, *ph = b->h_prefix + (b->capacity + 1),
          *pm = b->h_prefix + 2 * (b->capacity + 1), *ps = b->h_prefix + 3 * (b->capacity + 1);
  pi[0] = ph[0] = pm[0] = ps[0] = 0;
  int unfinished = 0;
  bool wide = false;
  for (int g = 0; g < count; ++g) {
    lpa_handle *h = hs[g];
    if (!h) return LPA_ERR_ARG;
    wide = wide || h->row_ptr.p64 != nullptr;
    if (h->poisoned) return LPA_ERR_HIP;
    if (h->sm.on && b != h->self) return LPA_ERR_ARG;  // streamed graphs run alone
    if (kernel_k(h->k, h->flags) != b->k || ((h->flags & LPA_RESCAN) != 0) != b->rescan ||
        ((h->flags & LPA_HUB_SHARED) != 0) != b->hub_shared ||
        ((h->flags & LPA_SHARED_VARS) != 0) != b->shared_vars ||
        h->async_mode != b->async_mode || h->device != b->device || h->stream != b->stream)
      return LPA_ERR_ARG;
    for (int q = 0; q < g; ++q)
      if (hs[q] == h) return LPA_ERR_ARG;
    b->h_desc[g] = h->desc;
    const bool live = !h->finished;
    unfinished += live ? 1 : 0;
    const int64_t next[4] = {
        (int64_t)pi[g] + (live ? move_items(h) : 0),
        (int64_t)ph[g] + (live && b->async_mode ? h->desc.n_hubs : 0),
        (int64_t)pm[g] + (live && b->async_mode ? (h->desc.n_hubs + kMergeHubs - 1) / kMergeHubs : 0),
        (int64_t)ps[g] + (live && b->async_mode ? h->desc.n_seg : 0)};
    for (int64_t x : next)  // the launch's work item numbers are int32
      if (x > (int64_t)INT32_MAX) return LPA_ERR_UNSUPPORTED;
    pi[g + 1] = (int32_t)next[0];
    ph[g + 1] = (int32_t)next[1];
    pm[g + 1] = (int32_t)next[2];
    ps[g + 1] = (int32_t)next[3];
  }
  // pad the prefixes to the table capacity so the three arrays keep their offsets
  b->total_items = pi[count];
  b->total_hubs = ph[count];
  b->total_merge = pm[count];
  b->total_segs = ps[count];
  b->unfinished = unfinished;
  b->wide = wide;
  b->loaded.assign(hs, hs + count);
  HIP_TRY_B(b, hipMemcpyAsync(b->d_desc, b->h_desc, (size_t)count * sizeof(GraphDesc),
                              hipMemcpyHostToDevice, b->stream));
  HIP_TRY_B(b, hipMemcpyAsync(b->d_prefix, b->h_prefix,
                              kPrefixArrays * (b->capacity + 1) * sizeof(int32_t),
                              hipMemcpyHostToDevice, b->stream));
  return LPA_OK;
}

Launch make_launch(lpa_batch *b) {
  Launch L;
  L.d = b->d_desc;
  L.prefix_items = b->d_prefix;
  L.prefix_hubs = b->d_prefix + (b->capacity + 1);
  L.prefix_merge = b->d_prefix + 2 * (b->capacity + 1);
  L.prefix_segs = b->d_prefix + 3 * (b->capacity + 1);
  L.G = (int32_t)b->loaded.size();
  L.total_items = b->total_items;
  L.total_hubs = b->total_hubs;
  L.total_merge = b->total_merge;
  L.total_segs = b->total_segs;
  L.finished = b->d_finished;
  L.status_out = b->d_status;
  L.no_finish = 0;
  return L;
}

// Read the status of every loaded graph back into the handles.
int batch_read_status(lpa_batch *b) {
  const int G = (int)b->loaded.size();
  if (G > 0)
    HIP_TRY_B(b, hipMemcpyAsync(b->h_status, b->d_status, 3 * (size_t)G * sizeof(int32_t),
                                hipMemcpyDeviceToHost, b->stream));
  HIP_TRY_B(b, hipMemcpyAsync(b->h_finished, b->d_finished, sizeof(int32_t), hipMemcpyDeviceToHost,
                              b->stream));
  HIP_TRY_B(b, hipStreamSynchronize(b->stream));
  for (int g = 0; g < G; ++g) {
    lpa_handle *h = b->loaded[g];
    if (h->finished) continue;
    h->iter = b->h_status[3 * g];
    h->finished = b->h_status[3 * g + 1] != 0;
  }
  return LPA_OK;
}

// Run up to `iters` iterations of the loaded graphs; poll every check_every.
// prof: handle whose per-iteration events are recorded (single-graph runs).
int batch_iterate(lpa_batch *b, int iters, lpa_handle *prof) {
  if (b->unfinished == 0 || iters <= 0) return LPA_OK;
  const Launch L = make_launch(b);
  const int waves_per_block = kBlock / kWave;
  int grid = (b->total_items + waves_per_block - 1) / waves_per_block;
  if (grid > b->grid_cap[b->wide]) grid = b->grid_cap[b->wide];
  if (grid < 1) grid = 1;
  int mg = (b->total_merge + waves_per_block - 1) / waves_per_block;
  if (mg > b->cus * 4) mg = b->cus * 4;
  if (mg < 1) mg = 1;
  const bool profiling = prof && !prof->ev_beg.empty();
  if (b->capture && b->check_every == 0 && !profiling) {
    // every remaining iteration as one hipGraph, captured on a private
    // stream once per launch shape and replayed on the caller's stream
    // (the descriptor table it reads is uploaded before each replay)
    const long long key[9] = {iters, grid, mg, L.G, L.total_items, L.total_hubs, L.total_merge,
                              L.total_segs, b->wide};
    if (!b->graph_exec || memcmp(key, b->graph_key, sizeof(key)) != 0) {
      if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
      if (b->graph) (void)hipGraphDestroy(b->graph);
      b->graph_exec = nullptr;
      b->graph = nullptr;
      HIP_TRY_B(b, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
      hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, b->cap_stream, b->d_finished, 1);
      hipError_t e = hipSuccess;
      for (int i = 0; i < iters && e == hipSuccess; ++i)
        e = launch_iteration(b->k, b->async_mode, b->rescan, b->hub_shared, b->shared_vars,
                             b->wide, L, grid, mg, b->cap_stream, nullptr, nullptr);
      hipGraph_t g = nullptr;
      const hipError_t ee = hipStreamEndCapture(b->cap_stream, &g);
      if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail_hip_b(b, e, "iteration capture");
      }
      HIP_TRY_B(b, ee);
      b->graph = g;
      HIP_TRY_B(b, hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0));
      memcpy(b->graph_key, key, sizeof(key));
    }
    HIP_TRY_B(b, hipGraphLaunch(b->graph_exec, b->stream));
    return LPA_OK;
  }
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, b->stream, b->d_finished, 1);
  for (int i = 0; i < iters; ++i) {
    hipEvent_t eb = nullptr, ee = nullptr;
    if (prof && !prof->ev_beg.empty()) {
      const int l = prof->iter + i;
      if (l < (int)prof->ev_beg.size()) {
        eb = prof->ev_beg[l];
        ee = prof->ev_end[l];
        prof->ev_rec[l] = 1;
      }
    }
    hipError_t e =
        launch_iteration(b->k, b->async_mode, b->rescan, b->hub_shared, b->shared_vars, b->wide, L,
                         grid, mg, b->stream, eb, ee);
    if (e != hipSuccess) return fail_hip_b(b, e, "iteration launch");
    if (b->check_every > 0 && (i + 1) % b->check_every == 0 && i + 1 < iters) {
      HIP_TRY_B(b, hipMemcpyAsync(b->h_finished, b->d_finished, sizeof(int32_t),
                                  hipMemcpyDeviceToHost, b->stream));
      HIP_TRY_B(b, hipStreamSynchronize(b->stream));
      if (*b->h_finished >= b->unfinished) break;
    }
  }
  return LPA_OK;
}

int batch_error_to_handles(lpa_batch *b, int rc) {
  if (rc == LPA_ERR_HIP)
    for (lpa_handle *h : b->loaded) {
      h->poisoned = true;
      h->err = b->err;
    }
  return rc;
}

int max_remaining(lpa_batch *b) {
  int m = 0;
  for (lpa_handle *h : b->loaded)
    if (!h->finished && h->max_iter - h->iter > m) m = h->max_iter - h->iter;
  return m;
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
    case LPA_ERR_NOMEM: return "device allocation failed or workspace too small";
    case LPA_ERR_HIP: return "HIP runtime error (handle poisoned)";
    case LPA_ERR_STATE: return "handle in the wrong state for this call";
    default: return "unknown status";
  }
}

const char *lpa_last_error(const lpa_handle *h) { return h ? h->err.c_str() : ""; }

int lpa_pointer_location(const void *ptr, int *location) {
  if (!location) return LPA_ERR_ARG;
  *location = pointer_location(ptr);
  return LPA_OK;
}

static int check_config(const lpa_config &cfg) {
  for (int i = 0; i < 2; ++i)
    if (cfg.reserved[i] != 0) return LPA_ERR_ARG;
  if (cfg.move_blocks_per_cu < 0 || cfg.move_blocks_per_cu > 64) return LPA_ERR_ARG;
  if (cfg.rho < 0 || cfg.lane_max_degree < 0 || cfg.lane_max_degree > 65536 ||
      cfg.check_every < 0 || cfg.stream_chunk_kib < 0)
    return LPA_ERR_ARG;
  const uint32_t mode = cfg.flags & LPA_MODE_MASK;
  if (mode != LPA_MODE_DET && mode != LPA_MODE_ASYNC) return LPA_ERR_UNSUPPORTED;
  if ((cfg.flags &
       ~(LPA_MODE_MASK | LPA_VALIDATE | LPA_RULE_BM_PAPER | LPA_RESCAN | LPA_HUB_SHARED |
         LPA_CAPTURE | LPA_SHARED_VARS | LPA_STREAM_CSR | LPA_RANKED_LAYOUT)) != 0)
    return LPA_ERR_UNSUPPORTED;
  if (cfg.workspace_bytes && !cfg.workspace) return LPA_ERR_ARG;
  return LPA_OK;
}

int lpa_workspace_bytes(int32_t n, int64_t nnz, int k, int max_iter, const lpa_config *cfg_in,
                        size_t *bytes) {
  if (!bytes) return LPA_ERR_ARG;
  lpa_config cfg;
  if (cfg_in)
    cfg = *cfg_in;
  else
    lpa_config_default(&cfg);
  if (n < 0 || nnz < 0 || nnz >= kMaxEntries || max_iter < 0) return LPA_ERR_ARG;
  int rc = check_config(cfg);
  if (rc) return rc;
  if ((rc = check_k(k, cfg.flags)) != LPA_OK) return rc;
  const bool async_mode = (cfg.flags & LPA_MODE_MASK) == LPA_MODE_ASYNC;
  const int lane_max = cfg.lane_max_degree > 0 ? cfg.lane_max_degree : default_lane_max(async_mode);
  const Layout Ly = plan_layout(n, nnz, k, max_iter, async_mode, lane_max,
                                (cfg.flags & LPA_RESCAN) != 0, true,
                                (cfg.flags & LPA_RANKED_LAYOUT) != 0);
  if (Ly.too_many_segs) return LPA_ERR_UNSUPPORTED;
  *bytes = Ly.total;
  return LPA_OK;
}

namespace {

// Degree-bin the vertices [v0, v0 + nr) into order[0 .. nr) (hubs, lane
// vertices, then the isolated ones): the binning kernels above, with the label buffer C[0] as their count matrix
// (before the labels are initialised) and synchronising once for the
// totals.
hipError_t bin_range(lpa_handle *h, int v0, int nr, int32_t *order, int *hubs, int *lanes,
                     int *shorts = nullptr) {
  *hubs = *lanes = 0;
  if (shorts) *shorts = 0;
  if (nr <= 0) return hipSuccess;
  const int nblk = (nr + kBinIds - 1) / kBinIds;
  const size_t cells = (size_t)kBinClasses * nblk;
  const int nchunks = (int)((cells + kScanChunk - 1) / kScanChunk);
  unsigned *counts = (unsigned *)h->desc.C[0];
  hipLaunchKernelGGL(k_bin_count, dim3(nblk), dim3(256), 0, h->stream, v0, nr, h->row_ptr,
                     h->lane_max, nblk, counts);
  hipLaunchKernelGGL(k_scan_chunks, dim3(nchunks), dim3(256), 0, h->stream, counts, cells,
                     (unsigned *)h->hist);
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(64), 0, h->stream, (unsigned *)h->hist, nchunks,
                     counts, nblk, h->st->totals);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, h->stream,
                     counts, cells, (const unsigned *)h->hist);
  hipLaunchKernelGGL(k_bin_place, dim3(nblk), dim3(256), 0, h->stream, v0, nr, h->row_ptr,
                     h->lane_max, nblk, (const unsigned *)counts, order);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int totals[4] = {0, 0, 0, 0};
  if ((e = hipMemcpyAsync(totals, h->st->totals, sizeof(totals), hipMemcpyDeviceToHost,
                          h->stream)) != hipSuccess ||
      (e = hipStreamSynchronize(h->stream)) != hipSuccess)
    return e;
  *hubs = totals[0];
  *lanes = totals[1];
  if (shorts) *shorts = totals[3];
  return hipSuccess;
}

// --- LPA_STREAM_CSR ---------------------------------------------------------
// Cut the vertices into id ranges of at most the chunk size in CSR entries
// (one vertex when it alone is larger), copy the row offsets to the device
// (h->row_ptr then points there) and allocate the device side: a second
// degree order, one descriptor and prefix pair per range, two slice buffers
// sized for the largest range, a copy stream and its events.
int stream_prepare(lpa_handle *h, const lpa_graph *g, const lpa_config &cfg) {
  lpa_handle::Streamed &S = h->sm;
  S.on = true;
  S.host_col = g->col_idx;
  S.host_w = h->w;
  const int n = h->n;
  std::vector<int64_t> rp((size_t)n + 1);
  if (g->row_ptr64) {
    HIP_TRY(h, hipMemcpy(rp.data(), g->row_ptr64, ((size_t)n + 1) * 8, hipMemcpyDefault));
  } else {
    std::vector<int32_t> t((size_t)n + 1);
    HIP_TRY(h, hipMemcpy(t.data(), g->row_ptr, ((size_t)n + 1) * 4, hipMemcpyDefault));
    for (size_t i = 0; i <= (size_t)n; ++i) rp[i] = t[i];
  }
  if (rp[0] != 0 || rp[n] != h->nnz) return set_err(h, LPA_ERR_GRAPH, "row offsets");
  for (int v = 0; v < n; ++v)
    if (rp[v + 1] < rp[v] || rp[v + 1] - rp[v] > (int64_t)INT32_MAX)
      return set_err(h, LPA_ERR_GRAPH, "row offsets");
  const int64_t kib = cfg.stream_chunk_kib > 0 ? cfg.stream_chunk_kib : 262144;
  const int64_t chunk = kib * 1024 / 4;  // entries (4-byte column indices)
  int64_t cap = 1;
  for (int v0 = 0; v0 < n;) {
    const int64_t b = rp[v0];
    int v1 = v0 + 1;
    if (rp[v1] - b <= chunk) {  // the largest v1 whose rows fit the chunk
      int lo = v1, hi = n;
      while (lo < hi) {
        const int mid = lo + (hi - lo + 1) / 2;
        if (rp[mid] - b <= chunk)
          lo = mid;
        else
          hi = mid - 1;
      }
      v1 = lo;
    }
    S.first.push_back(v0);
    S.base.push_back(b);
    S.entries.push_back(rp[v1] - b);
    cap = std::max(cap, rp[v1] - b);
    v0 = v1;
  }
  S.first.push_back(n);
  const size_t P = S.base.size();
  const size_t rp_bytes = ((size_t)n + 1) * (g->row_ptr64 ? 8 : 4);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = align_up(off + (bytes ? bytes : 1));
    return at;
  };
  const size_t o_rp = take(rp_bytes), o_order = take((size_t)n * 4),
               o_desc = take(P * sizeof(GraphDesc)), o_pref = take(P * 8 * sizeof(int32_t));
  if (h->async_mode) {  // per range: pbase, hub flags, segment hubs, partials, candidates
    const int64_t Sd = h->lane_max, k = h->k;
    for (size_t p = 0; p < P; ++p) {
      const int64_t nv = S.first[p + 1] - S.first[p];
      const int32_t hc = (int32_t)std::min<int64_t>(S.entries[p] / (Sd + 1) + 1, nv);
      const int32_t sc = (int32_t)(2 * (S.entries[p] / Sd) + 2);
      S.hub_cap.push_back(hc);
      S.seg_cap.push_back(sc);
      std::array<size_t, 6> o;
      o[0] = take(((size_t)hc + 1) * 4);
      o[1] = take((size_t)hc);
      o[2] = take((size_t)sc * 4);
      o[3] = take((size_t)sc * k * 4);
      o[4] = take((size_t)sc * k * 4);
      o[5] = take((size_t)hc * k * 4);
      S.o_hub.push_back(o);
    }
  }
  constexpr int NB = lpa_handle::Streamed::kBufs;
  size_t o_col[NB], o_w[NB] = {};
  for (int i = 0; i < NB; ++i) {
    o_col[i] = take((size_t)cap * 4);
    if (S.host_w) o_w[i] = take((size_t)cap * 4);
  }
  if (hipMalloc(&S.dev, off) != hipSuccess) {
    (void)hipGetLastError();
    return set_err(h, LPA_ERR_NOMEM, "hipMalloc failed (stream buffers)");
  }
  S.dev_bytes = off;
  char *base = (char *)S.dev;
  const void *rp_src = g->row_ptr64 ? (const void *)g->row_ptr64 : (const void *)g->row_ptr;
  HIP_TRY(h, hipMemcpy(base + o_rp, rp_src, rp_bytes, hipMemcpyDefault));
  h->row_ptr = g->row_ptr64 ? RowPtr{nullptr, (const int64_t *)(base + o_rp)}
                            : RowPtr{(const int32_t *)(base + o_rp), nullptr};
  S.order = (int32_t *)(base + o_order);
  S.desc = (GraphDesc *)(base + o_desc);
  S.prefix = (int32_t *)(base + o_pref);
  for (int i = 0; i < NB; ++i) {
    S.col_buf[i] = (int32_t *)(base + o_col[i]);
    S.w_buf[i] = S.host_w ? (float *)(base + o_w[i]) : nullptr;
  }
  HIP_TRY(h, hipStreamCreateWithFlags(&S.copy, hipStreamNonBlocking));
  S.cs[0] = h->stream;
  for (int i = 1; i < NB; ++i) HIP_TRY(h, hipStreamCreateWithFlags(&S.cs[i], hipStreamNonBlocking));
  for (int i = 0; i < NB; ++i) {
    HIP_TRY(h, hipEventCreateWithFlags(&S.copied[i], hipEventDisableTiming));
    HIP_TRY(h, hipEventCreateWithFlags(&S.done[i], hipEventDisableTiming));
  }
  HIP_TRY(h, hipEventCreateWithFlags(&S.start, hipEventDisableTiming));
  return LPA_OK;
}

// Bin every range by degree into the second order and upload one
// descriptor per range: the handle's own, with that range's vertices and
// the column and weight pointers moved so that a CSR position q of the
// range addresses its slice buffer (buffer - first position + q).
int stream_bin(lpa_handle *h) {
  lpa_handle::Streamed &S = h->sm;
  const size_t P = S.base.size();
  std::vector<GraphDesc> descs(P, h->desc);
  std::vector<int32_t> pref(8 * P, 0);
  S.items.assign(P, 0);
  S.hubs.assign(P, 0);
  S.segs.assign(P, 0);
  char *dev = (char *)S.dev;
  int64_t off = 0;
  for (size_t p = 0; p < P; ++p) {
    int hubs = 0, lanes = 0;
    HIP_TRY(h, bin_range(h, S.first[p], S.first[p + 1] - S.first[p], S.order + off, &hubs,
                         &lanes));
    GraphDesc &d = descs[p];
    const int slot = (int)(p % lpa_handle::Streamed::kBufs);
    const uintptr_t shift = (uintptr_t)S.base[p] * 4;
    d.col = (const int32_t *)((uintptr_t)S.col_buf[slot] - shift);
    d.w = S.host_w ? (const float *)((uintptr_t)S.w_buf[slot] - shift) : nullptr;
    d.order = S.order + off;
    d.n_hubs = hubs;
    d.n_lane = lanes;
    d.n_short = 0;  // a range's lane vertices all run as staged lane units
    d.n_seg = 0;
    int nseg = 0;
    if (h->async_mode) {  // this range's hubs split into segments of lane_max entries
      const std::array<size_t, 6> &o = S.o_hub[p];
      d.hub_pbase = (const int32_t *)(dev + o[0]);
      d.hub_act = (uint8_t *)(dev + o[1]);
      d.seg_hub = (const int32_t *)(dev + o[2]);
      d.part_key = (int32_t *)(dev + o[3]);
      d.part_val = (float *)(dev + o[4]);
      d.hub_cand = (int32_t *)(dev + o[5]);
      if (hubs > S.hub_cap[p]) return set_err(h, LPA_ERR_GRAPH, "hub bound violated");
      if (hubs > 0) {
        hipLaunchKernelGGL(k_hub_plan, dim3(1), dim3(1024), 0, h->stream, d.order, hubs,
                           h->row_ptr, h->lane_max, (int32_t *)d.hub_pbase, &h->st->totals[2]);
        HIP_TRY(h, hipGetLastError());
        HIP_TRY(h, hipMemcpyAsync(&nseg, &h->st->totals[2], sizeof(int), hipMemcpyDeviceToHost,
                                  h->stream));
        HIP_TRY(h, hipStreamSynchronize(h->stream));
        if (nseg > S.seg_cap[p]) return set_err(h, LPA_ERR_GRAPH, "segment bound violated");
        hipLaunchKernelGGL(k_fill_seg_hub, dim3(grid_for(hubs)), dim3(kAuxBlock), 0, h->stream,
                           d.hub_pbase, hubs, (int32_t *)d.seg_hub);
        HIP_TRY(h, hipGetLastError());
      }
      d.n_seg = nseg;
      d.items = (nseg + lanes + kWave - 1) / kWave;
    } else {
      d.items = hubs + (lanes + kWave - 1) / kWave;
    }
    S.items[p] = d.items;
    S.hubs[p] = hubs;
    S.segs[p] = nseg;
    pref[8 * p + 1] = d.items;
    pref[8 * p + 3] = h->async_mode ? hubs : 0;
    pref[8 * p + 5] = h->async_mode ? (hubs + kMergeHubs - 1) / kMergeHubs : 0;
    pref[8 * p + 7] = nseg;
    off += hubs + lanes;
  }
  HIP_TRY(h, hipMemcpy(S.desc, descs.data(), P * sizeof(GraphDesc), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(S.prefix, pref.data(), pref.size() * sizeof(int32_t),
                       hipMemcpyHostToDevice));
  int cus = 1;
  HIP_TRY(h, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
  S.cus = cus;
  S.grid_cap = cus * move_blocks_per_cu(kernel_k(h->k, h->flags), h->async_mode,
                                        (h->flags & LPA_RESCAN) != 0,
                                        (h->flags & LPA_SHARED_VARS) != 0,
                                        h->row_ptr.p64 != nullptr);
  return LPA_OK;
}

void stream_release(lpa_handle *h) {
  lpa_handle::Streamed &S = h->sm;
  constexpr int NB = lpa_handle::Streamed::kBufs;
  if (S.copy) (void)hipStreamSynchronize(S.copy);
  for (int i = 1; i < NB; ++i)
    if (S.cs[i]) (void)hipStreamSynchronize(S.cs[i]);
  for (int i = 0; i < NB; ++i) {
    if (S.copied[i]) (void)hipEventDestroy(S.copied[i]);
    if (S.done[i]) (void)hipEventDestroy(S.done[i]);
  }
  if (S.start) (void)hipEventDestroy(S.start);
  for (int i = 1; i < NB; ++i)
    if (S.cs[i]) (void)hipStreamDestroy(S.cs[i]);
  if (S.copy) (void)hipStreamDestroy(S.copy);
  if (S.dev) (void)hipFree(S.dev);
  S = lpa_handle::Streamed{};
}

// Up to `iters` iterations of a streamed graph.  Range p uses buffer and
// compute stream p % kBufs: the copy stream fills the buffer once the kernel
// that last read it has finished, the compute stream runs the range's move
// kernel once the copy has landed.  The ranges of one iteration may run
// concurrently (the synchronous update reads only the previous labels and
// writes each vertex once; neighbour flags are set, never cleared, by the
// move kernels); every compute stream starts after the previous stop test,
// and the handle's stream joins them all before this iteration's.  The
// status is read back after every iteration.
int stream_iterate(lpa_handle *h, int iters) {
  lpa_handle::Streamed &S = h->sm;
  lpa_batch *b = h->self;
  lpa_handle *one[1] = {h};
  int rc;
  if ((rc = batch_load(b, one, 1)) != LPA_OK) return rc;
  const Launch L0 = make_launch(b);
  const int kk = kernel_k(h->k, h->flags);
  const bool rescan = (h->flags & LPA_RESCAN) != 0, sv = (h->flags & LPA_SHARED_VARS) != 0;
  const bool wide = h->row_ptr.p64 != nullptr;
  const int waves_per_block = kBlock / kWave;
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, h->stream, b->d_finished, 1);
  constexpr int NB = lpa_handle::Streamed::kBufs;
  for (int i = 0; i < iters && !h->finished; ++i) {
    const int l = h->iter;
    const bool prof = !h->ev_beg.empty() && l < (int)h->ev_beg.size();
    if (prof) {
      HIP_TRY(h, hipEventRecord(h->ev_beg[l], h->stream));
      h->ev_rec[l] = 1;
    }
    HIP_TRY(h, hipEventRecord(S.start, h->stream));
    for (int c = 1; c < NB; ++c) HIP_TRY(h, hipStreamWaitEvent(S.cs[c], S.start, 0));
    for (size_t p = 0; p < S.base.size(); ++p) {
      const int s = (int)(p % NB);
      if (S.entries[p] > 0) {
        HIP_TRY(h, hipStreamWaitEvent(S.copy, S.done[s], 0));
        HIP_TRY(h, hipMemcpyAsync(S.col_buf[s], S.host_col + S.base[p], (size_t)S.entries[p] * 4,
                                  hipMemcpyHostToDevice, S.copy));
        if (S.host_w)
          HIP_TRY(h, hipMemcpyAsync(S.w_buf[s], S.host_w + S.base[p], (size_t)S.entries[p] * 4,
                                    hipMemcpyHostToDevice, S.copy));
        HIP_TRY(h, hipEventRecord(S.copied[s], S.copy));
        HIP_TRY(h, hipStreamWaitEvent(S.cs[s], S.copied[s], 0));
      }
      Launch Lp = L0;
      Lp.d = S.desc + p;
      Lp.prefix_items = S.prefix + 8 * p;
      Lp.prefix_hubs = S.prefix + 8 * p + 2;
      Lp.prefix_merge = S.prefix + 8 * p + 4;
      Lp.prefix_segs = S.prefix + 8 * p + 6;
      Lp.G = 1;
      Lp.total_items = S.items[p];
      Lp.total_hubs = h->async_mode ? S.hubs[p] : 0;
      Lp.total_merge = h->async_mode ? (S.hubs[p] + kMergeHubs - 1) / kMergeHubs : 0;
      Lp.total_segs = S.segs[p];
      Lp.no_finish = 1;
      int grid = (S.items[p] + waves_per_block - 1) / waves_per_block;
      grid = std::max(1, std::min(grid, S.grid_cap));
      int mg = (Lp.total_merge + waves_per_block - 1) / waves_per_block;
      mg = std::max(1, std::min(mg, S.cus * 4));
      HIP_TRY(h, launch_iteration(kk, h->async_mode, rescan, false, sv, wide, Lp, grid, mg,
                                  S.cs[s], nullptr, nullptr));
      HIP_TRY(h, hipEventRecord(S.done[s], S.cs[s]));
    }
    for (int c = 1; c < NB; ++c) HIP_TRY(h, hipStreamWaitEvent(h->stream, S.done[c], 0));
    HIP_TRY(h, launch_finish(L0, h->stream));
    if (prof) HIP_TRY(h, hipEventRecord(h->ev_end[l], h->stream));
    if ((rc = batch_read_status(b)) != LPA_OK) return rc;
  }
  return LPA_OK;
}

}  // namespace

int lpa_free(lpa_handle *h) {
  if (!h) return LPA_OK;
  (void)hipStreamSynchronize(h->stream);
  for (hipEvent_t e : h->ev_beg) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->ev_end) (void)hipEventDestroy(e);
  for (void *p : h->eval_allocs) (void)hipFree(p);
  stream_release(h);
  if (h->part_block) (void)hipFree(h->part_block);
  if (h->owns_block && h->block) (void)hipFree(h->block);
  batch_release(h->self);
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
  int rc = check_config(cfg);
  if (rc) return rc;
  if (g->n < 0 || g->n == INT32_MAX || g->nnz < 0 || g->nnz >= kMaxEntries) return LPA_ERR_ARG;
  if (g->row_ptr && g->row_ptr64) return LPA_ERR_ARG;
  if (g->n > 0 && !g->row_ptr && !g->row_ptr64) return LPA_ERR_ARG;
  if (!g->row_ptr64 && g->nnz >= (int64_t)INT32_MAX) return LPA_ERR_ARG;  // int32 offsets
  if (g->nnz > 0 && !g->col_idx) return LPA_ERR_ARG;
  if (g->n == 0 && g->nnz != 0) return LPA_ERR_ARG;
  if (!(tol >= 0.0 && tol <= 1.0) || max_iter < 0) return LPA_ERR_ARG;
  if ((rc = check_k(k, cfg.flags)) != LPA_OK) return rc;
  // graph arrays the kernels could not read are refused here, not faulted on
  const void *rp_any = g->row_ptr64 ? (const void *)g->row_ptr64 : (const void *)g->row_ptr;
  if (g->n > 0 && pointer_location(rp_any) == LPA_PTR_UNUSABLE) return LPA_ERR_ARG;
  if (g->nnz > 0 && pointer_location(g->col_idx) == LPA_PTR_UNUSABLE) return LPA_ERR_ARG;
  if (weights && g->nnz > 0 && pointer_location(weights) == LPA_PTR_UNUSABLE) return LPA_ERR_ARG;
  const bool streamed = (cfg.flags & LPA_STREAM_CSR) != 0;
  if (streamed && g->nnz > 0 &&
      (pointer_location(g->col_idx) != LPA_PTR_HOST ||
       (weights && pointer_location(weights) != LPA_PTR_HOST)))
    return LPA_ERR_ARG;  // streaming copies from pinned host memory

  lpa_handle *h = new (std::nothrow) lpa_handle();
  if (!h) return LPA_ERR_NOMEM;
  h->stream = (hipStream_t)cfg.stream;
  h->n = g->n;
  h->nnz = g->nnz;
  h->row_ptr = RowPtr{g->row_ptr64 ? nullptr : g->row_ptr, g->row_ptr64};
  h->col = g->col_idx;
  h->w = weights;
  h->k = k;
  h->tol = tol;
  h->max_iter = max_iter;
  h->rho = cfg.rho;
  h->flags = cfg.flags;
  h->async_mode = (cfg.flags & LPA_MODE_MASK) == LPA_MODE_ASYNC;
  h->seed = seed;
  h->check_every = cfg.check_every;
  h->lane_max = cfg.lane_max_degree > 0 ? cfg.lane_max_degree : default_lane_max(h->async_mode);
  auto bail = [&](int code) {
    lpa_free(h);
    return code;
  };
  if (hipGetDevice(&h->device) != hipSuccess) return bail(LPA_ERR_HIP);

  // one block for every array of the handle: the caller's workspace or ours
  const int n = h->n;
  const bool bound_partials = cfg.workspace != nullptr;
  const bool ranked = (cfg.flags & LPA_RANKED_LAYOUT) != 0;
  const Layout Ly = plan_layout(n, h->nnz, k, max_iter, h->async_mode, h->lane_max,
                                (cfg.flags & LPA_RESCAN) != 0, bound_partials, ranked);
  if (Ly.too_many_segs) return bail(set_err(h, LPA_ERR_UNSUPPORTED, "too many hub segments"));
  if (cfg.workspace) {
    if (cfg.workspace_bytes < Ly.total || ((uintptr_t)cfg.workspace & 255) != 0)
      return bail(LPA_ERR_NOMEM);
    h->block = cfg.workspace;
  } else {
    if (hipMalloc(&h->block, Ly.total) != hipSuccess) {
      (void)hipGetLastError();
      return bail(set_err(h, LPA_ERR_NOMEM, "hipMalloc failed"));
    }
    h->owns_block = true;
  }
  h->core_bytes = Ly.total;
  if (streamed && n > 0) {
    if ((rc = stream_prepare(h, g, cfg)) != LPA_OK) return bail(rc);
  }
  char *base = (char *)h->block;
  h->st = (GraphStatus *)(base + Ly.st);
  h->hist = (uint32_t *)(base + Ly.hist);
  GraphDesc &d = h->desc;
  d.n = n;
  d.seg_len = h->lane_max;
  d.max_iter = max_iter;
  d.rho = h->rho;
  d.tol = tol;
  d.row_ptr = h->row_ptr;
  d.col = h->col;
  d.w = h->w;
  d.C[0] = (int32_t *)(base + Ly.C0);
  d.C[1] = (int32_t *)(base + Ly.C1);
  d.act[0] = (uint8_t *)(base + Ly.act0);
  d.act[1] = (uint8_t *)(base + Ly.act1);
  d.order = (const int32_t *)(base + Ly.order);
  d.dN = (unsigned long long *)(base + Ly.dN);
  d.scanned = (unsigned long long *)(base + Ly.scanned);
  d.st = h->st;
  h->hub_cap = Ly.hub_cap;
  h->seg_cap = Ly.seg_cap;
  if (Ly.seg_cap > 0) {
    d.hub_pbase = (const int32_t *)(base + Ly.hub_pbase);
    d.seg_hub = (const int32_t *)(base + Ly.seg_hub);
  }
  if (h->async_mode) {
    d.hub_act = (uint8_t *)(base + Ly.hub_act);
    d.part_key = (int32_t *)(base + Ly.pkey);
    d.part_val = (float *)(base + Ly.pval);
    d.hub_cand = (int32_t *)(base + Ly.hcand);
  }

  hipLaunchKernelGGL(k_status_set, dim3(1), dim3(64), 0, h->stream, h->st, 0, 0, 0);
  if (hipGetLastError() != hipSuccess) return bail(LPA_ERR_HIP);
  if (n > 0 && (cfg.flags & LPA_VALIDATE)) {
    hipLaunchKernelGGL(k_validate, dim3(grid_for(h->nnz > n ? (size_t)h->nnz : (size_t)n)),
                       dim3(kAuxBlock), 0, h->stream, n, h->nnz, h->row_ptr, h->col, h->w,
                       &h->st->err);
    int bad = 0;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&bad, &h->st->err, sizeof(int), hipMemcpyDeviceToHost, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
      return bail(LPA_ERR_HIP);
    if (bad) return bail(LPA_ERR_GRAPH);
  }

  // degree binning (once per graph)
  if (n > 0) {
    int hubs = 0, lanes = 0, shorts = 0;
    if (bin_range(h, 0, n, (int32_t *)d.order, &hubs, &lanes, &shorts) != hipSuccess)
      return bail(LPA_ERR_HIP);
    d.n_hubs = hubs;
    d.n_lane = lanes;
    // short units: single scan only (the double scan's second pass stays in
    // the staged lane units), and not for a streamed CSR, whose ranges are
    // binned on their own
    d.n_short = (cfg.flags & (LPA_RESCAN | LPA_STREAM_CSR)) ? 0 : shorts;
  }
  // split every hub into segments of lane_max entries (async: the move
  // kernels' work items; both modes: modularity's)
  if (d.n_hubs > 0 && h->seg_cap > 0) {
    if (d.n_hubs > h->hub_cap) return bail(set_err(h, LPA_ERR_GRAPH, "hub bound violated"));
    hipLaunchKernelGGL(k_hub_plan, dim3(1), dim3(1024), 0, h->stream, d.order, d.n_hubs,
                       h->row_ptr, h->lane_max, (int32_t *)d.hub_pbase, &h->st->totals[2]);
    int nseg = 0;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&nseg, &h->st->totals[2], sizeof(int), hipMemcpyDeviceToHost, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
      return bail(LPA_ERR_HIP);
    if (nseg > h->seg_cap) return bail(set_err(h, LPA_ERR_GRAPH, "segment bound violated"));
    h->n_segs = nseg;
    if (h->async_mode) d.n_seg = nseg;  // det mode scans whole hub rows
    hipLaunchKernelGGL(k_fill_seg_hub, dim3(grid_for(d.n_hubs)), dim3(kAuxBlock), 0, h->stream,
                       d.hub_pbase, d.n_hubs, (int32_t *)d.seg_hub);
    if (hipGetLastError() != hipSuccess) return bail(LPA_ERR_HIP);
    if (h->async_mode && !bound_partials && !streamed && nseg > 0) {  // partial sketches for exactly nseg
      const size_t half = align_up((size_t)nseg * k * 4);
      if (hipMalloc(&h->part_block, 2 * half) != hipSuccess) {
        (void)hipGetLastError();
        return bail(set_err(h, LPA_ERR_NOMEM, "hipMalloc failed (partial sketches)"));
      }
      h->core_bytes += 2 * half;
      d.part_key = (int32_t *)h->part_block;
      d.part_val = (float *)((char *)h->part_block + half);
    }
  }
  // det mode: at iteration 0 the hub chains may skip their slot lookups when
  // no hub row repeats a neighbour (checked on the column indices in device
  // memory; otherwise the general chain runs)
  if (!h->async_mode && !streamed && d.n_hubs > 0 && h->nnz > 0 &&
      pointer_location(h->col) == LPA_PTR_DEVICE) {
    hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, h->stream, &h->st->totals[3], 1);
    hipLaunchKernelGGL(k_check_hub_rows, dim3(grid_for(d.n_hubs, 4, 4096)), dim3(256), 0,
                       h->stream, d.order, d.n_hubs, h->row_ptr, h->col, &h->st->totals[3]);
    int bad = 1;
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(&bad, &h->st->totals[3], sizeof(int), hipMemcpyDeviceToHost, h->stream) !=
            hipSuccess ||
        hipStreamSynchronize(h->stream) != hipSuccess)
      return bail(LPA_ERR_HIP);
    d.hub_rows_distinct = bad ? 0 : 1;
  }
  // ranked layout: every vertex's state moves to its degree-order position,
  // and the column indices are rewritten as positions (C[0] holds the
  // positions meanwhile; the reset below sets the labels)
  if (ranked && n > 0) {
    h->colr = (int32_t *)(base + Ly.colr);
    h->tmp = base + Ly.tmp;
    hipLaunchKernelGGL(k_positions, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream, d.order, n,
                       d.C[0]);
    if (h->nnz > 0)
      hipLaunchKernelGGL(k_remap_cols, dim3(grid_for((size_t)h->nnz, kAuxBlock, 8192)),
                         dim3(kAuxBlock), 0, h->stream, h->col, h->nnz, d.C[0], h->colr);
    if (hipGetLastError() != hipSuccess) return bail(LPA_ERR_HIP);
    d.col = h->colr;
    d.ranked = 1;
  }
  d.hub_shared = (cfg.flags & LPA_HUB_SHARED) ? 1 : 0;
  d.items = (int32_t)(h->async_mode ? lane_items((d.hub_shared ? 0 : d.n_seg) + d.n_lane, d.n_short)
                                    : d.n_hubs + lane_items(d.n_lane, d.n_short));
  if (h->sm.on && (rc = stream_bin(h)) != LPA_OK) return bail(rc);

  // the batch of one that lpa_step / lpa_run use
  h->self = new (std::nothrow) lpa_batch();
  if (!h->self) return bail(LPA_ERR_NOMEM);
  h->self->capacity = 1;
  h->self->k = kernel_k(k, cfg.flags);
  h->self->rescan = (cfg.flags & LPA_RESCAN) != 0;
  h->self->hub_shared = (cfg.flags & LPA_HUB_SHARED) != 0;
  h->self->shared_vars = (cfg.flags & LPA_SHARED_VARS) != 0;
  h->self->capture = (cfg.flags & LPA_CAPTURE) != 0;
  h->self->async_mode = h->async_mode;
  h->self->stream = h->stream;
  h->self->check_every = h->check_every;
  h->self->blocks_cap = cfg.move_blocks_per_cu;
  if ((rc = batch_alloc(h->self)) != LPA_OK) return bail(rc);
  if ((rc = enqueue_reset(h)) != LPA_OK) return bail(rc);
  if (hipStreamSynchronize(h->stream) != hipSuccess) return bail(LPA_ERR_HIP);
  *out = h;
  return LPA_OK;
}

int lpa_set_stream(lpa_handle *h, void *stream) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (h->sm.on) return set_err(h, LPA_ERR_ARG, "a streamed CSR keeps the streams of lpa_init");
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  h->stream = (hipStream_t)stream;
  h->self->stream = h->stream;
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
  lpa_batch *b = h->self;
  lpa_handle *one[1] = {h};
  if (h->sm.on) {
    if ((rc = stream_iterate(h, 1)) != LPA_OK) return batch_error_to_handles(b, rc);
  } else {
    if ((rc = batch_load(b, one, 1)) != LPA_OK) return batch_error_to_handles(b, rc);
    if ((rc = batch_iterate(b, 1, h)) != LPA_OK) return batch_error_to_handles(b, rc);
  }
  unsigned long long dn = 0;
  HIP_TRY(h, hipMemcpyAsync(&dn, h->desc.dN + l, sizeof(dn), hipMemcpyDeviceToHost, h->stream));
  if ((rc = batch_read_status(b)) != LPA_OK) return batch_error_to_handles(b, rc);
  if (changed) *changed = (int64_t)dn;
  if (done) *done = h->finished ? 1 : 0;
  return LPA_OK;
}

int lpa_run(lpa_handle *h, int *iterations) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!h->finished && h->sm.on) {
    if ((rc = stream_iterate(h, h->max_iter - h->iter)) != LPA_OK)
      return batch_error_to_handles(h->self, rc);
  } else if (!h->finished) {
    lpa_batch *b = h->self;
    lpa_handle *one[1] = {h};
    if ((rc = batch_load(b, one, 1)) != LPA_OK) return batch_error_to_handles(b, rc);
    if ((rc = batch_iterate(b, h->max_iter - h->iter, h)) != LPA_OK)
      return batch_error_to_handles(b, rc);
    if ((rc = batch_read_status(b)) != LPA_OK) return batch_error_to_handles(b, rc);
  }
  if (iterations) *iterations = h->iter;
  return LPA_OK;
}

int lpa_batch_create(int capacity, int k, const lpa_config *cfg_in, lpa_batch **out) {
  if (!out) return LPA_ERR_ARG;
  *out = nullptr;
  if (capacity < 1 || capacity > (1 << 24)) return LPA_ERR_ARG;
  lpa_config cfg;
  if (cfg_in)
    cfg = *cfg_in;
  else
    lpa_config_default(&cfg);
  int rc = check_config(cfg);
  if (rc) return rc;
  if ((rc = check_k(k, cfg.flags)) != LPA_OK) return rc;
  lpa_batch *b = new (std::nothrow) lpa_batch();
  if (!b) return LPA_ERR_NOMEM;
  b->capacity = capacity;
  b->k = kernel_k(k, cfg.flags);
  b->rescan = (cfg.flags & LPA_RESCAN) != 0;
  b->hub_shared = (cfg.flags & LPA_HUB_SHARED) != 0;
  b->shared_vars = (cfg.flags & LPA_SHARED_VARS) != 0;
  b->capture = (cfg.flags & LPA_CAPTURE) != 0;
  b->async_mode = (cfg.flags & LPA_MODE_MASK) == LPA_MODE_ASYNC;
  b->stream = (hipStream_t)cfg.stream;
  b->check_every = cfg.check_every;
  b->blocks_cap = cfg.move_blocks_per_cu;
  if ((rc = batch_alloc(b)) != LPA_OK) {
    batch_release(b);
    return rc;
  }
  *out = b;
  return LPA_OK;
}

int lpa_batch_reset(lpa_batch *b, lpa_handle *const *hs, int count) {
  if (!b || (count > 0 && !hs)) return LPA_ERR_ARG;
  if (b->poisoned) return LPA_ERR_HIP;
  int rc = batch_load(b, hs, count);
  if (rc) return batch_error_to_handles(b, rc);
  if (count == 0) return LPA_OK;
  int maxn = 1;
  for (int g = 0; g < count; ++g) maxn = hs[g]->n > maxn ? hs[g]->n : maxn;
  const int gx = grid_for((size_t)maxn, kAuxBlock, 1024);
  const int gy = count < 65535 ? count : 65535;
  hipLaunchKernelGGL(k_batch_reset, dim3(gx, gy), dim3(kAuxBlock), 0, b->stream, b->d_desc, count);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return batch_error_to_handles(b, fail_hip_b(b, e, "batch reset"));
  for (int g = 0; g < count; ++g) {
    hs[g]->iter = 0;
    hs[g]->finished = hs[g]->n == 0 || hs[g]->max_iter == 0;
  }
  return LPA_OK;
}

int lpa_batch_free(lpa_batch *b) {
  batch_release(b);
  return LPA_OK;
}

int lpa_batch_step(lpa_batch *b, lpa_handle *const *hs, int count, int64_t *changed,
                   int *all_done) {
  if (!b || (count > 0 && !hs)) return LPA_ERR_ARG;
  if (b->poisoned) return LPA_ERR_HIP;
  int rc = batch_load(b, hs, count);
  if (rc) return batch_error_to_handles(b, rc);
  std::vector<char> ran(count);
  for (int g = 0; g < count; ++g) ran[g] = !hs[g]->finished;
  if ((rc = batch_iterate(b, 1, nullptr)) != LPA_OK) return batch_error_to_handles(b, rc);
  // the stop test wrote every graph's iteration, status and dN into the
  // status table, which this reads back with one copy
  if ((rc = batch_read_status(b)) != LPA_OK) return batch_error_to_handles(b, rc);
  int64_t total = 0;
  bool all = true;
  for (int g = 0; g < count; ++g) {
    if (ran[g]) total += (int64_t)b->h_status[3 * g + 2];
    all = all && hs[g]->finished;
  }
  if (changed) *changed = total;
  if (all_done) *all_done = all ? 1 : 0;
  return LPA_OK;
}

int lpa_batch_run(lpa_batch *b, lpa_handle *const *hs, int count, int *iterations) {
  if (!b || (count > 0 && !hs)) return LPA_ERR_ARG;
  if (b->poisoned) return LPA_ERR_HIP;
  int rc = batch_load(b, hs, count);
  if (rc) return batch_error_to_handles(b, rc);
  if ((rc = batch_iterate(b, max_remaining(b), nullptr)) != LPA_OK)
    return batch_error_to_handles(b, rc);
  if ((rc = batch_read_status(b)) != LPA_OK) return batch_error_to_handles(b, rc);
  int m = 0;
  for (int g = 0; g < count; ++g) m = hs[g]->iter > m ? hs[g]->iter : m;
  if (iterations) *iterations = m;
  return LPA_OK;
}

int lpa_get_labels(lpa_handle *h, int32_t *out, int out_is_host) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!out && h->n > 0) return LPA_ERR_ARG;
  if (h->n > 0 && (rc = state_out(h, cur_labels(h), out, sizeof(int32_t), out_is_host)) != LPA_OK)
    return rc;
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
      HIP_TRY(h, hipMemcpy(tmp.data(), h->desc.dN, m * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost));
      for (int i = 0; i < m; ++i) changed[i] = (int64_t)tmp[i];
    }
    if (scanned) {
      HIP_TRY(h, hipMemcpy(tmp.data(), h->desc.scanned, m * sizeof(unsigned long long),
                           hipMemcpyDeviceToHost));
      for (int i = 0; i < m; ++i) scanned[i] = (int64_t)tmp[i];
    }
  }
  if (count) *count = cnt;
  return LPA_OK;
}

}  // extern "C"

namespace {

// Modularity of `labels` (NULL: the handle's current labels) with the
// community totals in tot[0, n) (all zero on entry; left zero) and the four
// fp64 accumulators in acc.
int modularity_into(lpa_handle *h, const int32_t *labels, double *q, double *tot, double *acc) {
  const int n = h->n;
  if (labels && pointer_location(labels) == LPA_PTR_UNUSABLE)
    return set_err(h, LPA_ERR_ARG, "labels must be device or mapped pinned host memory");
  const int32_t *lab = labels ? labels : cur_labels(h);
  const GraphDesc &d = h->desc;
  hipLaunchKernelGGL(k_status_clear_err, dim3(1), dim3(64), 0, h->stream, h->st);
  if (labels) {  // the library's own labels are in range by construction
    hipLaunchKernelGGL(k_check_labels, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream, labels, n,
                       &h->st->err);
    LAUNCH_TRY(h, "label check");
    int bad = 0;
    HIP_TRY(h, hipMemcpyAsync(&bad, &h->st->err, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipStreamSynchronize(h->stream));
    if (bad) {
      hipLaunchKernelGGL(k_status_clear_err, dim3(1), dim3(64), 0, h->stream, h->st);
      LAUNCH_TRY(h, "label check reset");
      return set_err(h, LPA_ERR_GRAPH, "label out of range [0, n)");
    }
  }
  hipLaunchKernelGGL(k_zero_d, dim3(1), dim3(64), 0, h->stream, acc, 4);
  ModArgs m;
  m.order = d.order;
  m.n_hubs = d.n_hubs;
  m.n_lane = d.n_lane;
  m.n_short = d.n_short;
  // hubs are read segment by segment (one wavefront per segment) when the
  // handle planned its segments; otherwise one wavefront per hub
  m.n_seg = h->sm.on ? 0 : h->n_segs;
  m.seg_len = h->lane_max;
  m.seg_hub = d.seg_hub;
  m.hub_pbase = d.hub_pbase;
  m.row_ptr = h->row_ptr;
  // the handle's own labels are stored ranked with a ranked layout; a
  // caller's labels are indexed by vertex id
  m.ranked = labels ? 0 : d.ranked;
  m.col = labels ? h->col : d.col;
  m.w = h->w;
  m.lab = lab;
  m.tot = tot;
  m.acc = acc;
  if (h->mod_grid == 0) h->mod_grid = h->self->cus * modularity_blocks_per_cu();
  HIP_TRY(h, launch_modularity(m, h->mod_grid, h->stream));
  hipLaunchKernelGGL(k_mod_sq, dim3(grid_for(n, kAuxBlock, kModSqBlocks)), dim3(kAuxBlock), 0, h->stream,
                     tot, n, acc);
  LAUNCH_TRY(h, "modularity kernels");
  double out[4] = {0, 0, 0, 0};
  HIP_TRY(h, hipMemcpyAsync(out, acc, sizeof(out), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  const double two_m = out[0];
  *q = two_m > 0.0 ? out[1] / two_m - out[2] / (two_m * two_m) : 0.0;
  return LPA_OK;
}

// The allocation-free variant's scratch: the community totals of up to
// kScratchVertices vertices and the four accumulators, one copy per device
// (held until the process ends).  Host code never uses the symbol itself:
// its device address is looked up once per device (scratch_on_device) and
// that address is what the kernels receive.
constexpr int kScratchVertices = 1 << 21;
constexpr int kScratchDevices = 64;

}  // namespace

static __device__ __align__(256) double scratch[kScratchVertices + 32];

namespace {

std::mutex scratch_mu;
double *scratch_ptr[kScratchDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call made with that device current; nullptr on failure.
double *scratch_on_device(int dev) {
  if (dev < 0 || dev >= kScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    scratch_ptr[dev] = (double *)p;
  }
  return scratch_ptr[dev];
}

}  // namespace

extern "C" {

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
    void *p = nullptr;
    if (hipMalloc(&p, align_up((size_t)n * sizeof(double)) + 256) != hipSuccess) {
      (void)hipGetLastError();
      return set_err(h, LPA_ERR_NOMEM, "hipMalloc failed");
    }
    h->eval_allocs.push_back(p);
    h->eval_bytes += align_up((size_t)n * sizeof(double)) + 256;
    h->mod_tot = (double *)p;
    h->mod_acc = (double *)((char *)p + align_up((size_t)n * sizeof(double)));
    hipLaunchKernelGGL(k_zero_d, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream, h->mod_tot, n);
  }
  return modularity_into(h, labels, q, h->mod_tot, h->mod_acc);
}

int lpa_modularity_noalloc(lpa_handle *h, const int32_t *labels, double *q) {
  int rc = check_ready(h);
  if (rc) return rc;
  if (!q) return LPA_ERR_ARG;
  const int n = h->n;
  if (n > kScratchVertices)
    return set_err(h, LPA_ERR_UNSUPPORTED,
                   "lpa_modularity_noalloc: more vertices than its static scratch holds (2^21)");
  if (n == 0) {
    *q = 0.0;
    return LPA_OK;
  }
  int dev = -1;
  HIP_TRY(h, hipGetDevice(&dev));
  if (dev != h->device)
    return set_err(h, LPA_ERR_ARG, "lpa_modularity_noalloc: the handle's device must be current");
  double *sp = scratch_on_device(dev);
  if (!sp) return set_err(h, LPA_ERR_HIP, "lpa_modularity_noalloc: scratch address lookup failed");
  double *tot = sp, *acc = sp + kScratchVertices;
  // the totals must start at zero whatever an earlier call left behind
  hipLaunchKernelGGL(k_zero_d, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream, tot, n);
  LAUNCH_TRY(h, "scratch clear");
  return modularity_into(h, labels, q, tot, acc);
}

int lpa_get_state(lpa_handle *h, int32_t *labels, uint8_t *unprocessed, int *iteration,
                  int is_host) {
  int rc = check_ready(h);
  if (rc) return rc;
  const int n = h->n;
  if (n > 0 && labels &&
      (rc = state_out(h, cur_labels(h), labels, sizeof(int32_t), is_host)) != LPA_OK)
    return rc;
  if (n > 0 && unprocessed && (rc = state_out(h, cur_flags(h), unprocessed, 1, is_host)) != LPA_OK)
    return rc;
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
      hipLaunchKernelGGL(k_status_clear_err, dim3(1), dim3(64), 0, h->stream, h->st);
      hipLaunchKernelGGL(k_check_labels, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream, labels,
                         n, &h->st->err);
      LAUNCH_TRY(h, "label check");
      int bad = 0;
      HIP_TRY(h, hipMemcpyAsync(&bad, &h->st->err, sizeof(int), hipMemcpyDeviceToHost, h->stream));
      HIP_TRY(h, hipStreamSynchronize(h->stream));
      if (bad) return set_err(h, LPA_ERR_GRAPH, "label out of range [0, n)");
    }
  }
  // counters of every iteration start from zero again
  if ((rc = enqueue_reset(h)) != LPA_OK) return rc;
  const GraphDesc &d = h->desc;
  if (n > 0) {
    uint8_t *cur = d.act[iteration & 1];
    if ((rc = state_in(h, labels, d.C[0], sizeof(int32_t), is_host)) != LPA_OK) return rc;
    if (d.C[1] != d.C[0])  // both buffers: vertices of degree 0 are never rewritten
      HIP_TRY(h, hipMemcpyAsync(d.C[1], d.C[0], (size_t)n * sizeof(int32_t),
                                hipMemcpyDeviceToDevice, h->stream));
    if ((rc = state_in(h, unprocessed, cur, 1, is_host)) != LPA_OK) return rc;
    hipLaunchKernelGGL(k_normalize_u8, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream, cur, n);
    if (d.act[1] != d.act[0])
      hipLaunchKernelGGL(k_fill_u8, dim3(grid_for(n)), dim3(kAuxBlock), 0, h->stream,
                         d.act[(iteration + 1) & 1], (size_t)n, (uint8_t)0);
    LAUNCH_TRY(h, "state restore");
  }
  const bool fin = (n == 0 || iteration >= h->max_iter);
  // labels restored from the caller are not the initial ones, even at iteration 0
  hipLaunchKernelGGL(k_status_set, dim3(1), dim3(64), 0, h->stream, h->st, iteration, fin ? 1 : 0,
                     0);
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
  h->ev_rec.clear();
  if (enable) {
    const int T = h->max_iter > 0 ? h->max_iter : 1;
    h->ev_beg.resize(T);
    h->ev_end.resize(T);
    h->ev_rec.assign(T, 0);
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
  // iterations run before profiling was enabled, restored by lpa_set_state
  // or run through a batch have no events: -1
  for (int i = 0; i < cnt && i < capacity && move_ms; ++i)
    move_ms[i] = -1.0f;
  for (int i = 0; i < cnt && i < capacity && move_ms; ++i)
    if (i < (int)h->ev_rec.size() && h->ev_rec[i])
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
    hipLaunchKernelGGL(k_scan_floor, dim3(4096), dim3(kAuxBlock), 0, h->stream, h->desc.col, h->w,
                       (const int32_t *)cur_labels(h), h->nnz, &h->st->sink);
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

int lpa_progress(const lpa_handle *h, int *iteration, int *finished) {
  if (!h) return LPA_ERR_ARG;
  if (h->poisoned) return LPA_ERR_HIP;
  if (iteration) *iteration = h->iter;
  if (finished) *finished = h->finished ? 1 : 0;
  return LPA_OK;
}

int lpa_memory(const lpa_handle *h, size_t *core_bytes, size_t *eval_bytes) {
  if (!h) return LPA_ERR_ARG;
  if (core_bytes) *core_bytes = h->core_bytes + h->sm.dev_bytes;
  if (eval_bytes) *eval_bytes = h->eval_bytes;
  return LPA_OK;
}

}  // extern "C"
