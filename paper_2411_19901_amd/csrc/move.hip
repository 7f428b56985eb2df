// lpaMove kernels for gfx950 (paper Algorithm 1, lpaMove; Algorithm 2,
// sketchAccumulate; Sections 4.1-4.5).
//
// One persistent kernel per iteration.  Work items are the hubs (one
// wavefront per vertex, in decreasing degree) followed by chunks of 64
// lower-degree vertices (one lane per vertex), dealt to the wavefronts
// round-robin; vertices were ordered by decreasing degree once per graph, so
// every wavefront receives a similar mix.  Changed and scanned counts are
// kept per wavefront and added to the global counters once at the end.
//
// Sketch step (Section 4.1, with the decrement reading used throughout the
// library): a pair (c, w) adds w to the slot holding c; otherwise it fills a
// free slot (value 0); otherwise every slot loses d = min(w, smallest slot)
// and the residue w - d, if positive, fills a slot that became free.  Keys
// left behind in free slots may still match c: adding w to a free slot that
// holds c gives the same multiset of live (label, weight) pairs as placing
// (c, w) in any free slot, and keys stay unique because a key is only
// written when c is in no slot.  A weight of 0 leaves the sketch unchanged,
// which is how self-loops are skipped without a branch.
//
// LPA_MODE_DET: every sketch is fed in CSR order; labels are read from C and
// every binned vertex writes its label for the next iteration into Cn
// (Jacobi, double-buffered labels).
// LPA_MODE_ASYNC: labels and flags are updated in place; a hub is scanned
// by 64 lanes with one partial sketch each, merged pairwise (Section 4.3).
#include "lpa_internal.h"

#include <limits.h>
#include <math.h>

namespace lpa {

__device__ __forceinline__ int rfl(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float rfl_f(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ unsigned long long rfl_u64(unsigned long long x) {
  unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)x);
  unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(x >> 32));
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ int lanes_below(unsigned long long m) {
  return __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// ---------------------------------------------------------------------------
// Register sketch: one lane owns all K slots.
// ---------------------------------------------------------------------------
template <int K>
struct LaneSketch {
  int key[K];
  float val[K];

  __device__ __forceinline__ void clear() {
#pragma unroll
    for (int s = 0; s < K; ++s) {
      key[s] = -1;
      val[s] = 0.0f;
    }
  }

  __device__ __forceinline__ void add(int c, float w) {
    bool hit = false;
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const bool m = key[s] == c;
      hit = hit || m;
      val[s] = m ? val[s] + w : val[s];
    }
    if (!hit) {
      // With a free slot the minimum is 0: nothing is subtracted and the
      // whole weight is placed.  Otherwise the decrement step.
      float d = w;
#pragma unroll
      for (int s = 0; s < K; ++s) d = fminf(d, val[s]);
#pragma unroll
      for (int s = 0; s < K; ++s) val[s] = val[s] - d;
      const float r = w - d;
      bool placed = !(r > 0.0f);
#pragma unroll
      for (int s = 0; s < K; ++s) {
        const bool t = !placed && val[s] == 0.0f;
        key[s] = t ? c : key[s];
        val[s] = t ? r : val[s];
        placed = placed || t;
      }
    }
  }

  // Heaviest live slot, ties to the lowest label; keep when empty.
  __device__ __forceinline__ int max_key(int keep) const {
    int bk = keep;
    float bv = 0.0f;
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const bool better = val[s] > bv || (val[s] == bv && val[s] > 0.0f && key[s] < bk);
      bk = better ? key[s] : bk;
      bv = better ? val[s] : bv;
    }
    return bk;
  }
};

// ---------------------------------------------------------------------------
// Wave sketch: lane s < K owns slot s; every lane sees the same (c, w).
// ---------------------------------------------------------------------------
template <int K>
__device__ __forceinline__ void wave_sketch_add(int &key, float &val, int c, float w, int lane) {
  const bool mine = lane < K;
  const bool eq = mine && key == c;
  if (__ballot(eq)) {
    if (eq) val = val + w;
    return;
  }
  unsigned long long z = __ballot(mine && val == 0.0f);
  float r = w;
  if (z == 0ull) {
    float m = mine ? val : INFINITY;
#pragma unroll
    for (int off = K / 2; off >= 1; off >>= 1) m = fminf(m, __shfl_xor(m, off));
    const float d = fminf(w, rfl_f(m));
    if (mine) val = val - d;
    r = w - d;
    if (!(r > 0.0f)) return;
    z = __ballot(mine && val == 0.0f);
  }
  const int s = __ffsll((long long)z) - 1;
  if (lane == s) {
    key = c;
    val = r;
  }
}

template <int K>
__device__ __forceinline__ int wave_max_key(int key, float val, int lane, int keep) {
  const bool live = lane < K && val > 0.0f;
  float bv = live ? val : 0.0f;
  int bk = live ? key : INT_MAX;
#pragma unroll
  for (int off = K / 2; off >= 1; off >>= 1) {
    const float ov = __shfl_xor(bv, off);
    const int ok = __shfl_xor(bk, off);
    const bool better = ov > bv || (ov == bv && ok < bk);
    bv = better ? ov : bv;
    bk = better ? ok : bk;
  }
  bv = rfl_f(bv);
  bk = rfl(bk);
  return bv > 0.0f ? bk : keep;
}

// ---------------------------------------------------------------------------
// Lane path: one lane per vertex, CSR order (exact for LPA_MODE_DET).
// ---------------------------------------------------------------------------
template <int K, bool ASYNC>
__device__ __forceinline__ void lane_vertex(const MoveArgs &a, int v, unsigned long long &scanned,
                                            unsigned long long &changed) {
  bool active = false;
  int beg = 0, end = 0, cv = 0;
  if (v >= 0) {
    active = a.act_cur[v] != 0;
    cv = a.C[v];
    if (active) {
      a.act_cur[v] = 0;
      beg = a.row_ptr[v];
      end = a.row_ptr[v + 1];
    }
  }
  LaneSketch<K> S;
  S.clear();
  if (a.w) {
    for (int e = beg; e < end; ++e) {
      const int j = a.col[e];
      const float x = a.w[e];
      S.add(a.C[j], j == v ? 0.0f : x);
    }
  } else {
    for (int e = beg; e < end; ++e) {
      const int j = a.col[e];
      S.add(a.C[j], j == v ? 0.0f : 1.0f);
    }
  }
  const int c = S.max_key(cv);
  const bool moved = active && c != cv && (!a.pickless || c < cv);
  if (ASYNC) {
    if (moved) a.C[v] = c;
  } else if (v >= 0) {
    a.Cn[v] = moved ? c : cv;
  }
  changed += (unsigned long long)__popcll(__ballot(moved));
  if (moved)
    for (int e = beg; e < end; ++e) a.act_next[a.col[e]] = 1;
  if (active) scanned += (unsigned long long)(end - beg);
}

// ---------------------------------------------------------------------------
// Hub path, LPA_MODE_DET: one wavefront per vertex.  The 64 lanes load and
// gather 64 consecutive neighbours at a time; the sketch then consumes them
// one by one in CSR order.
// ---------------------------------------------------------------------------
template <int K>
__device__ void hub_vertex_det(const MoveArgs &a, int v, unsigned long long &scanned,
                               unsigned long long &changed) {
  const int lane = threadIdx.x & (kWave - 1);
  const int cv = a.C[v];
  if (a.act_cur[v] == 0) {
    if (lane == 0) a.Cn[v] = cv;
    return;
  }
  if (lane == 0) a.act_cur[v] = 0;
  const int beg = a.row_ptr[v], end = a.row_ptr[v + 1];
  int key = -1;
  float val = 0.0f;
  int e = beg + lane;
  int nlab = 0;
  float nw = 0.0f;
  if (e < end) {
    const int j = a.col[e];
    nw = (j == v) ? 0.0f : (a.w ? a.w[e] : 1.0f);
    nlab = a.C[j];
  }
  for (int base = beg; base < end; base += kWave) {
    const int lab = nlab;
    const float x = nw;
    // prefetch the next 64 neighbours while this block is consumed
    e = base + kWave + lane;
    if (e < end) {
      const int j = a.col[e];
      nw = (j == v) ? 0.0f : (a.w ? a.w[e] : 1.0f);
      nlab = a.C[j];
    }
    const int cnt = min(kWave, end - base);
    for (int t = 0; t < cnt; ++t) {
      const int c = __builtin_amdgcn_readlane(lab, t);
      const float xw = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), t));
      if (xw == 0.0f) continue;
      wave_sketch_add<K>(key, val, c, xw, lane);
    }
  }
  const int c = wave_max_key<K>(key, val, lane, cv);
  const bool moved = c != cv && (!a.pickless || c < cv);
  if (lane == 0) a.Cn[v] = moved ? c : cv;
  if (moved) {
    changed += 1;
    for (int q = beg + lane; q < end; q += kWave) a.act_next[a.col[q]] = 1;
  }
  scanned += (unsigned long long)(end - beg);
}

// ---------------------------------------------------------------------------
// Hub path, LPA_MODE_ASYNC: lane l keeps a partial sketch of neighbours
// beg + l, beg + l + 64, ...; the 64 partial sketches are merged by feeding
// the partner's live slots into one's own (Section 4.3), six times.
// ---------------------------------------------------------------------------
template <int K>
__device__ void hub_vertex_async(const MoveArgs &a, int v, unsigned long long &scanned,
                                 unsigned long long &changed) {
  const int lane = threadIdx.x & (kWave - 1);
  if (a.act_cur[v] == 0) return;
  if (lane == 0) a.act_cur[v] = 0;
  const int beg = a.row_ptr[v], end = a.row_ptr[v + 1];
  const int cv = a.C[v];
  LaneSketch<K> S;
  S.clear();
  if (a.w) {
    for (int e = beg + lane; e < end; e += kWave) {
      const int j = a.col[e];
      const float x = a.w[e];
      S.add(a.C[j], j == v ? 0.0f : x);
    }
  } else {
    for (int e = beg + lane; e < end; e += kWave) {
      const int j = a.col[e];
      S.add(a.C[j], j == v ? 0.0f : 1.0f);
    }
  }
#pragma unroll 1
  for (int off = kWave / 2; off >= 1; off >>= 1) {
    int pk[K];
    float pv[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {  // snapshot the partner before merging
      pk[s] = __shfl_xor(S.key[s], off);
      pv[s] = __shfl_xor(S.val[s], off);
    }
#pragma unroll
    for (int s = 0; s < K; ++s) S.add(pk[s], pv[s] > 0.0f ? pv[s] : 0.0f);
  }
  const int c = rfl(S.max_key(cv));
  const bool moved = c != cv && (!a.pickless || c < cv);
  if (moved) {
    if (lane == 0) a.C[v] = c;
    changed += 1;
    for (int q = beg + lane; q < end; q += kWave) a.act_next[a.col[q]] = 1;
  }
  scanned += (unsigned long long)(end - beg);
}

// ---------------------------------------------------------------------------
template <int K, bool ASYNC>
__global__ __launch_bounds__(kBlock) void k_move(MoveArgs a) {
  if (*a.done) return;
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = (blockIdx.x * kBlock + threadIdx.x) / kWave;
  const int nwaves = gridDim.x * (kBlock / kWave);
  // per-wavefront totals: hub counts are uniform, lane counts are summed
  // over the wavefront before they are added
  unsigned long long scanned_lane = 0, changed_w = 0, scanned_w = 0;
  for (int item = wave; item < a.total_items; item += nwaves) {
    if (item < a.n_hubs) {
      const int v = a.order[item];
      if (ASYNC)
        hub_vertex_async<K>(a, v, scanned_w, changed_w);
      else
        hub_vertex_det<K>(a, v, scanned_w, changed_w);
    } else {
      const int idx = (item - a.n_hubs) * kWave + lane;
      const int v = idx < a.n_lane ? a.order[a.n_hubs + idx] : -1;
      lane_vertex<K, ASYNC>(a, v, scanned_lane, changed_w);
    }
  }
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) scanned_lane += __shfl_xor(scanned_lane, off);
  if (lane == 0) {
    const unsigned long long sc = scanned_lane + scanned_w;
    if (sc) atomicAdd(a.scanned + a.iter, sc);
    if (changed_w) atomicAdd(a.dN + a.iter, changed_w);
  }
}

template <int K, bool ASYNC>
static hipError_t launch_t(const MoveArgs &a, int grid, hipStream_t s) {
  hipLaunchKernelGGL((k_move<K, ASYNC>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <int K, bool ASYNC>
static int occ_t() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)k_move<K, ASYNC>, kBlock, 0) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

template <bool ASYNC>
static hipError_t launch_mode(int k, const MoveArgs &a, int grid, hipStream_t s) {
  switch (k) {
    case 1: return launch_t<1, ASYNC>(a, grid, s);
    case 2: return launch_t<2, ASYNC>(a, grid, s);
    case 4: return launch_t<4, ASYNC>(a, grid, s);
    case 8: return launch_t<8, ASYNC>(a, grid, s);
    case 16: return launch_t<16, ASYNC>(a, grid, s);
    case 32: return launch_t<32, ASYNC>(a, grid, s);
    default: return hipErrorInvalidValue;
  }
}

template <bool ASYNC>
static int occ_mode(int k) {
  switch (k) {
    case 1: return occ_t<1, ASYNC>();
    case 2: return occ_t<2, ASYNC>();
    case 4: return occ_t<4, ASYNC>();
    case 8: return occ_t<8, ASYNC>();
    case 16: return occ_t<16, ASYNC>();
    case 32: return occ_t<32, ASYNC>();
    default: return 1;
  }
}

hipError_t launch_move(int k, bool async_mode, const MoveArgs &a, int grid, hipStream_t s) {
  return async_mode ? launch_mode<true>(k, a, grid, s) : launch_mode<false>(k, a, grid, s);
}

int move_blocks_per_cu(int k, bool async_mode) {
  return async_mode ? occ_mode<true>(k) : occ_mode<false>(k);
}

}  // namespace lpa
