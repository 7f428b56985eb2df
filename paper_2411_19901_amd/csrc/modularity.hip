// Modularity of a labelling (paper Eq. 1, community-sum form) in fp64:
//   2m      = sum of the CSR weights,
//   sigma   = weight of the CSR entries whose two endpoints share a label
//             (both directions of every edge),
//   Sigma_c = sum of K_i over the vertices labelled c,
//   Q       = sigma / 2m - sum_c (Sigma_c / 2m)^2.
// k_modularity accumulates 2m and sigma and scatters K_i into Sigma_c; the
// square sum is taken by a second pass over Sigma (in capi.hip).
//
// Same decomposition as the move kernels: vertices above the binning
// threshold are read by one wavefront each (coalesced), the others one lane
// per row with the rows staged through LDS so the wavefront's loads are
// row-contiguous.  The labels are only read, so no ordering is needed.
#include "lpa_internal.h"
#include "wave.h"

namespace lpa {
namespace {

// tot[c] += x for every lane where `on` holds.  The lanes that share the
// lowest active lane's label are summed across the wavefront and added
// with one atomic (a converged labelling often gives most of a wavefront's
// vertices one community, whose atomics on one address would serialise);
// the other lanes are summed per run of consecutive lanes with one label
// (vertices close in the degree order are often neighbours, so a label
// tends to come in runs) and each run's first lane adds its sum.
__device__ void add_by_label(double *tot, int c, double x, bool on) {
  const int lane = threadIdx.x & (kWave - 1);
  unsigned long long rest = __ballot(on);
  if (!rest) return;
  {
    const int src = __ffsll((long long)rest) - 1;
    const int cs = rl(c, src);
    const bool grp = on && c == cs;
    const unsigned long long gm = __ballot(grp);
    if (gm & (gm - 1)) {  // two or more lanes
      const double s = wave_sum_d(grp ? x : 0.0);
      if (lane == src) atomicAdd(&tot[cs], s);
      rest &= ~gm;
    }
  }
  if (!rest) return;
  // runs: a lane in `rest` continues the run of the lane below it when
  // that lane is in `rest` with the same label; rid = the lane where the
  // run starts (lanes outside `rest` carry 0 and join the run below them)
  const bool mine = (rest >> lane) & 1ull;
  const int cp = __shfl_up(c, 1);
  const bool cont = lane > 0 && ((rest >> (lane - 1)) & 1ull) && cp == c;
  const unsigned long long heads = __ballot(mine && !cont);
  const unsigned long long below = lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull);
  const int rid = 63 - __clzll(heads & below);
  double v = mine ? x : 0.0;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const double y = __shfl_down(v, off);
    const int ro = __shfl_down(rid, off);
    if (lane + off < kWave && ro == rid) v += y;
  }
  if (mine && !cont) atomicAdd(&tot[c], v);
}

// One step of TW entries per row (TW <= T), as in the move kernel's
// staging: adds matching weights to `in` and stages the weights for the
// row owners' K_i sums.  Slots are taken kModBatch at a time, column loads,
// then weights, then labels, so that each phase's loads are in flight
// together (slots past a row's end issue no load).
constexpr int kModBatch = 4;

template <int TW, int T>
__device__ __forceinline__ void mod_step(const ModArgs &m, Stage<T, long long> &st, int lane, int t0,
                                         int tn, double &ki, double &in) {
  const gptr<const int32_t> col = as_global(m.col);
  const gptr<const float> wp = as_global(m.w);
  const gptr<const int32_t> lab = as_global(m.lab);
  constexpr int B = TW < kModBatch ? TW : kModBatch;
#pragma unroll
  for (int i0 = 0; i0 < TW; i0 += B) {
    bool ok[B];
    int c[B], l[B];
    float x[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int slot = (i0 + b) * kWave + lane;
      const int r = slot / TW, j = slot % TW;
      ok[b] = t0 + j < st.len[r];
      c[b] = ok[b] ? __builtin_nontemporal_load(col + (st.beg[r] + (t0 + j))) : -1;
    }
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int slot = (i0 + b) * kWave + lane;
      const int r = slot / TW, j = slot % TW;
      x[b] = !ok[b] ? 0.0f : (wp ? __builtin_nontemporal_load(wp + (st.beg[r] + (t0 + j))) : 1.0f);
    }
#pragma unroll
    for (int b = 0; b < B; ++b) l[b] = ok[b] ? lab[c[b]] : -1;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int slot = (i0 + b) * kWave + lane;
      const int r = slot / TW, j = slot % TW;
      if (ok[b] && l[b] == st.self[r]) in += (double)x[b];
      st.w[r * (TW + 1) + j] = x[b];
    }
  }
  wave_lds_sync();
  if (m.w) {
#pragma unroll
    for (int j = 0; j < TW; ++j)
      if (j < tn) ki += (double)st.w[lane * (TW + 1) + j];
  }
  wave_lds_sync();
}

// One lane per row: entries [beg, beg + len) of vertex v at degree-order
// position p (v < 0: none).
template <int T>
__device__ void mod_lane_rows(const ModArgs &m, Stage<T, long long> &st, int lane, int p, int v,
                              double &k_acc, double &in_acc) {
  long long beg = 0;
  int len = 0, ci = -1;
  if (v >= 0) {
    ci = m.lab[m.ranked ? p : v];
    beg = m.row_ptr[v];
    len = (int)(m.row_ptr[v + 1] - beg);
  }
  st.beg[lane] = beg;
  st.len[lane] = len;
  st.self[lane] = ci;
  const int maxlen = rfl(wave_max(len));
  wave_lds_sync();
  double ki = 0.0, in = 0.0;
  for (int t0 = 0; t0 < maxlen;) {
    const int rem = maxlen - t0;
    if (rem <= 4) {
      mod_step<4>(m, st, lane, t0, rem, ki, in);
      t0 += 4;
    } else if (rem <= 8) {
      mod_step<8>(m, st, lane, t0, rem, ki, in);
      t0 += 8;
    } else {
      mod_step<T>(m, st, lane, t0, min(T, rem), ki, in);
      t0 += T;
    }
  }
  if (!m.w) ki = (double)len;
  k_acc += ki;
  in_acc += in;
  add_by_label(m.tot, ci, ki, v >= 0 && len > 0);
}

// One wavefront per hub segment: entries [rb, re) of the row of vertex v
// at degree-order position p; (pc, ps) is this wavefront's pending
// contribution to Sigma_pc, flushed when the label changes.
__device__ void mod_hub(const ModArgs &m, int p, int v, long long rb, long long re,
                        double &k_acc, double &in_acc, int &pc, double &ps) {
  const int lane = threadIdx.x & (kWave - 1);
  const gptr<const int32_t> col = as_global(m.col);
  const gptr<const float> wp = as_global(m.w);
  const gptr<const int32_t> lab = as_global(m.lab);
  const int ci = lab[m.ranked ? p : v];
  constexpr int U = 4;
  double ki = 0.0, in = 0.0;
  for (long long e0 = rb; e0 < re; e0 += U * kWave) {
    int c[U];
    float x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long e = e0 + u * kWave + lane;
      c[u] = e < re ? __builtin_nontemporal_load(col + e) : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long e = e0 + u * kWave + lane;
      x[u] = e >= re ? 0.0f : (wp ? __builtin_nontemporal_load(wp + e) : 1.0f);
    }
    int l[U];
#pragma unroll
    for (int u = 0; u < U; ++u) l[u] = c[u] >= 0 ? lab[c[u]] : -1;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ki += (double)x[u];
      if (l[u] == ci) in += (double)x[u];
    }
  }
  k_acc += ki;
  in_acc += in;
  const double kv = wave_sum_d(ki);
  if (ci != pc) {
    if (pc >= 0 && lane == 0) atomicAdd(&m.tot[pc], ps);
    pc = ci;
    ps = 0.0;
  }
  ps += kv;
}

// Short rows (degree 1 .. kShortDeg, the last n_short lane vertices): each
// lane reads its own kShortRows rows, with no stage, their column indices,
// weights and labels loaded phase by phase, as the move kernels' short units
// do; such rows are bound by their dependent loads, not by bandwidth.
// q0: index of the first row among the short ones.
__device__ void mod_short_rows(const ModArgs &m, int q0, double &k_acc, double &in_acc) {
  constexpr int R = kShortRows, D = kShortDeg;
  const int lane = threadIdx.x & (kWave - 1);
  const int p0 = m.n_hubs + m.n_lane - m.n_short;
  const gptr<const int32_t> col = as_global(m.col);
  const gptr<const float> wp = as_global(m.w);
  const gptr<const int32_t> lab = as_global(m.lab);
  int v[R], ci[R], len[R];
  long long beg[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int q = q0 + r * kWave + lane;
    v[r] = q < m.n_short ? m.order[p0 + q] : -1;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int q = q0 + r * kWave + lane;
    ci[r] = v[r] >= 0 ? lab[m.ranked ? p0 + q : v[r]] : -1;
    beg[r] = v[r] >= 0 ? m.row_ptr[v[r]] : 0;
    len[r] = v[r] >= 0 ? (int)(m.row_ptr[v[r] + 1] - beg[r]) : 0;
  }
  int c[R][D], l[R][D];
  float x[R][D];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < D; ++j)
      c[r][j] = j < len[r] ? __builtin_nontemporal_load(col + (beg[r] + j)) : -1;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < D; ++j)
      x[r][j] = j < len[r] ? (wp ? __builtin_nontemporal_load(wp + (beg[r] + j)) : 1.0f) : 0.0f;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < D; ++j) l[r][j] = c[r][j] >= 0 ? lab[c[r][j]] : -1;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    double ki = 0.0, in = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
      if (j < len[r]) {
        ki += (double)x[r][j];
        if (l[r][j] == ci[r]) in += (double)x[r][j];
      }
    }
    k_acc += ki;
    in_acc += in;
    add_by_label(m.tot, ci[r], ki, v[r] >= 0 && len[r] > 0);
  }
}

__global__ __launch_bounds__(kBlock) void k_modularity(ModArgs m) {
  __shared__ Stage<kStageT, long long> stage[kBlock / kWave];  // 64-bit row positions
  const int lane = threadIdx.x & (kWave - 1);
  const int wib = rfl(threadIdx.x / kWave);
  const int wave = rfl(blockIdx.x * (kBlock / kWave) + wib);
  const int nwaves = gridDim.x * (kBlock / kWave);
  // hub items: one per segment, or one per whole hub without segments
  const int hub_items = m.n_seg > 0 ? m.n_seg : m.n_hubs;
  const int lane_rows = m.n_lane - m.n_short;  // staged lane rows, then the short ones
  const int row_items = (lane_rows + kWave - 1) / kWave;
  const int items = hub_items + (int)lane_items(m.n_lane, m.n_short);
  double k_acc = 0.0, in_acc = 0.0, ps = 0.0;
  int pc = -1;
  for (int item = wave; item < items; item += nwaves) {
    if (item < hub_items) {
      int h = item;
      long long q = 0;
      if (m.n_seg > 0) {
        h = m.seg_hub[item];
        q = item - m.hub_pbase[h];
      }
      const int v = m.order[h];
      const long long rb = m.row_ptr[v], re = m.row_ptr[v + 1];
      const long long b = m.n_seg > 0 ? rb + q * m.seg_len : rb;
      const long long e = m.n_seg > 0 ? min(b + (long long)m.seg_len, re) : re;
      mod_hub(m, h, v, b, e, k_acc, in_acc, pc, ps);
    } else if (item - hub_items < row_items) {
      const int u = (item - hub_items) * kWave + lane;
      const int v = u < lane_rows ? m.order[m.n_hubs + u] : -1;
      mod_lane_rows<kStageT>(m, stage[wib], lane, m.n_hubs + u, v, k_acc, in_acc);
    } else {
      mod_short_rows(m, (item - hub_items - row_items) * (kWave * kShortRows), k_acc, in_acc);
    }
  }
  if (pc >= 0 && lane == 0) atomicAdd(&m.tot[pc], ps);
  // one pair of atomics per workgroup: atomics on the two accumulators
  // serialise, so the workgroup sums its wavefronts' parts first
  __shared__ double part[2][kBlock / kWave];
  k_acc = wave_sum_d(k_acc);
  in_acc = wave_sum_d(in_acc);
  if (lane == 0) {
    part[0][wib] = k_acc;
    part[1][wib] = in_acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a0 = 0.0, a1 = 0.0;
    for (int w = 0; w < kBlock / kWave; ++w) {
      a0 += part[0][w];
      a1 += part[1][w];
    }
    atomicAdd(&m.acc[0], a0);
    atomicAdd(&m.acc[1], a1);
  }
}

}  // namespace

hipError_t launch_modularity(const ModArgs &m, int grid, hipStream_t s) {
  if (m.n_hubs + m.n_lane > 0)
    hipLaunchKernelGGL(k_modularity, dim3(grid > 0 ? grid : 1), dim3(kBlock), 0, s, m);
  return hipGetLastError();
}

int modularity_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, (const void *)k_modularity, kBlock, 0) !=
      hipSuccess)
    return 1;
  return nb > 0 ? nb : 1;
}

}  // namespace lpa
