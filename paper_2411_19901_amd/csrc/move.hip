// lpaMove kernels for gfx950 (paper Algorithm 1, lpaMove; Algorithm 2,
// sketchAccumulate; Sections 4.1-4.5).
//
// Work decomposition (fixed once per graph by the degree binning):
//   * a "unit" is a run of at most S consecutive CSR entries of one vertex;
//     vertices of degree <= S are one unit, vertices above S ("hubs") are
//     split into ceil(deg / S) segment units;
//   * one lane owns one unit and feeds its entries into a register sketch in
//     CSR order, so no sketch merging is needed below S;
//   * a wavefront takes 64 units at a time (units are ordered by decreasing
//     length, so its lanes finish together) and stages T entries of each of
//     its 64 rows through LDS per step: the column, weight and gathered label
//     loads are issued row-contiguous by the whole wavefront, then every
//     lane consumes its own row from LDS;
//   * LPA_MODE_ASYNC: segment sketches are written out as partial sketches
//     and merged per hub by k_hub_merge (Section 4.3, partial sketches);
//     labels and flags are updated in place;
//   * LPA_MODE_DET: vertices above S are scanned by one wavefront each, which
//     stages 64 entries at a time and feeds them one by one into a sketch
//     held one slot per lane, so every sketch sees its row in CSR order;
//     labels are double-buffered (Jacobi).
//
// The CSR arrays are streamed once per iteration with non-temporal loads so
// that they do not evict the label lines that the gathers reuse.
//
// Sketch step (Section 4.1, with the decrement reading used throughout the
// library): a pair (c, w) adds w to the slot holding c; otherwise it fills a
// free slot (value 0); otherwise every slot loses d = min(w, smallest slot)
// and the residue w - d, if positive, fills a slot that became free.  Keys
// left behind in free slots may still match c: adding w to a free slot that
// holds c gives the same multiset of live (label, weight) pairs as placing
// (c, w) in any free slot, and keys stay unique because a key is only
// written when c is in no slot.  A weight of 0 leaves the sketch unchanged,
// which is how self-loops and padding are skipped without a branch.
#include "lpa_internal.h"
#include "wave.h"

#include <limits.h>
#include <math.h>

#include <type_traits>

namespace lpa {


// Row offset v of a graph as position type Pos: int reads the int32 offsets
// (graphs of fewer than 2^31 entries); long long reads either width.
template <class Pos>
__device__ __forceinline__ Pos row_at(const RowPtr &rp, int v) {
  if constexpr (sizeof(Pos) == 8)
    return rp[v];
  else
    return as_global(rp.p32)[v];
}

// Index of the labels and flags of the vertex at degree-order position p
// (id v): its id, or its position when the graph keeps its state ranked.
// The same index is what `col` holds for the vertex, so a row entry equal to
// it is the vertex itself.
__device__ __forceinline__ int state_at(const MoveArgs &a, int p, int v) { return a.ranked ? p : v; }

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

  // Feed another sketch's live slots (merge of partial sketches).
  __device__ __forceinline__ void merge_from(const int *pk, const float *pv) {
#pragma unroll
    for (int s = 0; s < K; ++s) add(pk[s], pv[s] > 0.0f ? pv[s] : 0.0f);
  }
};

// ---------------------------------------------------------------------------
// The weighted Boyer-Moore vote of Algorithm 3 (nu-BM-LPA): one candidate
// (key, val).  A pair (c, w) adds w when c is the candidate, subtracts w when
// the candidate's weight is larger, and otherwise becomes the candidate.
// The paper starts the candidate at (C[i], 0); starting at (-1, 0) gives the
// same result: from weight 0 the first positive pair becomes (c, w) either
// way, a zero-weight pair leaves a weight-0 candidate empty in effect, and
// a positive weight never returns to 0 (val > w implies val - w > 0 with
// denormals kept).  So an empty vote keeps the current label.
// Selected by K = 0 in the kernels below.
// ---------------------------------------------------------------------------
struct BmSketch {
  int key[1];
  float val[1];

  __device__ __forceinline__ void clear() {
    key[0] = -1;
    val[0] = 0.0f;
  }

  __device__ __forceinline__ void add(int c, float w) {
    const bool same = key[0] == c;
    const bool down = !same && val[0] > w;
    val[0] = same ? val[0] + w : (down ? val[0] - w : w);
    key[0] = (same || down) ? key[0] : c;
  }

  __device__ __forceinline__ int max_key(int keep) const { return val[0] > 0.0f ? key[0] : keep; }

  // Partial votes of one hub combine by the largest weight (ties to the
  // lowest label), as the paper's pair-max block reduction does.
  __device__ __forceinline__ void merge_from(const int *pk, const float *pv) {
    const bool better = pv[0] > val[0] || (pv[0] == val[0] && pv[0] > 0.0f && pk[0] < key[0]);
    key[0] = better ? pk[0] : key[0];
    val[0] = better ? pv[0] : val[0];
  }
};

template <int K>
struct SketchOf {
  using type = LaneSketch<K>;
};
template <>
struct SketchOf<0> {
  using type = BmSketch;
};
// Slots stored per partial sketch.
constexpr int slots_of(int K) { return K == 0 ? 1 : K; }

// Load one staging step of TW entries for each of the 64 rows (TW <= T):
// slot i * 64 + lane holds entry t0 + j of row r, (r, j) = (slot / TW,
// slot % TW), stored at r * (TW + 1) + j.  The slots are taken kLoadBatch
// at a time in three phases (column indices, weights, gathered labels), so
// that each phase's loads are in flight together; a slot past its row's end
// issues no load and is stored as padding (label -1, weight 0).  A step of
// TW <= T / 2 leaves lab[] words 64 (TW + 1) onwards unused: with KEEP, slot
// s's column index is kept at kept_col<TW>(s) there, for the marking pass.
constexpr int kLoadBatch = 4;

template <int TW>
__device__ __forceinline__ int kept_col(int slot) { return kWave * (TW + 1) + slot; }

template <int TW, bool KEEP, int T, class Pos>
__device__ __forceinline__ void stage_load(const MoveArgs &a, Stage<T, Pos> &st, int lane, int t0) {
  constexpr int B = TW < kLoadBatch ? TW : kLoadBatch;
#pragma unroll
  for (int i0 = 0; i0 < TW; i0 += B) {
    bool ok[B];
    Pos e[B];
    int c[B], lab[B];
    float x[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int slot = (i0 + b) * kWave + lane;
      const int r = slot / TW, j = slot % TW;
      ok[b] = t0 + j < st.len[r];
      e[b] = st.beg[r] + (t0 + j);
    }
#pragma unroll
    for (int b = 0; b < B; ++b) c[b] = ok[b] ? __builtin_nontemporal_load(a.col + e[b]) : -1;
#pragma unroll
    for (int b = 0; b < B; ++b)
      x[b] = !ok[b] ? 0.0f : (a.w ? __builtin_nontemporal_load(a.w + e[b]) : 1.0f);
#pragma unroll
    for (int b = 0; b < B; ++b) lab[b] = ok[b] ? a.C[c[b]] : -1;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int slot = (i0 + b) * kWave + lane;
      const int r = slot / TW, j = slot % TW;
      st.lab[r * (TW + 1) + j] = lab[b];
      st.w[r * (TW + 1) + j] = c[b] == st.self[r] ? 0.0f : x[b];
      if constexpr (KEEP && 2 * TW <= T) st.lab[kept_col<TW>(slot)] = c[b];
    }
  }
}

// Feed entries [beg, beg + len) of row `self` to feed(label, weight) in CSR
// order (len = 0: nothing); entries of the vertex itself come with weight 0.
// All lanes of the wavefront must call it together.  Each step takes 4, 8
// or T entries per row, the narrowest that covers what the wavefront's
// longest row has left: with short rows a wide step would leave most load
// slots idle.  With KEEP, returns the step width when every row fit one
// step of width 4 or 8 (the rows' column indices are then kept in the
// stage); otherwise 0.  Keeping them costs registers: only kernels that
// stay within their register budget with it pass KEEP.
template <int T, bool KEEP = false, class Pos, class Feed>
__device__ __forceinline__ int staged_rows(const MoveArgs &a, Stage<T, Pos> &st, int lane, Pos beg,
                                           int len, int self, Feed &&feed) {
  st.beg[lane] = beg;
  st.len[lane] = len;
  st.self[lane] = self;
  const int maxlen = rfl(wave_max(len));
  wave_lds_sync();
  for (int t0 = 0; t0 < maxlen;) {
    const int rem = maxlen - t0;
    const int tw = rem <= 4 ? 4 : (rem <= 8 ? 8 : T);
    if (tw == 4)
      stage_load<4, KEEP>(a, st, lane, t0);
    else if (tw == 8)
      stage_load<8, KEEP>(a, st, lane, t0);
    else
      stage_load<T, KEEP>(a, st, lane, t0);
    wave_lds_sync();
    // this lane's row: its first tn staged entries (later columns of the
    // step are padding for every row: label -1, weight 0)
    const int tn = min(tw, rem);
    const int row = lane * (tw + 1);
    for (int j = 0; j < tn; ++j) feed(st.lab[row + j], st.w[row + j]);
    wave_lds_sync();
    t0 += tw;
  }
  return KEEP && maxlen <= 8 && 16 <= T ? (maxlen <= 4 ? 4 : 8) : 0;
}

// Feed entries [beg, beg + len) of row `self` into S in CSR order (len = 0:
// nothing).  All lanes of the wavefront must call it together.
template <class SK, int T, bool KEEP = false, class Pos>
__device__ __forceinline__ int staged_scan(const MoveArgs &a, Stage<T, Pos> &st, int lane, Pos beg,
                                           int len, int self, SK &S) {
  return staged_rows<T, KEEP>(a, st, lane, beg, len, self, [&](int lab, float x) { S.add(lab, x); });
}

// Double scan (Section 4.4, Algorithm 4 rescan): the live slots of the
// single scan's sketch are the candidates; a second pass in CSR order sums
// each candidate's exact weight, and the heaviest wins (ties to the lowest
// label; no candidate keeps `keep`).
template <int K>
struct Rescan {
  int key[K];  // candidate labels, -1 for slots that were empty
  float acc[K];

  __device__ __forceinline__ void from(const LaneSketch<K> &S) {
#pragma unroll
    for (int s = 0; s < K; ++s) {
      key[s] = S.val[s] > 0.0f ? S.key[s] : -1;
      acc[s] = 0.0f;
    }
  }
  __device__ __forceinline__ void add(int c, float x) {
#pragma unroll
    for (int s = 0; s < K; ++s) acc[s] = (c >= 0 && key[s] == c) ? acc[s] + x : acc[s];
  }
  __device__ __forceinline__ int best(int keep) const {
    int bk = keep;
    float bv = 0.0f;
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const bool better = acc[s] > bv || (acc[s] == bv && acc[s] > 0.0f && key[s] < bk);
      bk = better ? key[s] : bk;
      bv = better ? acc[s] : bv;
    }
    return bk;
  }
};

// Flag a neighbour of a changed vertex as unprocessed (plain byte store:
// reading the flag first to skip repeated marks measured slower).
__device__ __forceinline__ void mark(const MoveArgs &a, int j) { a.act_next[j] = 1; }

// Mark the neighbours of every lane whose `moved` is set (entries [beg, beg +
// len) of its row), with row-contiguous column loads by the whole wavefront:
// all of a step's column loads are issued before its flag stores.
template <int TW, int T, class Pos>
__device__ __forceinline__ void mark_step(const MoveArgs &a, const Stage<T, Pos> &st, int lane,
                                          int t0) {
  bool ok[TW];
  int c[TW];
#pragma unroll
  for (int i = 0; i < TW; ++i) {
    const int slot = i * kWave + lane;
    const int r = slot / TW, j = slot % TW;
    ok[i] = t0 + j < st.len[r];
    c[i] = ok[i] ? __builtin_nontemporal_load(a.col + (st.beg[r] + (t0 + j))) : 0;
  }
#pragma unroll
  for (int i = 0; i < TW; ++i)
    if (ok[i]) mark(a, c[i]);
}

// Mark the neighbours of entries [beg, end) of one row, the whole wavefront
// taking 64 x U entries at a time (loads first, then stores).  The move
// kernels use kMarkUnroll; k_hub_mark, which only marks, takes a whole hub
// segment per step so that one load latency is waited for per segment.
constexpr int kMarkUnroll = 4;

template <int U = kMarkUnroll, class Pos>
__device__ __forceinline__ void mark_row(const MoveArgs &a, Pos beg, Pos end, int lane) {
  for (Pos q0 = beg; q0 < end; q0 += U * kWave) {
    int c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const Pos q = q0 + u * kWave + lane;
      c[u] = q < end ? __builtin_nontemporal_load(a.col + q) : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (c[u] >= 0) mark(a, c[u]);
  }
}

// Mark from the column indices a single scan step of width TW kept in the
// stage: each lane takes the slots it loaded (st.len already holds 0 for
// rows that did not move).
template <int TW, int T, class Pos>
__device__ __forceinline__ void mark_kept(const MoveArgs &a, const Stage<T, Pos> &st, int lane) {
#pragma unroll
  for (int i = 0; i < TW; ++i) {
    const int slot = i * kWave + lane;
    const int r = slot / TW, j = slot % TW;
    if (j < st.len[r]) mark(a, st.lab[kept_col<TW>(slot)]);
  }
}

// Mark the neighbours of every lane whose `moved` is set (entries [beg, beg +
// len) of its row), with row-contiguous column loads by the whole wavefront
// and the same step widths as staged_rows.  kept = the width staged_rows
// returned for these rows (the stage then still holds their column indices
// and nothing is read from the CSR), or 0.
template <int T, class Pos>
__device__ __forceinline__ void staged_mark(const MoveArgs &a, Stage<T, Pos> &st, int lane, Pos beg,
                                            int len, bool moved, int kept) {
  if (__ballot(moved) == 0ull) return;
  st.beg[lane] = beg;
  st.len[lane] = moved ? len : 0;
  const int maxlen = rfl(wave_max(moved ? len : 0));
  wave_lds_sync();
  if (kept == 4) {
    mark_kept<4>(a, st, lane);
    wave_lds_sync();
    return;
  }
  if (kept == 8) {
    mark_kept<8>(a, st, lane);
    wave_lds_sync();
    return;
  }
  for (int t0 = 0; t0 < maxlen;) {
    const int rem = maxlen - t0;
    if (rem <= 4) {
      mark_step<4>(a, st, lane, t0);
      t0 += 4;
    } else if (rem <= 8) {
      mark_step<8>(a, st, lane, t0);
      t0 += 8;
    } else {
      mark_step<T>(a, st, lane, t0);
      t0 += T;
    }
  }
  wave_lds_sync();
}

// ---------------------------------------------------------------------------
// LPA_MODE_DET hub path: one wavefront per vertex, CSR order.
//
// The row is read in super-chunks of kHubDepth x 64 entries (lane t of
// chunk d holds entry base + 64 d + t): the next super-chunk's column,
// weight and label loads are in flight while the current one is consumed,
// so the serial sketch chain is not paced by the gather latency.
// ---------------------------------------------------------------------------
constexpr int kHubDepth = 8;

template <int D>
struct HubChunks {
  int lab[D];
  float x[D];  // 0 for padding and self-loops

  // self: the vertex's own index as its row entries name it.  Column
  // indices, then weights, then labels: no load waits for another of its
  // phase, so each phase's D loads are in flight together (a weight load
  // conditioned on its column index would wait for that index first).
  template <class Pos>
  __device__ __forceinline__ void load(const MoveArgs &a, int self, Pos sb, Pos end, int lane) {
    int c[D];
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const Pos e = sb + d * kWave + lane;
      c[d] = e < end ? __builtin_nontemporal_load(a.col + e) : -1;
    }
    if (a.w) {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const Pos e = sb + d * kWave + lane;
        x[d] = e < end ? __builtin_nontemporal_load(a.w + e) : 0.0f;
      }
    } else {
#pragma unroll
      for (int d = 0; d < D; ++d) x[d] = 1.0f;
    }
#pragma unroll
    for (int d = 0; d < D; ++d) lab[d] = c[d] >= 0 ? a.C[c[d]] : 0;
#pragma unroll
    for (int d = 0; d < D; ++d) x[d] = (c[d] < 0 || c[d] == self) ? 0.0f : x[d];
  }
};

// Call consume(lab, x, cnt) for every 64-entry chunk of [beg, end) in order
// (cnt = entries of the chunk; lanes >= cnt hold padding).
template <class Pos, class Consume>
__device__ __forceinline__ void hub_feed(const MoveArgs &a, int self, Pos beg, Pos end, int lane,
                                         Consume &&consume) {
  // The chain of one hub bounds the whole iteration while the other
  // wavefronts of its SIMD stream short rows: let it issue first.
  __builtin_amdgcn_s_setprio(3);
  HubChunks<kHubDepth> cur, nxt;
  cur.load(a, self, beg, end, lane);
  for (Pos sb = beg; sb < end; sb += kHubDepth * kWave) {
    const Pos nb = sb + kHubDepth * kWave;
    if (nb < end) nxt.load(a, self, nb, end, lane);
#pragma unroll 1
    for (int d = 0; d < kHubDepth; ++d) {
      const Pos base = sb + d * kWave;
      if (base >= end) break;
      consume(cur.lab[0], cur.x[0], (int)min((Pos)kWave, (Pos)(end - base)));
#pragma unroll
      for (int q = 0; q + 1 < kHubDepth; ++q) {
        cur.lab[q] = cur.lab[q + 1];
        cur.x[q] = cur.x[q + 1];
      }
    }
    cur = nxt;
  }
  __builtin_amdgcn_s_setprio(0);
}

// Smallest value of lanes 0..K-1 for K = 16 or 32, in every lane: rotations
// within each 16-lane row, then the two rows' minima for K = 32.  A minimum
// is exact, so the order of the reduction does not matter.  (For k <= 8 the
// K independent lane reads are the shorter chain.)
template <int K>
__device__ __forceinline__ float slot_min(float val, int lane) {
  static_assert(K == 16 || K == 32, "slot_min: 16 or 32 slots");
  float t = lane < K ? val : __int_as_float(0x7f800000);
  t = fminf(t, dpp_f<0x128>(t));  // row_ror:8
  t = fminf(t, dpp_f<0x124>(t));  // row_ror:4
  t = fminf(t, dpp_f<0x122>(t));  // row_ror:2
  t = fminf(t, dpp_f<0x121>(t));  // row_ror:1
  float m = rl_f(t, 0);
  if constexpr (K > 16) m = fminf(m, rl_f(t, 16));
  return m;
}

// Adds the entries `run` (lanes whose label is a key, slot: that key's slot)
// to their slots.  UNIT: every such entry weighs 1 and every slot value is
// an integer below 2^24 (unit weights on a row shorter than 2^24 entries),
// so each slot takes its count of entries at once, exactly the sum that
// adding them one by one in CSR order gives; otherwise one entry at a time
// in lane order, with scalar lane indices and no cross-lane votes.
template <bool UNIT>
__device__ __forceinline__ void add_hits(unsigned long long run, int slot, float x, int lane,
                                         float &val) {
  if constexpr (UNIT) {
    while (run) {
      const int s = rl(slot, __ffsll((long long)run) - 1);
      const unsigned long long ms = __ballot(slot == s) & run;
      run &= ~ms;
      val = (lane == s) ? val + (float)(int)__popcll(ms) : val;
    }
  } else {
    while (run) {
      const int h = __ffsll((long long)run) - 1;
      run &= run - 1;
      const int sh = rl(slot, h);
      const float xh = rl_f(x, h);
      val = (lane == sh) ? val + xh : val;
    }
  }
}

// Iteration 0 from the initial labels on a row without repeated neighbours
// (MoveArgs::fresh_hubs): every entry's label differs from every key (live
// or stale), so every entry takes the step for a new label, and the free
// slots change only here: they are tracked in a scalar mask, with no slot
// lookups and no runs of hits.  The same steps as det_chain, UNIT likewise.
template <int K, bool UNIT, class Pos>
__device__ __forceinline__ void det_fresh(const MoveArgs &a, int x0, Pos beg, Pos end, int lane,
                                          int &key, float &val) {
  unsigned long long z = K >= 64 ? ~0ull : ((1ull << K) - 1ull);  // all slots free
  hub_feed(a, x0, beg, end, lane, [&](int lab, float x, int cnt) {
    unsigned long long pend = __ballot(lane < cnt && x > 0.0f);
    while (pend) {
      const int j = __ffsll((long long)pend) - 1;
      pend &= pend - 1;
      const int c = rl(lab, j);
      float r;
      if constexpr (UNIT) {
        if (z == 0ull) {  // every slot live: each loses 1, the entry is used up
          if (lane < K) val = val - 1.0f;
          z = __ballot(lane < K && val == 0.0f);
          continue;
        }
        r = 1.0f;
      } else {
        const float xw = rl_f(x, j);
        r = xw;
        if (z == 0ull) {  // every slot live: decrement by d = min(w, smallest slot)
          float m = xw;
          if constexpr (K >= 16) {
            m = fminf(m, slot_min<K>(val, lane));
          } else {
#pragma unroll
            for (int s = 0; s < K; ++s) m = fminf(m, rl_f(val, s));
          }
          if (lane < K) val = val - m;
          r = xw - m;
          z = __ballot(lane < K && val == 0.0f);
          if (!(r > 0.0f)) continue;
        }
      }
      const int s = __ffsll((long long)z) - 1;  // the lowest free slot
      z &= z - 1;
      key = (lane == s) ? c : key;  // selects, not a branch on the lane
      val = (lane == s) ? r : val;
    }
  });
}

// The sketch of one hub row in det mode after iteration 0 (see
// hub_vertex_det), lane s < K holding slot s in key / val.  UNIT (see
// add_hits): every slot value is an integer, so when every slot is live
// each holds at least 1 and the entry's decrement, min(1, smallest slot),
// is 1: every slot loses 1 and nothing is left to place.
template <int K, bool UNIT, class Pos>
__device__ __forceinline__ void det_chain(const MoveArgs &a, int x0, Pos beg, Pos end, int lane,
                                          int &key, float &val) {
  hub_feed(a, x0, beg, end, lane, [&](int lab, float x, int cnt) {
    int slot = -1;  // the slot holding this lane's label, if any
#pragma unroll
    for (int s = 0; s < K; ++s) slot = (lab == rl(key, s)) ? s : slot;
    unsigned long long pend = __ballot(lane < cnt && x > 0.0f);
    while (pend) {
      const unsigned long long missm = __ballot(slot < 0) & pend;
      // entries before the first miss only add to existing slots
      const unsigned long long run = missm ? (pend & ((missm & (~missm + 1)) - 1)) : pend;
      pend &= ~run;
      add_hits<UNIT>(run, slot, x, lane, val);
      if (!missm) break;
      const int jm = __ffsll((long long)missm) - 1;
      pend &= ~(1ull << jm);
      const int c = rl(lab, jm);
      unsigned long long z = __ballot(lane < K && val == 0.0f);
      float r;
      if constexpr (UNIT) {
        if (z == 0ull) {  // every slot live: each loses 1, the entry is used up
          if (lane < K) val = val - 1.0f;
          continue;
        }
        r = 1.0f;
      } else {
        const float xw = rl_f(x, jm);
        r = xw;
        if (z == 0ull) {  // every slot live: decrement by d = min(w, smallest slot)
          float m = xw;
          if constexpr (K >= 16) {
            m = fminf(m, slot_min<K>(val, lane));
          } else {
#pragma unroll
            for (int s = 0; s < K; ++s) m = fminf(m, rl_f(val, s));
          }
          if (lane < K) val = val - m;
          r = xw - m;
          z = r > 0.0f ? __ballot(lane < K && val == 0.0f) : 0ull;
        }
      }
      if (z) {  // the (residue of the) pair takes a free slot
        const int s = __ffsll((long long)z) - 1;
        const int old = rl(key, s);
        key = (lane == s) ? c : key;
        val = (lane == s) ? r : val;
        slot = (lab == old) ? -1 : slot;
        slot = (lab == c) ? s : slot;
      }
    }
  });
}

// Double scan: the labels of key (-1: none) re-weighted exactly, each slot's
// entries added in CSR order by the slot's lane (val starts at 0).
template <int K, bool UNIT, class Pos>
__device__ __forceinline__ void det_rescan(const MoveArgs &a, int x0, Pos beg, Pos end, int lane,
                                           const int key, float &val) {
  hub_feed(a, x0, beg, end, lane, [&](int lab, float x, int cnt) {
    int slot = -1;
#pragma unroll
    for (int s = 0; s < K; ++s) slot = (lab == rl(key, s)) ? s : slot;
    add_hits<UNIT>(__ballot(slot >= 0 && lane < cnt && x > 0.0f), slot, x, lane, val);
  });
}

// Lane s < K holds slot s.  For each chunk every lane first finds the slot
// whose key equals its label (at most one: keys are unique).  Entries are
// consumed in lane order: a run of entries whose label is already a key
// only adds weights to those slots (add_hits); the first entry without a
// key takes the full sketch step, after which only the lanes whose label
// was the replaced key or is the new key change their slot.
// p: the vertex's degree-order position.
template <int K, bool RS, class Pos>
__device__ void hub_vertex_det(const MoveArgs &a, int p, unsigned long long &scanned,
                               unsigned long long &changed) {
  const int lane = threadIdx.x & (kWave - 1);
  const int v = a.order[p], x0 = state_at(a, p, v);
  const int cv = a.C[x0];
  if (a.act_cur[x0] == 0) {
    if (lane == 0) a.Cn[x0] = cv;
    return;
  }
  if (lane == 0) a.act_cur[x0] = 0;
  const Pos beg = rfl_as(row_at<Pos>(a.row_ptr, v)), end = rfl_as(row_at<Pos>(a.row_ptr, v + 1));
  int key = -1;
  float val = 0.0f;
  // Unit weights (see add_hits).  The double-scan kernels keep the general
  // chains only: more copies of the chunk loop there put its chunk buffers
  // in scratch memory.
  const bool unit = !RS && !a.w && (long long)(end - beg) < (1ll << 24);
  if (unit) {
    if constexpr (!RS) {
      if (a.fresh_hubs) {
        det_fresh<K, true>(a, x0, beg, end, lane, key, val);
      } else {
        det_chain<K, true>(a, x0, beg, end, lane, key, val);
      }
    }
  } else if (a.fresh_hubs) {
    det_fresh<K, false>(a, x0, beg, end, lane, key, val);
  } else {
    det_chain<K, false>(a, x0, beg, end, lane, key, val);
  }
  if constexpr (RS) {
    // double scan: the live slots' labels are re-weighted exactly, each
    // slot's entries added in CSR order by the slot's lane
    key = val > 0.0f ? key : -1;
    val = 0.0f;
    det_rescan<K, false>(a, x0, beg, end, lane, key, val);
  }
  // heaviest live slot, ties to the lowest label; keep when empty
  int bk = cv;
  float bv = 0.0f;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const float vs = rl_f(val, s);
    const int ks = rl(key, s);
    if (vs > bv || (vs == bv && vs > 0.0f && ks < bk)) {
      bk = ks;
      bv = vs;
    }
  }
  const int c = bk;
  const bool moved = c != cv && (!a.pickless || c < cv);
  if (lane == 0) a.Cn[x0] = moved ? c : cv;
  if (moved) {
    changed += 1;
    mark_row(a, beg, end, lane);
  }
  scanned += (unsigned long long)(end - beg);
}

// LPA_SHARED_VARS: the same slot-per-lane sketch and CSR order as
// hub_vertex_det, with the lanes communicating through shared variables in
// LDS instead of wavefront votes (the shared-variable protocol of Algorithm
// 5 and Section 4.1): per entry, the lane whose slot holds the label
// announces its slot index; if none does, the lanes of empty slots take the
// lowest index with an LDS atomic minimum; if none is empty, the smallest
// slot value is found the same way (non-negative floats order like their
// bit patterns) and every slot is decremented.  Same results as
// hub_vertex_det; one entry at a time, with LDS round trips instead of
// register votes.
template <int K, class Pos>
__device__ void hub_vertex_det_sv(const MoveArgs &a, int p, unsigned long long &scanned,
                                  unsigned long long &changed) {
  __shared__ int sv[kBlock / kWave][2];  // per wavefront: [0] slot index, [1] minimum (bits)
  const int lane = threadIdx.x & (kWave - 1);
  int *has = sv[threadIdx.x / kWave];
  const int v = a.order[p], x0 = state_at(a, p, v);
  const int cv = a.C[x0];
  if (a.act_cur[x0] == 0) {
    if (lane == 0) a.Cn[x0] = cv;
    return;
  }
  if (lane == 0) a.act_cur[x0] = 0;
  const Pos beg = rfl_as(row_at<Pos>(a.row_ptr, v)), end = rfl_as(row_at<Pos>(a.row_ptr, v + 1));
  int key = -1;
  float val = 0.0f;
  auto first_free = [&]() {  // lowest empty slot, K if none
    if (lane == 0) has[0] = K;
    wave_lds_sync();
    if (lane < K && val == 0.0f) atomicMin(&has[0], lane);
    wave_lds_sync();
    const int s = rfl(has[0]);
    wave_lds_sync();
    return s;
  };
  hub_feed(a, x0, beg, end, lane, [&](int lab, float x, int cnt) {
    for (int t = 0; t < cnt; ++t) {
      const int c = rl(lab, t);
      const float w = rl_f(x, t);
      if (!(w > 0.0f)) continue;  // zero weight: no-op (self-loops, padding)
      if (lane == 0) has[0] = -1;
      wave_lds_sync();
      if (lane < K && key == c) has[0] = lane;  // keys are unique: one writer at most
      wave_lds_sync();
      const int hs = rfl(has[0]);
      wave_lds_sync();
      if (hs >= 0) {
        if (lane == hs) val += w;
        continue;
      }
      float r = w;
      int s = first_free();
      if (s == K) {  // every slot live: decrement by d = min(w, smallest slot)
        if (lane == 0) has[1] = __float_as_int(w);
        wave_lds_sync();
        if (lane < K) atomicMin(&has[1], __float_as_int(val));
        wave_lds_sync();
        const float m = __int_as_float(rfl(has[1]));
        wave_lds_sync();
        if (lane < K) val = val - m;
        r = w - m;
        s = r > 0.0f ? first_free() : K;
      }
      if (lane == s) {  // the (residue of the) pair takes the free slot
        key = c;
        val = r;
      }
    }
  });
  // heaviest live slot, ties to the lowest label; keep when empty
  int bk = cv;
  float bv = 0.0f;
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const float vs = rl_f(val, s);
    const int ks = rl(key, s);
    if (vs > bv || (vs == bv && vs > 0.0f && ks < bk)) {
      bk = ks;
      bv = vs;
    }
  }
  const bool moved = bk != cv && (!a.pickless || bk < cv);
  if (lane == 0) a.Cn[x0] = moved ? bk : cv;
  if (moved) {
    changed += 1;
    mark_row(a, beg, end, lane);
  }
  scanned += (unsigned long long)(end - beg);
}

// LPA_MODE_DET hub path for the vote of Algorithm 3: the vote consumes each
// chunk in CSR order through lane reads (every lane holds the same
// candidate).
template <class Pos>
__device__ void hub_vertex_det_bm(const MoveArgs &a, int p, unsigned long long &scanned,
                                  unsigned long long &changed) {
  const int lane = threadIdx.x & (kWave - 1);
  const int v = a.order[p], x0 = state_at(a, p, v);
  const int cv = a.C[x0];
  if (a.act_cur[x0] == 0) {
    if (lane == 0) a.Cn[x0] = cv;
    return;
  }
  if (lane == 0) a.act_cur[x0] = 0;
  const Pos beg = rfl_as(row_at<Pos>(a.row_ptr, v)), end = rfl_as(row_at<Pos>(a.row_ptr, v + 1));
  BmSketch S;
  S.clear();
  hub_feed(a, x0, beg, end, lane, [&](int lab, float x, int cnt) {
    for (int t = 0; t < cnt; ++t) S.add(rl(lab, t), rl_f(x, t));
  });
  const int c = S.max_key(cv);
  const bool moved = c != cv && (!a.pickless || c < cv);
  if (lane == 0) a.Cn[x0] = moved ? c : cv;
  if (moved) {
    changed += 1;
    mark_row(a, beg, end, lane);
  }
  scanned += (unsigned long long)(end - beg);
}

// ---------------------------------------------------------------------------
// Lane units (both modes).  Unit u < n_seg is segment u - hub_pbase[h] of
// hub h = seg_hub[u] (async only); otherwise whole vertex order[n_hubs + u -
// n_seg].
// ---------------------------------------------------------------------------
template <int K, bool ASYNC, bool RS, class Pos, bool KEEP>
__device__ __forceinline__ void lane_units(const MoveArgs &a, Stage<kStageT, Pos> &st, int u,
                                           unsigned long long &scanned,
                                           unsigned long long &changed) {
  const int lane = threadIdx.x & (kWave - 1);
  int v = -1, sx = -1, len = 0, cv = 0, pslot = -1;  // sx: state index of v
  Pos beg = 0;
  bool whole = false, active = false;
  if (ASYNC && u < a.n_seg) {
    const int h = a.seg_hub[u];
    v = a.order[h];
    sx = state_at(a, h, v);
    active = a.hub_act[h] != 0;
    const int q = u - a.hub_pbase[h];
    const Pos rb = row_at<Pos>(a.row_ptr, v), re = row_at<Pos>(a.row_ptr, v + 1);
    beg = rb + (Pos)q * a.seg_len;
    len = (int)min((Pos)a.seg_len, (Pos)(re - beg));
    pslot = u;
  } else if (u < a.n_seg + a.n_lane - a.n_short) {
    const int p = a.n_hubs + (u - a.n_seg);
    v = a.order[p];
    sx = state_at(a, p, v);
    whole = true;
    active = a.act_cur[sx] != 0;
    cv = a.C[sx];
    if (active) {
      a.act_cur[sx] = 0;
      beg = row_at<Pos>(a.row_ptr, v);
      len = (int)(row_at<Pos>(a.row_ptr, v + 1) - beg);
    }
  }
  if (!active) len = 0;
  typename SketchOf<K>::type S;
  S.clear();
  const int kept = staged_scan<typename SketchOf<K>::type, kStageT, KEEP>(a, st, lane, beg, len, sx, S);
  scanned += (unsigned long long)len;
  int c = cv;
  if constexpr (RS) {
    // second pass over whole rows only: hub segments are re-weighted after
    // their sketches are merged (k_hub_rescan)
    Rescan<K> R;
    R.from(S);
    staged_rows<kStageT>(a, st, lane, beg, whole ? len : 0, sx,
                         [&](int lab, float x) { R.add(lab, x); });
    if (whole) c = R.best(cv);
  } else {
    if (whole) c = S.max_key(cv);
  }
  bool moved = false;
  if (pslot >= 0) {
    if (active) {  // partial sketch of one hub segment
      constexpr int P = slots_of(K);
#pragma unroll
      for (int s = 0; s < P; ++s) {
        a.part_key[(size_t)pslot * P + s] = S.key[s];
        a.part_val[(size_t)pslot * P + s] = S.val[s];
      }
    }
  } else if (whole) {
    moved = active && c != cv && (!a.pickless || c < cv);
    if (ASYNC) {
      if (moved) a.C[sx] = c;
    } else {
      a.Cn[sx] = moved ? c : cv;
    }
  }
  // every lane reaches here: the marking pass is wavefront-cooperative
  changed += (unsigned long long)__popcll(__ballot(moved));
  staged_mark<kStageT>(a, st, lane, beg, len, moved, kept);
}

// ---------------------------------------------------------------------------
// Short units (both modes, single scan): the last n_short lane vertices,
// whose rows have at most kShortDeg entries.  A wavefront takes kShortRows x
// 64 of them and every lane reads its own kShortRows rows, with no LDS stage:
// the rows' offsets, then all their column indices, weights and labels are
// loaded phase by phase before any sketch step.  Such rows cost little
// bandwidth but four dependent loads each (vertex id, row offsets, columns,
// labels), so a wavefront that waits for two rows per lane at a time keeps
// twice the loads of a staged lane unit in flight.  Each row's entries feed
// its sketch in CSR order with the same weights as in lane_units (the stage's
// padding entries after a row's end are no-ops there), so det results are
// the same.
// q0: index of the unit's first vertex among the short vertices.
// ---------------------------------------------------------------------------
template <int K, bool ASYNC, class Pos>
__device__ __forceinline__ void short_units(const MoveArgs &a, int q0, unsigned long long &scanned,
                                            unsigned long long &changed) {
  constexpr int R = kShortRows, D = kShortDeg;
  const int lane = threadIdx.x & (kWave - 1);
  const int p0 = a.n_hubs + a.n_lane - a.n_short;  // degree-order position of the first one
  int v[R], sx[R], cv[R], len[R];
  bool act[R];
  Pos beg[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int q = q0 + r * kWave + lane;
    v[r] = q < a.n_short ? a.order[p0 + q] : -1;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int q = q0 + r * kWave + lane;
    sx[r] = v[r] >= 0 ? state_at(a, p0 + q, v[r]) : -1;
    act[r] = sx[r] >= 0 && a.act_cur[sx[r]] != 0;
    cv[r] = sx[r] >= 0 ? a.C[sx[r]] : 0;
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    beg[r] = 0;
    len[r] = 0;
    if (act[r]) {
      a.act_cur[sx[r]] = 0;
      beg[r] = row_at<Pos>(a.row_ptr, v[r]);
      len[r] = (int)(row_at<Pos>(a.row_ptr, v[r] + 1) - beg[r]);
    }
  }
  int c[R][D], lab[R][D];
  float x[R][D];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < D; ++j)
      c[r][j] = j < len[r] ? __builtin_nontemporal_load(a.col + (beg[r] + j)) : -1;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < D; ++j)
      x[r][j] = j < len[r] ? (a.w ? __builtin_nontemporal_load(a.w + (beg[r] + j)) : 1.0f) : 0.0f;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int j = 0; j < D; ++j) lab[r][j] = c[r][j] >= 0 ? a.C[c[r][j]] : -1;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    typename SketchOf<K>::type S;
    S.clear();
#pragma unroll
    for (int j = 0; j < D; ++j)
      if (j < len[r]) S.add(lab[r][j], c[r][j] == sx[r] ? 0.0f : x[r][j]);
    const int ch = S.max_key(cv[r]);
    const bool moved = act[r] && ch != cv[r] && (!a.pickless || ch < cv[r]);
    if (sx[r] >= 0) {
      if (ASYNC) {
        if (moved) a.C[sx[r]] = ch;
      } else {
        a.Cn[sx[r]] = moved ? ch : cv[r];
      }
    }
    changed += (unsigned long long)__popcll(__ballot(moved));
    scanned += (unsigned long long)len[r];
    if (moved) {
#pragma unroll
      for (int j = 0; j < D; ++j)
        if (j < len[r]) mark(a, c[r][j]);
    }
  }
}

// ---------------------------------------------------------------------------
// Multi-graph launches.  Work items of all graphs of a launch are numbered
// consecutively; prefix[g] is the first item of graph g.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int find_graph(const int32_t *prefix_, int G, int item) {
  const kptr<int32_t> prefix = as_const(prefix_);
  int lo = 0, hi = G;  // prefix[lo] <= item < prefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= item)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Status of graph g for the kernels other than the stop test (k_finish, the
// only writer, runs in a launch of its own), through the scalar cache.
__device__ __forceinline__ kptr<GraphStatus> status_of(const Launch &L, int g) {
  return as_const(as_const(L.d)[g].st);
}

// Descriptor of graph g, through the scalar cache (the table is written
// only by the host, before the launches).
using DescRef = const GraphDesc LPA_CONST &;
__device__ __forceinline__ DescRef desc_of(const Launch &L, int g) { return as_const(L.d)[g]; }

__device__ __forceinline__ MoveArgs make_args(DescRef d, int iter) {
  MoveArgs a;
  a.n = d.n;
  a.row_ptr.p32 = d.row_ptr.p32;
  a.row_ptr.p64 = d.row_ptr.p64;
  a.col = as_global(d.col);
  a.w = as_global(d.w);
  a.C = as_global(d.C[iter & 1]);
  a.Cn = as_global(d.C[(iter + 1) & 1]);
  a.act_cur = as_global(d.act[iter & 1]);
  a.act_next = as_global(d.act[(iter + 1) & 1]);
  a.order = as_global(d.order);
  a.ranked = d.ranked;
  a.n_hubs = d.n_hubs;
  a.n_lane = d.n_lane;
  a.n_short = d.n_short;
  a.seg_len = d.seg_len;
  a.n_seg = d.hub_shared ? 0 : d.n_seg;  // shared hubs: no segment units in k_move
  a.seg_hub = as_global(d.seg_hub);
  a.hub_pbase = as_global(d.hub_pbase);
  a.hub_act = as_global(d.hub_act);
  a.part_key = as_global(d.part_key);
  a.part_val = as_global(d.part_val);
  a.iter = iter;
  a.pickless = (d.rho > 0 && iter % d.rho == 0) ? 1 : 0;
  a.fresh_hubs = (iter == 0 && d.hub_rows_distinct && as_const(d.st)->fresh) ? 1 : 0;
  return a;
}

// Add a wavefront's per-graph totals to the graph's counters (all lanes
// call it together).
__device__ __forceinline__ void flush_counts(unsigned long long *dN, unsigned long long *sc,
                                             unsigned long long &scanned_lane,
                                             unsigned long long &scanned_w,
                                             unsigned long long &changed_w) {
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) scanned_lane += __shfl_xor(scanned_lane, off);
  if ((threadIdx.x & (kWave - 1)) == 0 && dN) {
    const unsigned long long t = scanned_lane + scanned_w;
    if (t) atomicAdd(sc, t);
    if (changed_w) atomicAdd(dN, changed_w);
  }
  scanned_lane = scanned_w = changed_w = 0;
}

// The last flush of a launch: every wavefront ends at once, and atomics on
// one counter serialise, so the workgroup's wavefronts combine their counts
// per counter (those that ended on the same graph) and one lane adds each
// sum.  Every thread of the workgroup must call it.
__device__ __forceinline__ void flush_last_counts(unsigned long long *dN, unsigned long long *sc,
                                                  unsigned long long &scanned_lane,
                                                  unsigned long long &scanned_w,
                                                  unsigned long long &changed_w, int wib) {
  constexpr int NW = kBlock / kWave;
  __shared__ unsigned long long *f_dN[NW], *f_sc[NW];
  __shared__ unsigned long long f_changed[NW], f_scanned[NW];
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) scanned_lane += __shfl_xor(scanned_lane, off);
  if ((threadIdx.x & (kWave - 1)) == 0) {
    f_dN[wib] = dN;
    f_sc[wib] = sc;
    f_changed[wib] = changed_w;
    f_scanned[wib] = scanned_lane + scanned_w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < NW; ++w) {
      if (!f_dN[w]) continue;
      unsigned long long c = f_changed[w], t = f_scanned[w];
      for (int u = w + 1; u < NW; ++u)
        if (f_dN[u] == f_dN[w]) {  // the same graph and iteration: the same two counters
          c += f_changed[u];
          t += f_scanned[u];
          f_dN[u] = nullptr;
        }
      if (t) atomicAdd(f_sc[w], t);
      if (c) atomicAdd(f_dN[w], c);
    }
  }
  scanned_lane = scanned_w = changed_w = 0;
}

// Lane units keep narrow rows' column indices in the stage for marking
// (staged_rows) only in the kernels whose wavefronts per SIMD it leaves
// unchanged: single scan, sketch votes, 32-bit positions (k <= 8 stays
// within 128 registers, k = 16 within 168, k = 32 within 256).  In the
// 64-bit, double-scan and shared-variable kernels the extra registers would
// cost a wavefront per SIMD, which the gathers need more.
template <int K, bool RS, class Pos, bool SV>
constexpr bool kKeepCols = !RS && !SV && sizeof(Pos) == 4;

template <int K, bool ASYNC, bool RS, class Pos, bool SV = false>
__device__ __forceinline__ void move_body(const Launch &L) {
  __shared__ Stage<kStageT, Pos> stage[kBlock / kWave];
  const int lane = threadIdx.x & (kWave - 1);
  const int wib = rfl(threadIdx.x / kWave);
  const int wave = rfl(blockIdx.x * (kBlock / kWave) + wib);
  const int nwaves = gridDim.x * (kBlock / kWave);
  unsigned long long scanned_lane = 0, changed_w = 0, scanned_w = 0;
  int cur = -1;
  unsigned long long *cdN = nullptr, *csc = nullptr;
  for (int item = wave; item < L.total_items; item += nwaves) {
    const int g = rfl(find_graph(L.prefix_items, L.G, item));
    const kptr<GraphStatus> st = status_of(L, g);
    if (st->done) continue;
    const int iter = st->iter;
    DescRef d = desc_of(L, g);
    if (g != cur) {
      flush_counts(cdN, csc, scanned_lane, scanned_w, changed_w);
      cur = g;
      cdN = d.dN + iter;
      csc = d.scanned + iter;
    }
    const MoveArgs a = make_args(d, iter);
    const int local = item - as_const(L.prefix_items)[g];
    // det mode: one wavefront per hub first; async mode has none (its hubs
    // are cut into segments, which are lane units), so the async kernels
    // carry no hub-chain code
    int hub_items = 0;
    if constexpr (!ASYNC) {
      hub_items = a.n_hubs;
      if (local < hub_items) {
        if constexpr (K == 0)
          hub_vertex_det_bm<Pos>(a, local, scanned_w, changed_w);
        else if constexpr (SV)
          hub_vertex_det_sv<K, Pos>(a, local, scanned_w, changed_w);
        else
          hub_vertex_det<K, RS, Pos>(a, local, scanned_w, changed_w);
        continue;
      }
    }
    // lane units (hub segments first in async mode, then whole vertices),
    // then the short units
    const int lane_local = local - hub_items;
    const int units = a.n_seg + a.n_lane - a.n_short;
    const int unit_items = (units + kWave - 1) / kWave;
    if constexpr (!RS) {
      if (lane_local >= unit_items) {
        short_units<K, ASYNC, Pos>(a, (lane_local - unit_items) * (kWave * kShortRows),
                                   scanned_lane, changed_w);
        continue;
      }
    }
    lane_units<K, ASYNC, RS, Pos, kKeepCols<K, RS, Pos, SV>>(
        a, stage[wib], lane_local * kWave + lane, scanned_lane, changed_w);
  }
  flush_last_counts(cdN, csc, scanned_lane, scanned_w, changed_w, wib);
}

// CSR positions are int for graphs of fewer than 2^31 entries (W = false),
// long long otherwise (W = true, which also reads int32 offsets): 32-bit
// positions keep one register per staged load address.
template <bool W>
using PosOf = typename std::conditional<W, long long, int>::type;

// One iteration's label moves (single scan) ...  With 32-bit positions the
// kernel is held to 128 registers up to k = 16, which keeps four wavefronts
// per SIMD for the gathers (async k = 16 spills a few registers there and
// still runs 8% faster on R-MAT-24 than with three wavefronts), and to 168
// for k = 32 in det mode (three); the other instantiations are left to the
// compiler.
template <int K, bool ASYNC, bool W>
constexpr int kMoveWaves = W                     ? 1
                           : (K <= 16)           ? 4
                           : (K == 32 && !ASYNC) ? 3
                                                 : 1;

template <int K, bool ASYNC, bool W>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kMoveWaves<K, ASYNC, W>)))
void k_move(Launch L) {
  move_body<K, ASYNC, false, PosOf<W>>(L);
}

// ... and with the double scan (LPA_RESCAN; sketch rule only).
template <int K, bool ASYNC, bool W>
__global__ __launch_bounds__(kBlock) void k_move_rescan(Launch L) {
  move_body<K, ASYNC, true, PosOf<W>>(L);
}

// ... and with shared variables instead of votes in the hub path
// (LPA_SHARED_VARS; LPA_MODE_DET, sketch rule, single scan).
template <int K, bool W>
__global__ __launch_bounds__(kBlock) void k_move_sv(Launch L) {
  move_body<K, false, false, PosOf<W>, true>(L);
}

// ---------------------------------------------------------------------------
// LPA_MODE_ASYNC hub epilogue.
// ---------------------------------------------------------------------------
// Snapshot and clear the unprocessed flags of the hubs before the move
// kernel, so that marks made while their segments are scanned are kept for
// the next iteration.
__global__ void k_hub_snapshot(Launch L) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < L.total_hubs;
       t += gridDim.x * blockDim.x) {
    const int g = find_graph(L.prefix_hubs, L.G, t);
    const GraphDesc &d = L.d[g];
    if (d.st->done) continue;
    const int h = t - L.prefix_hubs[g];
    const int x = d.ranked ? h : d.order[h];
    d.hub_act[h] = d.act[0][x];
    d.act[0][x] = 0;
  }
}

// A hub's decision is recorded in hub_act (its flag snapshot is no longer
// needed once the hub is decided): 1 if its label moved.  k_hub_mark then
// flags the neighbours of moved hubs, one wavefront per hub segment.
__device__ __forceinline__ void record_moved_hub(const MoveArgs &a, int h, bool moved) {
  if (h < a.n_hubs) a.hub_act[h] = moved ? 1 : 0;
}

// Flat feed for k = 8 and 16 with the sketch spread over a hub's four-lane
// group: lane q of the group holds slots P q .. P q + P - 1 (P = k / 4), and
// the group's lanes exchange values with quad permutes (DPP), so one sketch
// update is a few instructions per lane instead of a pass over all k slots.
// Same arithmetic and the same slot rules as LaneSketch<k>: a matching key
// adds the weight; otherwise every slot drops by d = min(w, smallest slot)
// and a positive residue takes the lowest free slot; heaviest slot wins,
// ties to the lowest label.
template <int CTRL>
__device__ __forceinline__ int quad_dpp(int x) {
  return dpp<CTRL>(x);
}
template <int CTRL>
__device__ __forceinline__ float quad_dpp_f(float x) {
  return dpp_f<CTRL>(x);
}
constexpr int kQuadX1 = 0xB1;  // lanes (1, 0, 3, 2) of the quad
constexpr int kQuadX2 = 0x4E;  // lanes (2, 3, 0, 1)

template <int P>
struct QuadSketch {
  int k[P];
  float v[P];
  int s0;  // index of this lane's first slot

  __device__ __forceinline__ void clear(int sub) {
#pragma unroll
    for (int q = 0; q < P; ++q) {
      k[q] = -1;
      v[q] = 0.0f;
    }
    s0 = P * sub;
  }

  __device__ __forceinline__ void add(int c, float w) {
    bool m = false;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      const bool mq = k[q] == c;
      v[q] = mq ? v[q] + w : v[q];
      m = m || mq;
    }
    int hit = m ? 1 : 0;
    hit |= quad_dpp<kQuadX1>(hit);
    hit |= quad_dpp<kQuadX2>(hit);
    if (!hit) {
      float d = w;
#pragma unroll
      for (int q = 0; q < P; ++q) d = fminf(d, v[q]);
      d = fminf(d, quad_dpp_f<kQuadX1>(d));
      d = fminf(d, quad_dpp_f<kQuadX2>(d));
#pragma unroll
      for (int q = 0; q < P; ++q) v[q] = v[q] - d;
      const float r = w - d;
      if (r > 0.0f) {
        int f = 4 * P;  // lowest free slot of the group
#pragma unroll
        for (int q = P - 1; q >= 0; --q) f = v[q] == 0.0f ? s0 + q : f;
        f = min(f, quad_dpp<kQuadX1>(f));
        f = min(f, quad_dpp<kQuadX2>(f));
#pragma unroll
        for (int q = 0; q < P; ++q) {
          if (f == s0 + q) {
            k[q] = c;
            v[q] = r;
          }
        }
      }
    }
  }

  __device__ __forceinline__ int max_key(int keep) const {
    int bk = keep;
    float bv = 0.0f;
#pragma unroll
    for (int q = 0; q < P; ++q) {
      if (v[q] > bv || (v[q] == bv && v[q] > 0.0f && k[q] < bk)) {
        bk = k[q];
        bv = v[q];
      }
    }
    int ok = quad_dpp<kQuadX1>(bk);
    float ov = quad_dpp_f<kQuadX1>(bv);
    if (ov > bv || (ov == bv && ov > 0.0f && ok < bk)) {
      bk = ok;
      bv = ov;
    }
    ok = quad_dpp<kQuadX2>(bk);
    ov = quad_dpp_f<kQuadX2>(bv);
    if (ov > bv || (ov == bv && ov > 0.0f && ok < bk)) {
      bk = ok;
      bv = ov;
    }
    return bk;
  }
};

// Feed the partial held by lane T of the quad (its live slots in slot order)
// into Q; a slot of weight 0 would change nothing and is skipped.
template <int T, int K>
__device__ __forceinline__ void quad_feed_partial(QuadSketch<K / 4> &Q, const int *ck,
                                                  const float *cw) {
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const int kk = quad_dpp<T * 0x55>(ck[s]);
    const float vv = quad_dpp_f<T * 0x55>(cw[s]);
    if (vv > 0.0f) Q.add(kk, vv);
  }
}

// Flat feed of one hub's np <= 64 partials (k = 8 or 16) by its four-lane
// group, segment order; returns the merged sketch's heaviest label (keep cv).
template <int K>
__device__ __forceinline__ int hub_flat_merge(const MoveArgs &a, int p0, int np, int sub, int cv) {
  QuadSketch<K / 4> Q;
  Q.clear(sub);
  int ck[K], nk[K];
  float cw[K], nv[K];
#pragma unroll
  for (int s = 0; s < K; ++s) {
    ck[s] = nk[s] = -1;
    cw[s] = nv[s] = 0.0f;
  }
  if (sub < np) {
#pragma unroll
    for (int s = 0; s < K; ++s) {
      ck[s] = a.part_key[(size_t)(p0 + sub) * K + s];
      cw[s] = a.part_val[(size_t)(p0 + sub) * K + s];
    }
  }
  for (int b = 0; b < np; b += kHubLanes) {
    if (b + kHubLanes + sub < np) {
#pragma unroll
      for (int s = 0; s < K; ++s) {
        nk[s] = a.part_key[(size_t)(p0 + b + kHubLanes + sub) * K + s];
        nv[s] = a.part_val[(size_t)(p0 + b + kHubLanes + sub) * K + s];
      }
    }
    const int nt = min(kHubLanes, np - b);
    quad_feed_partial<0, K>(Q, ck, cw);
    if (nt > 1) quad_feed_partial<1, K>(Q, ck, cw);
    if (nt > 2) quad_feed_partial<2, K>(Q, ck, cw);
    if (nt > 3) quad_feed_partial<3, K>(Q, ck, cw);
#pragma unroll
    for (int s = 0; s < K; ++s) {
      ck[s] = nk[s];
      cw[s] = nv[s];
    }
  }
  return Q.max_key(cv);
}

// Hub taken by lane group `grp` of merge item `it` of a graph with `ni`
// merge items: hubs are dealt out across the items (group j of item i takes
// hub j * ni + i).  The largest hubs sit next to each other in the degree
// order; dealt out, each lands in a wavefront of its own instead of one
// wavefront merging them one after another.
__device__ __forceinline__ int merge_hub(int it, int grp, int ni) { return grp * ni + it; }

__device__ __forceinline__ int merge_items(const Launch &L, int g) {
  return as_const(L.prefix_merge)[g + 1] - as_const(L.prefix_merge)[g];
}

// Merge the partial sketches of every active hub (Section 4.3).  A wavefront
// takes kMergeHubs hubs of one graph (merge_hub), kHubLanes lanes each.  For
// a hub with at most 64 partials the partials are fed one by one, in segment
// order, into a single sketch, which every lane of the group computes alike: lane
// t of the group loads partials t, t + kHubLanes, ... (the next one's loads
// in flight) and hands each over by a lane exchange.  Feeding every partial
// into one sketch follows the paper's merge into the first group's sketch;
// combining already merged sketches pairwise instead measured lower
// modularity.  Larger hubs are merged by the whole wavefront (lane l merges
// partials l, l + 64, ..., then a pairwise exchange across lanes).
// RS = false: the hub takes the merged sketch's heaviest label.  RS = true
// (double scan): the merged sketch's live labels are stored as the hub's
// candidates for k_hub_rescan / k_hub_pick.
template <int K, bool RS>
__device__ __forceinline__ void hub_merge_body(const Launch &L) {
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (kHubLanes - 1);
  const int wave = rfl((blockIdx.x * kBlock + threadIdx.x) / kWave);
  const int nwaves = gridDim.x * (kBlock / kWave);
  unsigned long long changed_w = 0, zero_lane = 0, zero_w = 0;
  int cur = -1;
  unsigned long long *cdN = nullptr;
  using SK = typename SketchOf<K>::type;
  constexpr int P = slots_of(K);
  for (int item = wave; item < L.total_merge; item += nwaves) {
    const int g = rfl(find_graph(L.prefix_merge, L.G, item));
    const kptr<GraphStatus> st = status_of(L, g);
    if (st->done) continue;
    const int iter = st->iter;
    DescRef gd = desc_of(L, g);
    if (g != cur) {
      flush_counts(cdN, cdN, zero_lane, zero_w, changed_w);
      cur = g;
      cdN = gd.dN + iter;
    }
    const MoveArgs a = make_args(gd, iter);
    const int it = item - as_const(L.prefix_merge)[g], ni = rfl(merge_items(L, g));
    const int h = merge_hub(it, lane / kHubLanes, ni);
    int x = -1, p0 = 0, np = 0, cv = 0;  // x: the hub's state index
    bool active = false;
    if (h < a.n_hubs) {
      x = state_at(a, h, a.order[h]);
      active = a.hub_act[h] != 0;
      p0 = a.hub_pbase[h];
      np = a.hub_pbase[h + 1] - p0;
      cv = a.C[x];
    }
    int c = cv;
    const bool small = active && np <= kWave;
    SK S;
    S.clear();
    if constexpr ((K == 8 || K == 16) && !RS) {
      if (small) c = hub_flat_merge<K>(a, p0, np, sub, cv);
    } else if (small) {  // np is the same on every lane of the group
      const int gbase = lane & ~(kHubLanes - 1);
      int ck[P], nk[P];
      float cw[P], nv[P];
#pragma unroll
      for (int s = 0; s < P; ++s) {
        ck[s] = -1;
        cw[s] = 0.0f;
        nk[s] = -1;
        nv[s] = 0.0f;
      }
      if (sub < np) {
#pragma unroll
        for (int s = 0; s < P; ++s) {
          ck[s] = a.part_key[(size_t)(p0 + sub) * P + s];
          cw[s] = a.part_val[(size_t)(p0 + sub) * P + s];
        }
      }
      for (int b = 0; b < np; b += kHubLanes) {
        if (b + kHubLanes + sub < np) {
#pragma unroll
          for (int s = 0; s < P; ++s) {
            nk[s] = a.part_key[(size_t)(p0 + b + kHubLanes + sub) * P + s];
            nv[s] = a.part_val[(size_t)(p0 + b + kHubLanes + sub) * P + s];
          }
        }
        const int nt = min(kHubLanes, np - b);
        for (int t = 0; t < nt; ++t) {
          int pk[P];
          float pv[P];
#pragma unroll
          for (int s = 0; s < P; ++s) {
            pk[s] = __shfl(ck[s], gbase + t);
            pv[s] = __shfl(cw[s], gbase + t);
          }
          S.merge_from(pk, pv);
        }
#pragma unroll
        for (int s = 0; s < P; ++s) {
          ck[s] = nk[s];
          cw[s] = nv[s];
        }
      }
    }
    if (small) {
      if constexpr (RS) {
        if (sub == 0) {
#pragma unroll
          for (int s = 0; s < P; ++s)
            gd.hub_cand[(size_t)h * P + s] = S.val[s] > 0.0f ? S.key[s] : -1;
        }
      } else if constexpr (K != 8 && K != 16) {
        c = S.max_key(cv);
      }
    }
    unsigned long long big = __ballot(active && !small && sub == 0);
    while (big) {
      const int src = __ffsll((long long)big) - 1;
      big &= big - 1;
      const int bp0 = __shfl(p0, src), bnp = __shfl(np, src), bcv = __shfl(cv, src);
      SK B;
      B.clear();
      for (int p = bp0 + lane; p < bp0 + bnp; p += kWave) {
        int pk[P];
        float pv[P];
#pragma unroll
        for (int s = 0; s < P; ++s) {
          pk[s] = a.part_key[(size_t)p * P + s];
          pv[s] = a.part_val[(size_t)p * P + s];
        }
        B.merge_from(pk, pv);
      }
#pragma unroll 1
      for (int off = kWave / 2; off >= 1; off >>= 1) {
        int pk[P];
        float pv[P];
#pragma unroll
        for (int s = 0; s < P; ++s) {  // snapshot the partner before merging
          pk[s] = __shfl_xor(B.key[s], off);
          pv[s] = __shfl_xor(B.val[s], off);
        }
        B.merge_from(pk, pv);
      }
      if constexpr (RS) {
        const int bh = merge_hub(it, src / kHubLanes, ni);
        if (lane == 0) {
#pragma unroll
          for (int s = 0; s < P; ++s)
            gd.hub_cand[(size_t)bh * P + s] = B.val[s] > 0.0f ? B.key[s] : -1;
        }
      } else {
        const int bc = rfl(B.max_key(bcv));
        if (lane / kHubLanes == src / kHubLanes) c = bc;
      }
    }
    if constexpr (!RS) {
      const bool moved = active && c != cv && (!a.pickless || c < cv);
      if (moved && sub == 0) a.C[x] = c;
      changed_w += (unsigned long long)__popcll(__ballot(moved && sub == 0));
      if (sub == 0) record_moved_hub(a, h, moved);
    }
  }
  flush_counts(cdN, cdN, zero_lane, zero_w, changed_w);
}

template <int K>
__global__ __launch_bounds__(kBlock) void k_hub_merge(Launch L) {
  hub_merge_body<K, false>(L);
}

// Double scan, hub candidates: merge the partial sketches into candidates.
template <int K>
__global__ __launch_bounds__(kBlock) void k_hub_cand(Launch L) {
  hub_merge_body<K, true>(L);
}

// Double scan, hub re-weighting: one wavefront per hub segment sums the
// exact weight of each of its hub's candidates over the segment's entries
// (any order: LPA_MODE_ASYNC only) into the segment's partial values.
template <int K>
__global__ __launch_bounds__(kBlock) void k_hub_rescan(Launch L) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = rfl((blockIdx.x * kBlock + threadIdx.x) / kWave);
  const int nwaves = gridDim.x * (kBlock / kWave);
  for (int item = wave; item < L.total_segs; item += nwaves) {
    const int g = rfl(find_graph(L.prefix_segs, L.G, item));
    const kptr<GraphStatus> st = status_of(L, g);
    if (st->done) continue;
    DescRef gd = desc_of(L, g);
    const MoveArgs a = make_args(gd, st->iter);
    const int u = item - as_const(L.prefix_segs)[g];
    const int h = a.seg_hub[u];
    if (a.hub_act[h] == 0) continue;
    const int v = a.order[h], self = state_at(a, h, v);
    const int q = u - a.hub_pbase[h];
    const long long rb = a.row_ptr[v], re = a.row_ptr[v + 1];
    const long long beg = rb + (long long)q * a.seg_len, end = min(beg + a.seg_len, re);
    int cand[K];
    float acc[K];
#pragma unroll
    for (int s = 0; s < K; ++s) {
      cand[s] = gd.hub_cand[(size_t)h * K + s];
      acc[s] = 0.0f;
    }
    constexpr int U = 4;
    for (long long e0 = beg; e0 < end; e0 += U * kWave) {
      int lab[U];
      float x[U];
#pragma unroll
      for (int t = 0; t < U; ++t) {
        const long long e = e0 + t * kWave + lane;
        lab[t] = -1;
        x[t] = 0.0f;
        if (e < end) {
          const int j = __builtin_nontemporal_load(a.col + e);
          x[t] = (j == self) ? 0.0f : (a.w ? __builtin_nontemporal_load(a.w + e) : 1.0f);
          lab[t] = a.C[j];
        }
      }
#pragma unroll
      for (int t = 0; t < U; ++t)
#pragma unroll
        for (int s = 0; s < K; ++s)
          acc[s] = (lab[t] >= 0 && lab[t] == cand[s]) ? acc[s] + x[t] : acc[s];
    }
#pragma unroll
    for (int s = 0; s < K; ++s) {
#pragma unroll
      for (int off = kWave / 2; off >= 1; off >>= 1) acc[s] += __shfl_xor(acc[s], off);
      if (lane == 0) a.part_val[(size_t)u * K + s] = acc[s];
    }
  }
}

// Double scan, hub decision: add up the segments' candidate weights, take
// the heaviest candidate (ties to the lowest label), update the label and
// flag the neighbours.  Same hub-to-lane layout as k_hub_merge (merge_hub).
template <int K>
__global__ __launch_bounds__(kBlock) void k_hub_pick(Launch L) {
  const int lane = threadIdx.x & (kWave - 1);
  const int sub = lane & (kHubLanes - 1);
  const int wave = rfl((blockIdx.x * kBlock + threadIdx.x) / kWave);
  const int nwaves = gridDim.x * (kBlock / kWave);
  unsigned long long changed_w = 0, zero_lane = 0, zero_w = 0;
  int cur = -1;
  unsigned long long *cdN = nullptr;
  for (int item = wave; item < L.total_merge; item += nwaves) {
    const int g = rfl(find_graph(L.prefix_merge, L.G, item));
    const kptr<GraphStatus> st = status_of(L, g);
    if (st->done) continue;
    const int iter = st->iter;
    DescRef gd = desc_of(L, g);
    if (g != cur) {
      flush_counts(cdN, cdN, zero_lane, zero_w, changed_w);
      cur = g;
      cdN = gd.dN + iter;
    }
    const MoveArgs a = make_args(gd, iter);
    const int it = item - as_const(L.prefix_merge)[g], ni = rfl(merge_items(L, g));
    const int h = merge_hub(it, lane / kHubLanes, ni);
    int x = -1, p0 = 0, np = 0, cv = 0;  // x: the hub's state index
    bool active = false;
    if (h < a.n_hubs) {
      x = state_at(a, h, a.order[h]);
      active = a.hub_act[h] != 0;
      p0 = a.hub_pbase[h];
      np = a.hub_pbase[h + 1] - p0;
      cv = a.C[x];
    }
    float tot[K];
#pragma unroll
    for (int s = 0; s < K; ++s) tot[s] = 0.0f;
    const bool small = active && np <= kWave;
    if (small)
      for (int p = p0 + sub; p < p0 + np; p += kHubLanes)
#pragma unroll
        for (int s = 0; s < K; ++s) tot[s] += a.part_val[(size_t)p * K + s];
#pragma unroll
    for (int s = 0; s < K; ++s)  // add up each lane group's sums
#pragma unroll
      for (int off = 1; off < kHubLanes; off <<= 1) tot[s] += __shfl_xor(tot[s], off);
    unsigned long long big = __ballot(active && !small && sub == 0);
    while (big) {
      const int src = __ffsll((long long)big) - 1;
      big &= big - 1;
      const int bp0 = __shfl(p0, src), bnp = __shfl(np, src);
      float t[K];
#pragma unroll
      for (int s = 0; s < K; ++s) t[s] = 0.0f;
      for (int p = bp0 + lane; p < bp0 + bnp; p += kWave)
#pragma unroll
        for (int s = 0; s < K; ++s) t[s] += a.part_val[(size_t)p * K + s];
#pragma unroll
      for (int s = 0; s < K; ++s) {
#pragma unroll
        for (int off = kWave / 2; off >= 1; off >>= 1) t[s] += __shfl_xor(t[s], off);
        tot[s] = (lane / kHubLanes == src / kHubLanes) ? t[s] : tot[s];
      }
    }
    int c = cv;
    if (active) {
      float bv = 0.0f;
#pragma unroll
      for (int s = 0; s < K; ++s) {
        const int ks = gd.hub_cand[(size_t)h * K + s];
        const bool better = ks >= 0 && (tot[s] > bv || (tot[s] == bv && tot[s] > 0.0f && ks < c));
        c = better ? ks : c;
        bv = better ? tot[s] : bv;
      }
    }
    const bool moved = active && c != cv && (!a.pickless || c < cv);
    if (moved && sub == 0) a.C[x] = c;
    changed_w += (unsigned long long)__popcll(__ballot(moved && sub == 0));
    if (sub == 0) record_moved_hub(a, h, moved);
  }
  flush_counts(cdN, cdN, zero_lane, zero_w, changed_w);
}

// Flag the neighbours of every hub that moved in this iteration: one
// wavefront per hub segment, coalesced column loads.
__global__ __launch_bounds__(kBlock) void k_hub_mark(Launch L) {
  const int lane = threadIdx.x & (kWave - 1);
  const int wave = rfl((blockIdx.x * kBlock + threadIdx.x) / kWave);
  const int nwaves = gridDim.x * (kBlock / kWave);
  for (int item = wave; item < L.total_segs; item += nwaves) {
    const int g = rfl(find_graph(L.prefix_segs, L.G, item));
    const kptr<GraphStatus> st = status_of(L, g);
    if (st->done) continue;
    const MoveArgs a = make_args(desc_of(L, g), st->iter);
    const int u = item - as_const(L.prefix_segs)[g];
    const int h = a.seg_hub[u];
    if (a.hub_act[h] == 0) continue;
    const int v = a.order[h];
    const int q = u - a.hub_pbase[h];
    const long long rb = a.row_ptr[v], re = a.row_ptr[v + 1];
    const long long beg = rb + (long long)q * a.seg_len, end = min(beg + a.seg_len, re);
    mark_row<16>(a, beg, end, lane);
  }
}

// LPA_HUB_SHARED (ablation of Section 4.3's partial sketches): one workgroup
// per active hub feeds all of the hub's entries into a single sketch in
// LDS that its 256 threads update concurrently with LDS atomics, in the
// manner of the shared mode of Algorithm 5: add to a matching slot, else
// claim a free slot by compare-and-swap (retry if another thread took it),
// else subtract from every slot (by d = min(w, smallest slot), then place
// the residue).  Updates race, so the sketch is approximate; every retry
// loop is bounded.  The hub then takes the heaviest slot.
template <int K>
__device__ __forceinline__ void shared_add(int *key, float *val, int c, float w) {
  for (int attempt = 0; attempt < 2 * K + 2 && w > 0.0f; ++attempt) {
    int hit = -1, freeslot = -1;
    float seen = 0.0f, m = w;
#pragma unroll
    for (int s = 0; s < K; ++s) {
      const float vs = __hip_atomic_load(&val[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      const int ks = __hip_atomic_load(&key[s], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (ks == c && vs > 0.0f && hit < 0) hit = s;
      if (!(vs > 0.0f) && freeslot < 0) {
        freeslot = s;
        seen = vs;
      }
      m = fminf(m, vs);
    }
    if (hit >= 0) {
      atomicAdd(&val[hit], w);
      return;
    }
    if (freeslot >= 0) {
      const unsigned want = __float_as_uint(seen);
      if (atomicCAS((unsigned *)&val[freeslot], want, __float_as_uint(w)) == want) {
        __hip_atomic_store(&key[freeslot], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        return;
      }
      continue;  // another thread took the slot: look again
    }
    if (m > 0.0f) {
#pragma unroll
      for (int s = 0; s < K; ++s) atomicAdd(&val[s], -m);
    }
    w -= m;  // the residue, if any, looks for a slot that just emptied
  }
}

template <int K>
__global__ __launch_bounds__(256) void k_hub_shared(Launch L) {
  __shared__ int key[K];
  __shared__ float val[K];
  for (int item = blockIdx.x; item < L.total_hubs; item += gridDim.x) {
    const int g = find_graph(L.prefix_hubs, L.G, item);
    const kptr<GraphStatus> st = status_of(L, g);
    if (st->done) continue;
    DescRef gd = desc_of(L, g);
    const MoveArgs a = make_args(gd, st->iter);
    const int h = item - as_const(L.prefix_hubs)[g];
    if (a.hub_act[h] == 0) continue;
    const int v = a.order[h], self = state_at(a, h, v);
    if (threadIdx.x < K) {
      key[threadIdx.x] = -1;
      val[threadIdx.x] = 0.0f;
    }
    __syncthreads();
    const long long rb = a.row_ptr[v], re = a.row_ptr[v + 1];
    for (long long e = rb + threadIdx.x; e < re; e += blockDim.x) {
      const int j = __builtin_nontemporal_load(a.col + e);
      if (j == self) continue;
      const float w = a.w ? __builtin_nontemporal_load(a.w + e) : 1.0f;
      shared_add<K>(key, val, a.C[j], w);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int cv = a.C[self];
      int c = cv;
      float bv = 0.0f;
      for (int s = 0; s < K; ++s)
        if (val[s] > bv || (val[s] == bv && val[s] > 0.0f && key[s] < c)) {
          c = key[s];
          bv = val[s];
        }
      const bool moved = c != cv && (!a.pickless || c < cv);
      if (moved) {
        a.C[self] = c;
        atomicAdd(gd.dN + st->iter, 1ull);
      }
      a.hub_act[h] = moved ? 1 : 0;  // k_hub_mark flags the neighbours
      atomicAdd(gd.scanned + st->iter, (unsigned long long)(re - rb));
    }
    __syncthreads();
  }
}

// Convergence test of Algorithm 1 for every graph of the launch: after
// iteration l, stop when l is not a pick-less iteration and dN / N < tol,
// or when max_iter iterations have run.
__global__ void k_finish(Launch L) {
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < L.G; g += gridDim.x * blockDim.x) {
    const GraphDesc &d = L.d[g];
    GraphStatus *st = d.st;
    int changed = 0;  // dN of the iteration this launch ran (0: none ran)
    if (!st->done) {
      const int l = st->iter;
      const bool pl = d.rho > 0 && l % d.rho == 0;
      const double frac = (double)d.dN[l] / (double)d.n;
      const bool stop = (!pl && frac < d.tol) || l + 1 >= d.max_iter;
      changed = (int)d.dN[l];  // at most n < 2^31
      st->iter = l + 1;
      if (stop) {
        st->done = 1;
        atomicAdd(L.finished, 1);
      }
    }
    L.status_out[3 * g] = st->iter;
    L.status_out[3 * g + 1] = st->done;
    L.status_out[3 * g + 2] = changed;
  }
}

// ---------------------------------------------------------------------------
template <int K, bool ASYNC, bool RS, bool W, bool HS = false, bool SV = false>
static hipError_t launch_t(const Launch &L, int grid, int merge_grid, hipStream_t s,
                           hipEvent_t ev_beg, hipEvent_t ev_end) {
  hipError_t e = hipSuccess;
  if (ASYNC && L.total_hubs > 0) {
    const int sg = (L.total_hubs + 255) / 256 < 1024 ? (L.total_hubs + 255) / 256 : 1024;
    hipLaunchKernelGGL(k_hub_snapshot, dim3(sg), dim3(256), 0, s, L);
  }
  if (ev_beg && (e = hipEventRecord(ev_beg, s)) != hipSuccess) return e;
  if (L.total_items > 0) {
    if constexpr (RS)
      hipLaunchKernelGGL((k_move_rescan<K, ASYNC, W>), dim3(grid), dim3(kBlock), 0, s, L);
    else if constexpr (SV)
      hipLaunchKernelGGL((k_move_sv<K, W>), dim3(grid), dim3(kBlock), 0, s, L);
    else
      hipLaunchKernelGGL((k_move<K, ASYNC, W>), dim3(grid), dim3(kBlock), 0, s, L);
  }
  if (ev_end && (e = hipEventRecord(ev_end, s)) != hipSuccess) return e;
  if constexpr (HS) {  // shared hub sketches replace segments and merging
    if (L.total_hubs > 0) {
      const int hg = L.total_hubs < grid * 4 ? L.total_hubs : grid * 4;
      hipLaunchKernelGGL((k_hub_shared<K>), dim3(hg), dim3(256), 0, s, L);
      if (L.total_segs > 0) hipLaunchKernelGGL(k_hub_mark, dim3(grid), dim3(kBlock), 0, s, L);
    }
  } else if (ASYNC && L.total_merge > 0) {
    if constexpr (RS) {
      hipLaunchKernelGGL((k_hub_cand<K>), dim3(merge_grid), dim3(kBlock), 0, s, L);
      if (L.total_segs > 0)
        hipLaunchKernelGGL((k_hub_rescan<K>), dim3(grid), dim3(kBlock), 0, s, L);
      hipLaunchKernelGGL((k_hub_pick<K>), dim3(merge_grid), dim3(kBlock), 0, s, L);
    } else {
      hipLaunchKernelGGL((k_hub_merge<K>), dim3(merge_grid), dim3(kBlock), 0, s, L);
    }
    if (L.total_segs > 0) hipLaunchKernelGGL(k_hub_mark, dim3(grid), dim3(kBlock), 0, s, L);
  }
  if (!L.no_finish) {
    const int fg = (L.G + 255) / 256 < 64 ? (L.G + 255) / 256 : 64;
    hipLaunchKernelGGL(k_finish, dim3(fg > 0 ? fg : 1), dim3(256), 0, s, L);
  }
  return hipGetLastError();
}

template <int K, bool ASYNC, bool RS, bool W, bool SV = false>
static int occ_t() {
  int nb = 0;
  const void *f;
  if constexpr (RS)
    f = (const void *)k_move_rescan<K, ASYNC, W>;
  else if constexpr (SV)
    f = (const void *)k_move_sv<K, W>;
  else
    f = (const void *)k_move<K, ASYNC, W>;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kBlock, 0) != hipSuccess) return 1;
  return nb > 0 ? nb : 1;
}

template <bool ASYNC, bool RS, bool W>
static hipError_t launch_mode(int k, const Launch &L, int grid, int merge_grid, hipStream_t s,
                              hipEvent_t b, hipEvent_t e) {
  switch (k) {
    case 1: return launch_t<1, ASYNC, RS, W>(L, grid, merge_grid, s, b, e);
    case 2: return launch_t<2, ASYNC, RS, W>(L, grid, merge_grid, s, b, e);
    case 4: return launch_t<4, ASYNC, RS, W>(L, grid, merge_grid, s, b, e);
    case 8: return launch_t<8, ASYNC, RS, W>(L, grid, merge_grid, s, b, e);
    case 16: return launch_t<16, ASYNC, RS, W>(L, grid, merge_grid, s, b, e);
    case 32: return launch_t<32, ASYNC, RS, W>(L, grid, merge_grid, s, b, e);
    default: return hipErrorInvalidValue;
  }
}

template <bool ASYNC, bool RS, bool W>
static int occ_mode(int k) {
  switch (k) {
    case 1: return occ_t<1, ASYNC, RS, W>();
    case 2: return occ_t<2, ASYNC, RS, W>();
    case 4: return occ_t<4, ASYNC, RS, W>();
    case 8: return occ_t<8, ASYNC, RS, W>();
    case 16: return occ_t<16, ASYNC, RS, W>();
    case 32: return occ_t<32, ASYNC, RS, W>();
    default: return 1;
  }
}

template <bool HS, bool W>
static hipError_t launch_hs(int k, const Launch &L, int grid, int merge_grid, hipStream_t s,
                            hipEvent_t b, hipEvent_t e) {
  switch (k) {
    case 1: return launch_t<1, true, false, W, HS>(L, grid, merge_grid, s, b, e);
    case 2: return launch_t<2, true, false, W, HS>(L, grid, merge_grid, s, b, e);
    case 4: return launch_t<4, true, false, W, HS>(L, grid, merge_grid, s, b, e);
    case 8: return launch_t<8, true, false, W, HS>(L, grid, merge_grid, s, b, e);
    case 16: return launch_t<16, true, false, W, HS>(L, grid, merge_grid, s, b, e);
    case 32: return launch_t<32, true, false, W, HS>(L, grid, merge_grid, s, b, e);
    default: return hipErrorInvalidValue;
  }
}

template <bool W>
static hipError_t launch_sv(int k, const Launch &L, int grid, int merge_grid, hipStream_t s,
                            hipEvent_t b, hipEvent_t e) {
  switch (k) {
    case 1: return launch_t<1, false, false, W, false, true>(L, grid, merge_grid, s, b, e);
    case 2: return launch_t<2, false, false, W, false, true>(L, grid, merge_grid, s, b, e);
    case 4: return launch_t<4, false, false, W, false, true>(L, grid, merge_grid, s, b, e);
    case 8: return launch_t<8, false, false, W, false, true>(L, grid, merge_grid, s, b, e);
    case 16: return launch_t<16, false, false, W, false, true>(L, grid, merge_grid, s, b, e);
    case 32: return launch_t<32, false, false, W, false, true>(L, grid, merge_grid, s, b, e);
    default: return hipErrorInvalidValue;
  }
}

template <bool W>
static int occ_sv(int k) {
  switch (k) {
    case 1: return occ_t<1, false, false, W, true>();
    case 2: return occ_t<2, false, false, W, true>();
    case 4: return occ_t<4, false, false, W, true>();
    case 8: return occ_t<8, false, false, W, true>();
    case 16: return occ_t<16, false, false, W, true>();
    case 32: return occ_t<32, false, false, W, true>();
    default: return 1;
  }
}

template <bool W>
static hipError_t launch_iteration_w(int k, bool async_mode, bool rescan, bool hub_shared,
                                     bool shared_vars, const Launch &L, int grid, int merge_grid,
                                     hipStream_t s, hipEvent_t ev_beg, hipEvent_t ev_end) {
  if (shared_vars) {  // det sketch rule without double scan only
    if (async_mode || rescan || hub_shared || k == 0) return hipErrorInvalidValue;
    return launch_sv<W>(k, L, grid, merge_grid, s, ev_beg, ev_end);
  }
  if (hub_shared) {  // async sketch rule without double scan only
    if (!async_mode || rescan || k == 0) return hipErrorInvalidValue;
    return launch_hs<true, W>(k, L, grid, merge_grid, s, ev_beg, ev_end);
  }
  if (k == 0) {  // the vote of Algorithm 3 (no double scan)
    if (rescan) return hipErrorInvalidValue;
    return async_mode ? launch_t<0, true, false, W>(L, grid, merge_grid, s, ev_beg, ev_end)
                      : launch_t<0, false, false, W>(L, grid, merge_grid, s, ev_beg, ev_end);
  }
  if (rescan)
    return async_mode ? launch_mode<true, true, W>(k, L, grid, merge_grid, s, ev_beg, ev_end)
                      : launch_mode<false, true, W>(k, L, grid, merge_grid, s, ev_beg, ev_end);
  return async_mode ? launch_mode<true, false, W>(k, L, grid, merge_grid, s, ev_beg, ev_end)
                    : launch_mode<false, false, W>(k, L, grid, merge_grid, s, ev_beg, ev_end);
}

hipError_t launch_iteration(int k, bool async_mode, bool rescan, bool hub_shared,
                            bool shared_vars, bool wide, const Launch &L, int grid,
                            int merge_grid, hipStream_t s, hipEvent_t ev_beg, hipEvent_t ev_end) {
  return wide ? launch_iteration_w<true>(k, async_mode, rescan, hub_shared, shared_vars, L, grid,
                                         merge_grid, s, ev_beg, ev_end)
              : launch_iteration_w<false>(k, async_mode, rescan, hub_shared, shared_vars, L, grid,
                                          merge_grid, s, ev_beg, ev_end);
}

template <bool W>
static int move_blocks_w(int k, bool async_mode, bool rescan, bool shared_vars) {
  if (shared_vars && k > 0 && !async_mode && !rescan) return occ_sv<W>(k);
  if (k == 0) return async_mode ? occ_t<0, true, false, W>() : occ_t<0, false, false, W>();
  if (rescan) return async_mode ? occ_mode<true, true, W>(k) : occ_mode<false, true, W>(k);
  return async_mode ? occ_mode<true, false, W>(k) : occ_mode<false, false, W>(k);
}

hipError_t launch_finish(const Launch &L, hipStream_t s) {
  const int fg = (L.G + 255) / 256 < 64 ? (L.G + 255) / 256 : 64;
  hipLaunchKernelGGL(k_finish, dim3(fg > 0 ? fg : 1), dim3(256), 0, s, L);
  return hipGetLastError();
}

int move_blocks_per_cu(int k, bool async_mode, bool rescan, bool shared_vars, bool wide) {
  return wide ? move_blocks_w<true>(k, async_mode, rescan, shared_vars)
              : move_blocks_w<false>(k, async_mode, rescan, shared_vars);
}

}  // namespace lpa
