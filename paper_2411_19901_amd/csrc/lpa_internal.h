// Internal declarations shared by the HIP translation units of liblpa.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lpa.h"

namespace lpa {

constexpr int kWave = 64;
constexpr int kBlock = 256;  // threads per workgroup for the move kernels
// Hub merge kernels: kHubLanes lanes per hub, kMergeHubs hubs per wavefront.
constexpr int kHubLanes = 4;
constexpr int kMergeHubs = kWave / kHubLanes;

// Degree classes used to order vertices by decreasing degree.  Classes
// 0..255 hold hubs (degree > lane_max) on a log scale with eight
// sub-buckets per octave; lane degrees 65..lane_max (lane_max <= 65536)
// use the same eighth-of-an-octave buckets (classes 256..343); degrees
// 64..1 have one class each (344..407).  Within a class vertices keep
// increasing id order (the binning is stable).
constexpr int kHubClasses = 256;
constexpr int kLaneBuckets = 88;  // eighth-octave buckets for degrees 65 .. 2^17 - 1
constexpr int kLaneExact = 64;    // one class per degree 1 .. 64
constexpr int kClasses = kHubClasses + kLaneBuckets + kLaneExact;
// The binning adds one class after these for the isolated vertices (degree
// 0), so that the degree order lists every vertex: hubs, lane vertices,
// then isolated ones.
constexpr int kBinClasses = kClasses + 1;

// Short units: the lane vertices of degree 1 .. kShortDeg (the last lane
// classes of the degree order) are scanned kShortRows rows per lane, each
// lane reading its own rows (see short_units in move.hip).
constexpr int kShortDeg = 4;
constexpr int kShortRows = 2;
// Class of degree kShortDeg: the short vertices are the lane vertices from
// its first position on.
constexpr int kShortClass = kHubClasses + kLaneBuckets + (kLaneExact - kShortDeg);

// Move-kernel work items of `units` lane units of which the last `n_short`
// are short vertices: kWave lane units per item, then kShortRows x kWave
// short vertices per item.
__host__ __device__ inline int64_t lane_items(int64_t units, int64_t n_short) {
  const int64_t per = (int64_t)kWave * kShortRows;
  return (units - n_short + kWave - 1) / kWave + (n_short + per - 1) / per;
}

__host__ __device__ inline int octave_bucket(int d) {  // d >= 1
  const int b = 31 - __builtin_clz((unsigned)d);
  const int sub = b >= 3 ? (d >> (b - 3)) & 7 : (d << (3 - b)) & 7;
  return b * 8 + sub;
}

__host__ __device__ inline int degree_class(int d, int lane_max) {
  if (d == 0) return kClasses;  // isolated: last
  if (d > lane_max) return kHubClasses - 1 - octave_bucket(d);
  if (d > kLaneExact) return kHubClasses + kLaneBuckets - 1 - (octave_bucket(d) - 6 * 8);
  return kHubClasses + kLaneBuckets + (kLaneExact - d);
}

// Device pointers into device or mapped host memory, never LDS or scratch.
// Typed as the global address space so that the compiler emits global
// (not flat) loads and stores: flat accesses may alias LDS, which forbids
// moving them across the LDS staging and serialises a wavefront's loads.
#define LPA_GLOBAL __attribute__((address_space(1)))
template <class T>
using gptr = T LPA_GLOBAL *;
template <class T>
__host__ __device__ __forceinline__ gptr<T> as_global(T *p) {
  return (gptr<T>)p;
}

// Launch tables that no kernel writes while it runs (the per-graph prefix
// sums and descriptors, and each graph's status outside the stop test,
// which writes it in a launch of its own): typed as the constant address
// space, so that reads at uniform addresses are scalar loads served by the
// scalar cache rather than vector-memory round trips.
#define LPA_CONST __attribute__((address_space(4)))
template <class T>
using kptr = const T LPA_CONST *;
template <class T>
__host__ __device__ __forceinline__ kptr<T> as_const(const T *p) {
  return (kptr<T>)p;
}

// CSR row offsets, 32- or 64-bit: exactly one pointer is set for a graph
// with vertices.  The choice is the same for every vertex of a graph, so
// the test is a uniform branch.
struct RowPtr {
  const int32_t *p32;
  const int64_t *p64;
  __device__ __forceinline__ long long operator[](long long i) const {
    return p64 ? (long long)as_global(p64)[i] : (long long)as_global(p32)[i];
  }
};

// Device-resident progress of one graph, updated by the convergence kernel.
struct GraphStatus {
  int32_t iter;       // iterations run so far
  int32_t done;       // converged or max_iter reached
  int32_t err;        // validation / label-check error bits
  int32_t totals[4];  // binning results: hubs, lane vertices, segments, short vertices
  int32_t fresh;      // 1: the labels are the initial ones (reset, no lpa_set_state since)
  unsigned long long sink;
};

// Static description of one graph's arrays (pointers never change after
// lpa_init); a launch reads a table of these.
struct GraphDesc {
  int32_t n;
  int32_t n_hubs;     // vertices of degree > seg_len
  int32_t n_lane;     // vertices of degree 1 .. seg_len
  int32_t n_short;    // the last n_short lane vertices run as short units (degree <= kShortDeg)
  int32_t n_seg;      // async hub segments (0 in det mode)
  int32_t seg_len;    // S: longest run of CSR entries one lane scans
  int32_t max_iter;
  int32_t rho;
  int32_t items;      // move-kernel work items per iteration
  double tol;
  RowPtr row_ptr;
  const int32_t *col;  // neighbour ids; with `ranked`, their degree-order positions
  const float *w;     // nullable: unit weights
  // 1: labels and flags are stored by degree-order position (the vertex at
  // order[p] keeps its state at index p) and `col` holds positions; the
  // label values are vertex ids either way
  int32_t ranked;
  int32_t *C[2];      // det: labels of even / odd iterations; async: both C[0]
  uint8_t *act[2];    // det: flags of even / odd iterations; async: both act[0]
  const int32_t *order;      // vertex ids: hubs (desc degree), then lane vertices
  const int32_t *seg_hub;    // [n_seg] hub index of each segment
  const int32_t *hub_pbase;  // [n_hubs + 1] first segment of each hub
  uint8_t *hub_act;          // [n_hubs] flags snapshot of this iteration
  int32_t *part_key;         // [n_seg * k]
  float *part_val;           // [n_seg * k]
  int32_t *hub_cand;         // [n_hubs * k] double-scan candidates (-1: none)
  int32_t hub_shared;        // 1: hubs use one shared sketch each (LPA_HUB_SHARED)
  // det: 1 when every hub row names each neighbour at most once (its column
  // indices strictly increase; checked at lpa_init), so that at iteration 0
  // from the initial labels every hub entry carries a label of its own
  int32_t hub_rows_distinct;
  unsigned long long *dN;       // [max_iter] changed vertices per iteration
  unsigned long long *scanned;  // [max_iter] CSR entries scanned per iteration
  GraphStatus *st;
};

// One set of launches over many graphs.  prefix_* hold G + 1 exclusive
// prefix sums of the per-graph counts (move items, hubs, merge items, hub
// segments).
struct Launch {
  const GraphDesc *d;
  const int32_t *prefix_items;
  const int32_t *prefix_hubs;
  const int32_t *prefix_merge;
  const int32_t *prefix_segs;  // hub segments (double scan in LPA_MODE_ASYNC)
  int32_t G;
  int32_t total_items;
  int32_t total_hubs;
  int32_t total_merge;
  int32_t total_segs;
  int32_t *finished;        // graphs that have finished (counter)
  int32_t *status_out;      // [3 * G]: iter, done, dN of the iteration just run (0: none)
  int32_t no_finish;        // 1: launch_iteration leaves out the stop test (k_finish)
};

// Per-graph view used by the move kernels for one iteration.
struct MoveArgs {
  int32_t n;
  RowPtr row_ptr;
  gptr<const int32_t> col;
  gptr<const float> w;
  gptr<int32_t> C;         // labels read this iteration (async: read/write)
  gptr<int32_t> Cn;        // labels written this iteration (async: == C)
  gptr<uint8_t> act_cur;   // unprocessed flags read (and cleared) this iteration
  gptr<uint8_t> act_next;  // flags set for the next iteration (async: == act_cur)
  gptr<const int32_t> order;
  int32_t ranked;          // state indexed by degree-order position (GraphDesc::ranked)
  int32_t n_hubs;
  int32_t n_lane;
  int32_t n_short;
  int32_t seg_len;
  int32_t n_seg;
  gptr<const int32_t> seg_hub;
  gptr<const int32_t> hub_pbase;
  gptr<uint8_t> hub_act;
  gptr<int32_t> part_key;
  gptr<float> part_val;
  int32_t iter;
  int32_t pickless;
  // det iteration 0 from the initial labels with duplicate-free hub rows:
  // every hub entry is a label no key holds (see GraphDesc::hub_rows_distinct)
  int32_t fresh_hubs;
};

// Kernel selector: k slots of the weighted Misra-Gries sketch, or 0 for the
// one-candidate vote of Algorithm 3 (LPA_RULE_BM_PAPER); rescan selects
// the double scan (LPA_RESCAN, k > 0 only); hub_shared replaces the hub
// segments' partial sketches by one shared sketch per hub (LPA_HUB_SHARED,
// async, k > 0, no double scan).
// shared_vars: LPA_SHARED_VARS (det sketch rule, single scan).
// wide: some graph of the launch has int64 row offsets (the kernels then
// compute CSR positions in 64 bits).
// Enqueue one iteration of every graph in the launch (async: hub flag
// snapshot, k_move, hub merge, and for the double scan the hub re-weighting
// and decision; det: k_move; then the convergence test).  Non-null events
// are recorded around k_move only.
hipError_t launch_iteration(int k, bool async_mode, bool rescan, bool hub_shared,
                            bool shared_vars, bool wide, const Launch &L, int grid,
                            int merge_grid, hipStream_t s, hipEvent_t ev_beg, hipEvent_t ev_end);
int move_blocks_per_cu(int k, bool async_mode, bool rescan, bool shared_vars, bool wide);
// The stop test alone (k_finish): an iteration split over id ranges of a
// graph runs launch_iteration once per range with Launch::no_finish set,
// then this once.
hipError_t launch_finish(const Launch &L, hipStream_t s);

// Modularity of one labelling (Eq. 1): vertices order[0, n_hubs) are read
// by one wavefront per segment (or per hub without segments),
// order[n_hubs, n_hubs + n_lane) one lane each (the last n_short of them,
// rows of at most kShortDeg entries, kShortRows rows per lane).
// Labels must lie in [0, n).  acc[0] += 2m, acc[1] += sigma,
// tot[c] += K_i for every vertex i labelled c.
struct ModArgs {
  const int32_t *order;
  int32_t n_hubs;
  int32_t n_lane;
  int32_t n_short;
  RowPtr row_ptr;
  const int32_t *col;  // ranked: degree-order positions of the neighbours
  const float *w;
  const int32_t *lab;  // ranked: indexed by degree-order position, else by id
  int32_t ranked;
  // hubs split into segments of seg_len entries (seg_hub[q] = hub of segment
  // q, hub_pbase[h] = first segment of hub h), or n_seg = 0: whole hubs
  int32_t n_seg;
  int32_t seg_len;
  const int32_t *seg_hub;
  const int32_t *hub_pbase;
  double *tot;
  double *acc;
};
hipError_t launch_modularity(const ModArgs &m, int grid, hipStream_t s);
int modularity_blocks_per_cu();

}  // namespace lpa
