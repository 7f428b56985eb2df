// Internal declarations shared by the HIP translation units of liblpa.so.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lpa.h"

namespace lpa {

constexpr int kWave = 64;
constexpr int kBlock = 256;  // threads per workgroup for the move kernels

// Degree classes used to order vertices by decreasing degree.  Classes
// 0..255 hold hubs (degree > lane_max_degree) on a log scale with eight
// sub-buckets per octave; classes 256..256+T-1 hold degrees T..1 exactly.
constexpr int kHubClasses = 256;

__host__ __device__ inline int degree_class(int d, int lane_max) {
  if (d > lane_max) {
    int b = 31 - __builtin_clz((unsigned)d);
    int sub = b >= 3 ? (d >> (b - 3)) & 7 : (d << (3 - b)) & 7;
    return kHubClasses - 1 - (b * 8 + sub);
  }
  return kHubClasses + (lane_max - d);
}

// Arguments of one lpaMove launch.
struct MoveArgs {
  int32_t n;
  const int32_t *row_ptr;
  const int32_t *col;
  const float *w;          // nullable: unit weights
  int32_t *C;              // labels read this iteration (async: read/write)
  int32_t *Cn;             // labels written this iteration (async: == C)
  uint8_t *act_cur;        // unprocessed flags read (and cleared) this iteration
  uint8_t *act_next;       // flags set for the next iteration (async: == act_cur)
  const int32_t *order;    // vertex ids: hubs (desc degree), then lane vertices
  int32_t n_hubs;          // vertices of degree > seg_len
  int32_t n_lane;          // vertices of degree 1 .. seg_len
  int32_t seg_len;         // S: longest run of CSR entries one lane scans
  // LPA_MODE_ASYNC hub segments and partial sketches
  int32_t n_seg;                // segment units (0 in det mode)
  const int32_t *seg_hub;       // [n_seg] hub index of each segment
  const int32_t *hub_pbase;     // [n_hubs + 1] first segment of each hub
  uint8_t *hub_act;             // [n_hubs] flags snapshot of this iteration
  int32_t *part_key;            // [n_seg * k]
  float *part_val;              // [n_seg * k]
  int32_t iter;
  int32_t pickless;
  unsigned long long *dN;       // [max_iter]
  unsigned long long *scanned;  // [max_iter]
  const int32_t *done;
};

// Enqueue one iteration's move pass (async: hub flag snapshot, k_move, hub
// merge; det: k_move).  Non-null events are recorded around k_move only.
hipError_t launch_move(int k, bool async_mode, const MoveArgs &a, int grid,
                       int merge_grid, hipStream_t s, hipEvent_t ev_beg,
                       hipEvent_t ev_end);
int move_blocks_per_cu(int k, bool async_mode);

}  // namespace lpa
