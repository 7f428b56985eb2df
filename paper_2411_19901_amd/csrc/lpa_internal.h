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
  int32_t n_hubs;
  int32_t n_lane;
  int32_t total_items;     // n_hubs + ceil(n_lane / 64)
  int32_t iter;
  int32_t pickless;
  unsigned long long *dN;       // [max_iter]
  unsigned long long *scanned;  // [max_iter]
  const int32_t *done;
};

hipError_t launch_move(int k, bool async_mode, const MoveArgs &a, int grid,
                       hipStream_t s);
int move_blocks_per_cu(int k, bool async_mode);

}  // namespace lpa
