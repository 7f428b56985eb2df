// Wavefront helpers and the LDS row stage shared by the scan kernels
// (lpaMove and modularity).
#pragma once

#include <hip/hip_runtime.h>

#include "lpa_internal.h"

namespace lpa {

__device__ __forceinline__ int rfl(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ long long rfl64(long long x) {
  const unsigned long long u = (unsigned long long)x;
  const unsigned lo = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)u);
  const unsigned hi = (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)(u >> 32));
  return (long long)(((unsigned long long)hi << 32) | lo);
}
// readfirstlane of an int or a long long
template <class T>
__device__ __forceinline__ T rfl_as(T x) {
  if constexpr (sizeof(T) == 8)
    return rfl64(x);
  else
    return rfl(x);
}
__device__ __forceinline__ float rfl_f(float x) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ int rl(int x, int lane) { return __builtin_amdgcn_readlane(x, lane); }
__device__ __forceinline__ float rl_f(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

// DPP move across lanes (CTRL: the dpp_ctrl encoding), every row and bank
// enabled; the source lanes are always active where these are used.
template <int CTRL>
__device__ __forceinline__ int dpp(int x) {
  return __builtin_amdgcn_update_dpp(x, x, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float x) {
  return __int_as_float(dpp<CTRL>(__float_as_int(x)));
}

// Order LDS accesses of this wavefront: the wavefront executes its LDS
// instructions in order, this only keeps the compiler from moving them.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int wave_max(int x) {
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) x = max(x, __shfl_xor(x, off));
  return x;
}

__device__ __forceinline__ double wave_sum_d(double x) {
#pragma unroll
  for (int off = kWave / 2; off >= 1; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// LDS staging of 64 rows (one per lane), T entries per row per step: the
// wavefront loads slot i * 64 + lane = entry j of row r with (r, j) =
// (slot / T, slot % T), so its loads are row-contiguous; each lane then
// reads its own row back.  Rows are padded to T + 1 words against bank
// conflicts.
template <int T, class P = int>
struct Stage {
  P beg[kWave];  // CSR position of each row's first entry (P: offset type)
  int len[kWave];
  int self[kWave];
  int lab[kWave * (T + 1)];
  float w[kWave * (T + 1)];
};

// Entries per row per staging step (LDS per wavefront: 64 x 17 x 8 bytes).
constexpr int kStageT = 16;

}  // namespace lpa
