// Cross-lane sums of doubles inside a wave of 64 lanes without LDS: DPP
// permutations inside rows of 16 lanes and the gfx950 row-pair and half
// swaps.  Each level adds the values of two paired lanes, and both lanes of
// a pair add the same two operands, so every lane of the group ends with the
// same bits.
#pragma once

#include <hip/hip_runtime.h>

namespace dsv {

// DPP lane permutations (both halves of a double):
//   0xB1 quad_perm [1,0,3,2]: lane ^ 1      0x4E quad_perm [2,3,0,1]: lane ^ 2
//   0x141 row_half_mirror:    lane ^ 7      0x140 row_mirror:         lane ^ 15
template <int CTRL>
__device__ __forceinline__ double lanes_dpp(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)(unsigned)lo) | ((long long)hi << 32));
}

// x + (x of lane ^ 16): the row-pair swap exchanges the operands, so the two
// results hold the value of each lane of the pair.
__device__ __forceinline__ double lanes_add_xor16(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  const auto l2 = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h2 = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  const double u = __longlong_as_double(((long long)(unsigned)l2[0]) | ((long long)h2[0] << 32));
  const double v = __longlong_as_double(((long long)(unsigned)l2[1]) | ((long long)h2[1] << 32));
  return u + v;
}

// x + (x of lane ^ 32), by the half swap.
__device__ __forceinline__ double lanes_add_xor32(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = (int)(b & 0xffffffffll), hi = (int)(b >> 32);
  const auto l2 = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h2 = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  const double u = __longlong_as_double(((long long)(unsigned)l2[0]) | ((long long)h2[0] << 32));
  const double v = __longlong_as_double(((long long)(unsigned)l2[1]) | ((long long)h2[1] << 32));
  return u + v;
}

// Sum over the 32 lanes of each half of the wave (every lane of both halves
// must be active).
__device__ __forceinline__ double lanes_half_sum(double x) {
  x += lanes_dpp<0xB1>(x);
  x += lanes_dpp<0x4E>(x);
  x += lanes_dpp<0x141>(x);
  x += lanes_dpp<0x140>(x);
  return lanes_add_xor16(x);
}

// Sum over the whole wave (every lane active).
__device__ __forceinline__ double lanes_wave_sum(double x) { return lanes_add_xor32(lanes_half_sum(x)); }

// Order the LDS accesses of the lanes of one wave: what a lane wrote before
// is visible to every lane of the wave after.
__device__ __forceinline__ void lanes_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace dsv
