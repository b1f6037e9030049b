// Sums over one wavefront on the vector unit, every lane getting the total: DPP moves inside each
// 16-lane row (neighbours, pairs of neighbours, the two halves of a row, the two halves of the
// row), then v_permlane16_swap (rows 0+1, 2+3) and v_permlane32_swap (the two halves of the
// wavefront).  No LDS round trip; the wavefront must be fully active.
#pragma once

#include <hip/hip_runtime.h>

namespace calib {

// ordering of LDS writes and reads among the lanes of one wavefront (in-order within a wavefront;
// the fences keep the compiler from moving accesses across); unlike a workgroup barrier it does
// not wait for the wavefront's outstanding global loads
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
namespace wred {

template <int CTRL>
__device__ inline double dpp_mov(double x) {
  const long long v = __builtin_bit_cast(long long, x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// x + (x of the lane 16 (kRows = 16) or 32 (kRows = 32) lanes away), from the two copies that the
// swap leaves
template <int kRows>
__device__ inline double swap_add(double x) {
  const long long v = __builtin_bit_cast(long long, x);
  const int vl = (int)v, vh = (int)(v >> 32);
  const auto lo = kRows == 16 ? __builtin_amdgcn_permlane16_swap(vl, vl, false, false)
                              : __builtin_amdgcn_permlane32_swap(vl, vl, false, false);
  const auto hi = kRows == 16 ? __builtin_amdgcn_permlane16_swap(vh, vh, false, false)
                              : __builtin_amdgcn_permlane32_swap(vh, vh, false, false);
  const long long a = ((long long)hi[0] << 32) | (unsigned int)lo[0];
  const long long b = ((long long)hi[1] << 32) | (unsigned int)lo[1];
  return __builtin_bit_cast(double, a) + __builtin_bit_cast(double, b);
}

}  // namespace wred

// NV sums at once, step by step, so the steps' moves of different values are independent
template <int NV>
__device__ inline void wave_sum_vec(double *v) {
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] += wred::dpp_mov<0xB1>(v[i]);    // quad_perm [1,0,3,2]
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] += wred::dpp_mov<0x4E>(v[i]);    // quad_perm [2,3,0,1]
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] += wred::dpp_mov<0x141>(v[i]);   // row_half_mirror
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] += wred::dpp_mov<0x140>(v[i]);   // row_mirror
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wred::swap_add<16>(v[i]);
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wred::swap_add<32>(v[i]);
}

__device__ inline double wave_sum(double x) {
  wave_sum_vec<1>(&x);
  return x;
}

}  // namespace calib
