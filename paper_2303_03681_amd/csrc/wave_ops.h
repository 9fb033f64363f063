// Wave-level helpers shared by the device kernels (64-lane wavefronts).
#pragma once

#include <hip/hip_runtime.h>

namespace mps {

// Lane permutation within rows of 16 lanes (DPP control CTRL) of a double.
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// A wave-uniform value moved to scalar registers (it is identical in all lanes).
__device__ __forceinline__ double wave_uniform(double x) {
  const int lo = __builtin_amdgcn_readfirstlane(__double2loint(x));
  const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(x));
  return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes of a wave, the same bits in every lane (each step
// adds a and b in both orders, and a + b == b + a exactly): DPP moves within
// rows of 16 lanes, then two cross-row exchanges.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);  // row_half_mirror
  v += dpp_mov<0x140>(v);  // row_mirror
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// wave_sum of N independent values, stage by stage so the N dependency
// chains interleave (the same bits as N separate wave_sum calls).
template <int N>
__device__ __forceinline__ void wave_sum_n(double (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_mov<0xB1>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_mov<0x4E>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_mov<0x141>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += dpp_mov<0x140>(v[i]);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], 16, 64);
#pragma unroll
  for (int i = 0; i < N; ++i) v[i] += __shfl_xor(v[i], 32, 64);
}

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

}  // namespace mps
