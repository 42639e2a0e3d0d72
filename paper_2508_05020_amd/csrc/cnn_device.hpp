// Device helpers shared by the 2D and 3D predictor kernels: BF16 rounding,
// the 16x16x16 BF16 MFMA and 4-element operand loads.
//
// MFMA used: v_mfma_f32_16x16x16_bf16 (__builtin_amdgcn_mfma_f32_16x16x16bf16_1k).
// Operand layout per lane l (0..63), element e (0..3):
//   A[i][k]: i = l % 16, k = 4 (l / 16) + e
//   B[k][j]: j = l % 16, k = 4 (l / 16) + e
//   D[i][j]: j = l % 16, i = 4 (l / 16) + e
// (checked on the device by amr_cnn_mfma_selftest).
#pragma once

#include <hip/hip_runtime.h>

namespace amr {
namespace cnnd {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned short f2bf(float f) {
  // round to nearest even
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40);  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float(((unsigned)h) << 16); }

__device__ __forceinline__ f4 mfma(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ s4 load4(const unsigned short* p) {
  // p is 8-byte aligned (4 consecutive channels of one pixel)
  const uint2 v = *reinterpret_cast<const uint2*>(p);
  s4 r;
  r.x = (short)(v.x & 0xffff);
  r.y = (short)(v.x >> 16);
  r.z = (short)(v.y & 0xffff);
  r.w = (short)(v.y >> 16);
  return r;
}

__device__ __forceinline__ s4 zero4() {
  s4 r = {0, 0, 0, 0};
  return r;
}

__device__ __forceinline__ s4 pack4(short a, short b, short c, short d) {
  s4 r;
  r.x = a;
  r.y = b;
  r.z = c;
  r.w = d;
  return r;
}

}  // namespace cnnd
}  // namespace amr
