// Wavefront-wide reductions, pivot keys and matrix-core steps shared by the element and line
// block eliminations.
#pragma once

#include <hip/hip_runtime.h>

namespace pmg {

// Maximum of an unsigned value over the 64 lanes of a wavefront, returned to every lane: DPP
// rotations within each row of 16 lanes, then the four row maxima through scalar registers.
__device__ __forceinline__ unsigned wave_max_u32(unsigned v) {
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x121, 0xf, 0xf, false));   // row_ror:1
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x122, 0xf, 0xf, false));   // row_ror:2
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xf, 0xf, false));   // row_ror:4
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xf, 0xf, false));   // row_ror:8
  const unsigned a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
  const unsigned c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
  return max(max(a, b), max(c, d));
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// 32-bit pivot key of |f| 2^e2 (the row's value after equilibration by the power of two 2^e2):
// the upper bits of that value (the FP32 pattern, or the upper word of the FP64 one), formed by
// adding e2 to the exponent field, with the low 10 bits replaced by 1023 - r, so that the wave
// maximum also names the row or thread; values whose scaled exponent leaves the normal range
// count as zero (below) or infinity (above), and unscaled subnormals as zero
__device__ __forceinline__ unsigned pivot_key(float f, int r, int e2) {
  const unsigned b = __float_as_uint(fabsf(f));
  const int eb = (int)(b >> 23) + e2;
  const unsigned sb = ((b >> 23) == 0u || eb <= 0) ? 0u : (eb >= 255 ? 0x7F800000u : b + ((unsigned)e2 << 23));
  return (sb & ~0x3FFu) | (unsigned)(1023 - r);
}
__device__ __forceinline__ unsigned pivot_key(double f, int r, int e2) {
  const unsigned b = (unsigned)__double2hiint(fabs(f));
  const int eb = (int)(b >> 20) + e2;
  const unsigned sb = ((b >> 20) == 0u || eb <= 0) ? 0u : (eb >= 2047 ? 0x7FF00000u : b + ((unsigned)e2 << 20));
  return (sb & ~0x3FFu) | (unsigned)(1023 - r);
}

typedef float flt4 __attribute__((ext_vector_type(4)));


// One 16x16x4 matrix-core step in T, and the row i of the 16 x 16 result held by accumulator
// register v in lane group lk: D[i][j] sits in lane j + 16 (i / 4), register i % 4 for FP32 and
// in lane j + 16 (i % 4), register i / 4 for FP64 (both checked on gfx950)
__device__ __forceinline__ flt4 mfma16x16x4(float a, float b, flt4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ dbl4 mfma16x16x4(double a, double b, dbl4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
template <typename T>
__device__ __forceinline__ int acc_row(int lk, int v) {
  return sizeof(T) == 4 ? 4 * lk + v : lk + 4 * v;
}

}  // namespace pmg
