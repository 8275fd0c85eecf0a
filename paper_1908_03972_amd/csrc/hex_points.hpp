// Point numbering on hexahedra shared by the residual/sweep and the element-block kernels:
// solution points p = i + (P+1) j + (P+1)^2 k, face points k1 + (P+1) k2 along the face's
// tangential directions, and the orientation code of a face pair.
#pragma once

#include <hip/hip_runtime.h>

namespace pmg {

// solution point m of the tensor line through face point (k1, k2) of face f (m along the normal)
__device__ __forceinline__ int line_point3(int f, int k1, int k2, int m, int n1) {
  if (f < 2) return m + n1 * (k1 + n1 * k2);
  if (f < 4) return k1 + n1 * (m + n1 * k2);
  return k1 + n1 * (k2 + n1 * m);
}

// the neighbour's face point met by (k1, k2): swap (bit 0), reverse first (bit 1), second (bit 2)
__device__ __forceinline__ void orient3(int o, int k1, int k2, int n1, int& a, int& b) {
  a = (o & 1) ? k2 : k1;
  b = (o & 1) ? k1 : k2;
  if (o & 2) a = n1 - 1 - a;
  if (o & 4) b = n1 - 1 - b;
}

}  // namespace pmg
