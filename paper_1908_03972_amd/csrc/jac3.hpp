// Sizes shared by the hexahedral element-block launcher and the factor allocation.
#pragma once

#include <cstddef>

namespace pmg {

// doubles of pointwise derivatives per element kept for the large-block elimination (P = 3): the
// three flux Jacobians and the diagonal term at every solution point, the common-flux derivative
// at every face point, Nv x Nv each
constexpr size_t jac3_point_elems(int P) {
  return (size_t)(4 * (P + 1) * (P + 1) * (P + 1) + 6 * (P + 1) * (P + 1)) * 25;
}

}  // namespace pmg
