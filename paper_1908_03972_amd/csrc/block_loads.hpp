// Loads of the smoother's FP32 inverse blocks in the fused sweeps. A level whose blocks exceed
// the 256 MB Infinity Cache streams them from HBM once per sweep with nothing to gain from caching
// them; non-temporal loads then keep the lines from displacing the state, residual and geometry
// arrays that the sweep reuses (measured on the P3 and P2 sphere levels, 15.1 GB and 2.7 GB of
// FP32 blocks: 2.94 -> 2.57 ms and 0.605 -> 0.524 ms per sweep). Blocks that fit the cache are
// loaded normally, so that successive sweeps find them there (the P1 sphere level, 236 MB: 2%
// slower with non-temporal loads). FP64 blocks keep normal loads: a lane reads its 32 bytes of a
// column as two 16-byte loads, and with the non-temporal hint the P3 FP64 sweep was 6% slower.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <type_traits>

namespace pmg {

constexpr size_t kStreamBlocksBytes = size_t(256) << 20;

typedef float blk_f4 __attribute__((ext_vector_type(4)));

template <bool NT>
__device__ __forceinline__ blk_f4 load_block4(const float* p) {
  if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const blk_f4*>(p));
  else return *reinterpret_cast<const blk_f4*>(p);
}

}  // namespace pmg
