// Launchers of the Newton-Krylov vector kernels (krylov_kernels.hip).
#pragma once

#include "internal.hpp"

namespace pmg {

constexpr int kNkMaxDim = 32;                 // Krylov directions per Newton step
constexpr int kNkMaxTerms = kNkMaxDim + 2;    // vectors in one linear combination or block of dots
constexpr int kNkDotBlocks = 256;             // per-workgroup partials of one dot product

// y = beta y + sum_k c[k] x[k] over n entries (c on the host; beta = 0 ignores y)
hipError_t launch_lincomb(size_t n, int nt, const double* const* x, const double* c, double beta, double* y,
                          hipStream_t st);
// out[k] = sum_i w[i] x[k][i], k < nt, with a fixed reduction order; part holds
// kNkMaxTerms * kNkDotBlocks doubles of partial sums
hipError_t launch_multidot(size_t n, int nt, const double* const* x, const double* w, double* part, double* out,
                           hipStream_t st);
// out = Gamma(q) z inv_dtau - (Fh - F0) inv_h on the points of level L
hipError_t launch_newton_op(const pmg_level_s& L, const double* q, const double* z, const double* Fh,
                            const double* F0, double inv_dtau, double inv_h, double* out, hipStream_t st);

}  // namespace pmg
