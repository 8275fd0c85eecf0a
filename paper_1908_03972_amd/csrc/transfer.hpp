// The fused pair of restrictions of a V-cycle level transition (transfer_kernels.hip).
#pragma once

#include "internal.hpp"

namespace pmg {

// xc = xc2 = R xf and xd = R xg from level Lf to level Lc (one kernel on quadrilaterals, two on
// hexahedra); xc2 may not be null
hipError_t launch_restrict_pair(const pmg_level_s& Lf, const pmg_level_s& Lc, const double* R1, const double* xf,
                                double* xc, double* xc2, const double* xg, double* xd, int nvar, hipStream_t st);

}  // namespace pmg
