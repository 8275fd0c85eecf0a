// Fused steps of the V-cycle's level transitions (transfer_kernels.hip, fr_kernels.hip).
#pragma once

#include "internal.hpp"

namespace pmg {

// xc = xc2 = R xf and xd = R xg from level Lf to level Lc (one kernel on quadrilaterals, two on
// hexahedra); xc2 may not be null
hipError_t launch_restrict_pair(const pmg_level_s& Lf, const pmg_level_s& Lc, const double* R1, const double* xf,
                                double* xc, double* xc2, const double* xg, double* xd, int nvar, hipStream_t st);

// The first pre-smoothing sweep of a coarse level at its restricted state q^b, with S holding the
// restricted fine residual P w on entry: the sweep's defect there is P w itself, and S leaves with
// the forcing S_{l+1} = F_{l+1}(q^b) - P w of eqs. (40), (43) (one kernel on quadrilaterals; a
// residual and a sweep on hexahedra)
hipError_t launch_sweep_forming_S(const pmg_level_s& L, const pmg_factors_s& fac, const double* q_in, double* q_out,
                                  double* S, double c_mass, double alpha, hipStream_t st);

}  // namespace pmg
