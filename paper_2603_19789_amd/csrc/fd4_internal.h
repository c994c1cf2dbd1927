// fd4_internal.h -- the finite-difference reference solver's launcher
// (fd4_kernels.hip), called by the host API (not part of the ABI).
#pragma once

#include <hip/hip_runtime_api.h>

#include "sslbm_internal.h"

namespace sslbm {

// nsteps RK4 steps of the fourth-order finite-difference system, in place
// in rho; work holds three states (two stage inputs and the running sum).
hipError_t launch_fd4(int dtype, void *rho, void *work, const GridDesc &g, const StepCoef &k,
                      long long nsteps, hipStream_t s);

}  // namespace sslbm
