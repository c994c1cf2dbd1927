// adjoint_internal.h -- declarations shared by the host side of the adjoint
// entry points and the adjoint kernels (not part of the ABI).
#pragma once

#include <hip/hip_runtime_api.h>

#include "sslbm_internal.h"

namespace sslbm {

constexpr int ADJ_SUMS = 10;  // partial sums kept per wavefront slot
constexpr int ADJ_SLOT = 16;  // doubles per slot (padded to 128 bytes)

// Wavefront decomposition of one adjoint step: strips of 62 columns times
// chunks of `rows` rows; one partials slot per wavefront.
struct AdjShape {
    int strips, chunks, rows;
    long long slots() const { return (long long)strips * chunks; }
};

// Factors applied to the summed partials at the end of a run.
struct AdjFactors {
    double dt;        // beta, alpha, gamma gradients
    double gamma_dt;  // phi gradient
    double phi;       // splits the removal flow between R and D
    double dt_dx2;    // diffusivity gradients: d tau / d d = 3 dt / dx^2, times 1/3
};

AdjShape adjoint_shape(int nx, int ny);
// One reverse step: out = A(rho)^T lam; the step's partial sums are written
// (first) or added to the wavefront slots of `partials`.
hipError_t launch_adjoint(int dtype, const void *rho, const void *lam, void *out,
                          const GridDesc &g, const StepCoef &k, const AdjShape &s,
                          double *partials, bool first, hipStream_t st);
// Two reverse steps in one pass (lam(n) from lam(n + 2) and rho(n)), the
// state of step n + 1 recomputed in registers; the sums of both steps are
// added to the wavefront slots (zeroed beforehand with launch_zero).
AdjShape adjoint2_shape(int nx, int ny);
hipError_t launch_adjoint2(int dtype, const void *rho, const void *lam, void *out,
                           const GridDesc &g, const StepCoef &k, const AdjShape &s,
                           double *partials, hipStream_t st);
hipError_t launch_zero(double *p, long long n, hipStream_t st);
// grad[0..8] += the scaled sums of all slots.
hipError_t launch_adjoint_finish(const double *partials, int slots, const AdjFactors &f,
                                 double *grad, hipStream_t st);

}  // namespace sslbm
