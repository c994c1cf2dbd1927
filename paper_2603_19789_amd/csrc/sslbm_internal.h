// sslbm_internal.h -- declarations shared by the host API and the kernel
// translation units of libsslbm.so (not installed, not part of the ABI).
#pragma once

#include <hip/hip_runtime_api.h>

#include <vector>

#include "sslbm.h"

namespace sslbm {

// Grid description passed by value to every kernel.
struct GridDesc {
    int nx, ny;
    long long plane;  // nx * ny
    int bc;           // SSLBM_PERIODIC or SSLBM_NOFLUX
};

// Per-step constants, derived once on the host in FP64 and rounded to the
// arithmetic type at launch:
//   dl[C] = d[C] dt / dx^2 (lattice diffusivity, tau = 1/2 + 3 dl),
//   bdt = beta dt, kE = alpha dt, kI = gamma dt,
//   kR = (1 - phi) gamma dt, kD = phi gamma dt   (Eq. sources, Eq. rhoD),
//   omega[C] = 1 / tau[C] (BGK collision frequency).
struct StepCoef {
    double dl[5];
    double bdt, kE, kI, kR, kD;
    double omega[4];
    bool diffuse_d;  // d[4] != 0
};

// Launch shape of the y-marching kernel.
struct MarchShape {
    int rows_per_wave;  // output rows each wavefront produces
    int cols_per_lane;  // adjacent columns per lane: 1 or 2
};

// ---- host helpers (sslbm_api.cpp) ---------------------------------------
// Validate parameters and derive the per-step constants (SSLBM status code).
sslbm_status derive_coef(const sslbm_params *p, StepCoef *k);
// How a run of nsteps splits into passes of at most K steps: the fewest
// passes, made even where that leaves every pass a step (so that ping-pong
// buffers end where they started), with the steps spread as evenly as possible over them (the
// first `longer` passes take one step more than the rest). A pass costs
// about the same HBM traffic whatever its depth, so a short tail pass would
// waste most of one.
struct PassPlan {
    long long count = 0;   // passes
    int base = 0;          // steps of the shorter passes
    long long longer = 0;  // passes with base + 1 steps (the first ones)
    int steps(long long i) const { return i < longer ? base + 1 : base; }
};
PassPlan plan_passes(long long nsteps, int K);

// One pass of k steps (1 <= k <= the register limit), in -> out, with the
// context's pass shape (SSLBM status code).
sslbm_status run_pass(sslbm_ctx *c, const void *in, void *out, int k, hipStream_t s);
// One pass of 4 steps in -> out writing the state after 2 steps to mid.
sslbm_status run_pass_mid2(sslbm_ctx *c, const void *in, void *mid, void *out, hipStream_t s);

// ---- launchers (sslbm_kernels.hip) --------------------------------------
// K steps in one pass: in -> out (no overlap). K in 1..SSLBM_MAX_BLOCKING.
hipError_t launch_march(int dtype, const void *in, void *out, const GridDesc &g,
                        const StepCoef &k, int K, const MarchShape &shape, hipStream_t s);
// Largest steps-per-pass whose kernel fits the register budget.
int march_max_depth(int dtype, int cols_per_lane);
// A pass of K steps in -> out that also writes the state after MID steps to
// mid (no overlap among the three); K = 4, MID = 2 only (else
// hipErrorNotSupported).
hipError_t launch_march_mid(int dtype, const void *in, void *mid, void *out, const GridDesc &g,
                            const StepCoef &k, int K, int MID, const MarchShape &shape,
                            hipStream_t s);
// Output columns of one wavefront strip at K steps per pass.
int strip_width(int K, int cols_per_lane);
// Wavefronts of the K-step pass kernel resident on the current device at
// once (occupancy x CUs), 0 when no device can be queried.
int march_resident_waves(int dtype, int K, int cols_per_lane, bool diffuse_d);

// ---- launchers (bgk_kernels.hip) ----------------------------------------
hipError_t launch_bgk_init(int dtype, const void *rho, void *f, void *rhoD, const GridDesc &g,
                           hipStream_t s);
hipError_t launch_bgk_step(int dtype, const void *f_in, const void *rhoD_in, void *f_out,
                           void *rhoD_out, const GridDesc &g, const StepCoef &k, hipStream_t s);
hipError_t launch_bgk_density(int dtype, const void *f, const void *rhoD, void *rho,
                              const GridDesc &g, hipStream_t s);

// ---- launchers (reduce_kernels.hip) -------------------------------------
// Number of partial blocks the total reduction uses (partials: blocks x 5 doubles).
int total_blocks(const GridDesc &g);
hipError_t launch_total(int dtype, const void *rho, const GridDesc &g, double *partials,
                        int blocks, double *out5_device, hipStream_t s);

}  // namespace sslbm

// The state behind the opaque sslbm_ctx handle.
struct sslbm_ctx {
    int nx = 0, ny = 0, dtype = 0, bc = 0;
    sslbm_params p{};
    sslbm::StepCoef coef{};
    sslbm_launch launch{};  // requested pass shape; zero fields = automatic
    int last_hip = 0;
    double *partials = nullptr;  // device buffer of sslbm_total
    int partial_blocks = 0;
    int partial_device = -1;
    double *adj_partials = nullptr;  // device slots of sslbm_adjoint_step
    long long adj_slots = 0;
    int adj_device = -1;
};
