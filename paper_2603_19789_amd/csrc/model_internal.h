// model_internal.h -- declarations shared by the generic-model entry points
// and kernels (not part of the ABI).
#pragma once

#include <hip/hip_runtime_api.h>

#include "sslbm_internal.h"

namespace sslbm {

constexpr int MODEL_MAX_C = SSLBM_MAX_COMPARTMENTS;
constexpr int MODEL_MAX_T = SSLBM_MAX_TRANSITIONS;
// device transition table: MODEL_MAX_T int4 records, then MODEL_MAX_T rows
// of MODEL_MAX_C stoichiometry values
constexpr size_t model_table_bytes(int dtype) {
    return (size_t)MODEL_MAX_T * 16 +
           (size_t)MODEL_MAX_T * MODEL_MAX_C * (dtype == SSLBM_F32 ? 4 : 8);
}

// Per-step constants passed to the kernel in the arithmetic type: dl =
// d dt / dx^2 (divided by 6 on D2Q9); counted = bit mask of the compartments
// summed into N. The transitions travel in a device table (model_table).
template <typename T>
struct ModelCoef {
    T dl[MODEL_MAX_C];
    int m, ntrans;
    unsigned counted;
};

// The same in FP64, derived once on the host.
struct ModelCoefHost {
    double dl[MODEL_MAX_C];
    double rate_dt[MODEL_MAX_T];
    int src[MODEL_MAX_T], dst[MODEL_MAX_T], cat[MODEL_MAX_T], freq[MODEL_MAX_T];
    int m, ntrans;
    unsigned counted;
};

struct ModelShape {
    int strips, chunks, rows;
};

// Steps per pass the kernels are built for (1..MODEL_MAX_K).
constexpr int MODEL_MAX_K = SSLBM_MODEL_MAX_BLOCKING;

// At most this many wavefronts per SIMD are asked for (the largest count
// measured to help).
constexpr int MODEL_MAX_WAVES_PER_SIMD = 4;

// Launch shape of a pass of K steps whose kernel fits resident_per_simd
// wavefronts per SIMD.
ModelShape model_shape(int nx, int ny, int K, int resident_per_simd);
// One pass of K steps, in -> out.
hipError_t launch_model(int dtype, int lattice, const void *in, void *out, const GridDesc &g,
                        const ModelCoefHost &h, const void *table, int K, hipStream_t s);
// The kernels of one arithmetic type and lattice (one translation unit each).
hipError_t launch_model_f32_d2q5(const void *in, void *out, const GridDesc &g,
                                 const ModelCoefHost &h, const void *table, int K, hipStream_t s);
hipError_t launch_model_f32_d2q9(const void *in, void *out, const GridDesc &g,
                                 const ModelCoefHost &h, const void *table, int K, hipStream_t s);
hipError_t launch_model_f64_d2q5(const void *in, void *out, const GridDesc &g,
                                 const ModelCoefHost &h, const void *table, int K, hipStream_t s);
hipError_t launch_model_f64_d2q9(const void *in, void *out, const GridDesc &g,
                                 const ModelCoefHost &h, const void *table, int K, hipStream_t s);
// The device table (model_table_bytes) written into host memory dst.
void model_table(const ModelCoefHost &h, int dtype, void *dst);

}  // namespace sslbm
