// ensemble_internal.h -- declarations shared by the ensemble host code and
// the ensemble kernels (not part of the ABI).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>

#include "sslbm_internal.h"

namespace sslbm {

// One wavefront's work in an ensemble pass: instance, first output column
// of its strip, output rows [y0, y1), marching up (odd chunks) or down.
struct EnsTile {
    int inst, x0, y0, y1, up;
};

// One pass of K steps over every tile: in -> out (whole ensemble buffers).
// insts is a device table of packed instance records (ensemble_pack_instance).
hipError_t launch_ensemble(int dtype, const void *in, void *out, const EnsTile *tiles,
                           int ntiles, const void *insts, int bc, int K, int V, bool diffuse_d,
                           hipStream_t s);
// Instances whose five fields fit ENS_LDS_BYTES of LDS (64 x 64 in FP32)
// run all nsteps steps on chip, one workgroup each: lds_inst is a device
// array of `count` instance indices; lds_bytes (the largest such instance,
// 5 nx ny elements) is the dynamic LDS of each workgroup. In place in state.
constexpr int ENS_LDS_BYTES = 81920;
hipError_t launch_ensemble_lds(int dtype, void *state, const int *lds_inst, int count,
                               const void *insts, int bc, long long nsteps, bool diffuse_d,
                               size_t lds_bytes, hipStream_t s);
// Size of one packed instance record for dtype, and packing of one record.
size_t ensemble_instance_bytes(int dtype);
void ensemble_pack_instance(int dtype, void *dst, long long offset, int nx, int ny,
                            const StepCoef &k);

}  // namespace sslbm
