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
// Size of one packed instance record for dtype, and packing of one record.
size_t ensemble_instance_bytes(int dtype);
void ensemble_pack_instance(int dtype, void *dst, long long offset, int nx, int ny,
                            const StepCoef &k);

}  // namespace sslbm
