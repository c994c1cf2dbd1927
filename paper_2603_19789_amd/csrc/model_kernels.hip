// model_kernels.hip -- host side of the generic-model pass kernels: launch
// shape, dispatch over arithmetic type and lattice, and the device
// transition table. The kernels are in model_march.h.
#include <hip/hip_runtime_api.h>

#include "march_core.h"
#include "model_internal.h"

namespace sslbm {

ModelShape model_shape(int nx, int ny, int K, int resident_per_simd) {
    // As many wavefronts per SIMD as fit (so that they hide each other's LDS
    // and memory waits in one round), at most MODEL_MAX_WAVES_PER_SIMD, on
    // chunks of at least max(8, 2K) rows. Measured at 4096 x 4096 with six
    // compartments, FP32, three steps per pass: 124 / 156 / 165 GLUPS at
    // 2 / 3 / 4 wavefronts per SIMD; with one step per pass 56 / 73 / 66 at
    // 1 / 2 / 4 (shorter chunks, more halo rows). FP64 with four steps per
    // pass fits two (196 VGPRs): asking for three drops it from 77 to 65.
    ModelShape s;
    const int wu = 64 - 2 * K;
    s.strips = (nx + wu - 1) / wu;
    int per = resident_per_simd < MODEL_MAX_WAVES_PER_SIMD ? resident_per_simd
                                                           : MODEL_MAX_WAVES_PER_SIMD;
    if (K == 1 && per > 2)
        per = 2;
    if (per < 1)
        per = 1;
    long long chunks = ((long long)per * 256 * WAVES_PER_BLOCK) / s.strips;
    if (chunks < 1)
        chunks = 1;
    long long rows = (ny + chunks - 1) / chunks;
    if (rows < 8)
        rows = 8;
    if (rows < 2 * K)
        rows = 2 * K;
    if (rows > ny)
        rows = ny;
    s.rows = (int)rows;
    s.chunks = (int)((ny + rows - 1) / rows);
    return s;
}

hipError_t launch_model(int dtype, int lattice, const void *in, void *out, const GridDesc &g,
                        const ModelCoefHost &h, const void *table, int K, hipStream_t s) {
    if (K < 1 || K > MODEL_MAX_K)
        return hipErrorInvalidValue;
    if (dtype == SSLBM_F32)
        return lattice == 9 ? launch_model_f32_d2q9(in, out, g, h, table, K, s)
                            : launch_model_f32_d2q5(in, out, g, h, table, K, s);
    return lattice == 9 ? launch_model_f64_d2q9(in, out, g, h, table, K, s)
                        : launch_model_f64_d2q5(in, out, g, h, table, K, s);
}

void model_table(const ModelCoefHost &h, int dtype, void *dst) {
    // MODEL_MAX_T records {src, catalyst slot (m: the constant 1),
    // destination, frequency}, then MODEL_MAX_T stoichiometry rows of
    // MODEL_MAX_C values rate dt (delta_dst - delta_src); records past the
    // last transition are zero (the kernel reads the table in groups)
    int *ints = static_cast<int *>(dst);
    void *rows = ints + 4 * MODEL_MAX_T;
    for (int r = 0; r < MODEL_MAX_T; ++r) {
        const bool live = r < h.ntrans;
        ints[4 * r + 0] = live ? h.src[r] : 0;
        ints[4 * r + 1] = live && h.cat[r] >= 0 ? h.cat[r] : h.m;
        ints[4 * r + 2] = live ? h.dst[r] : -1;
        ints[4 * r + 3] = live ? h.freq[r] : 0;
        for (int c = 0; c < MODEL_MAX_C; ++c) {
            double v = 0.0;
            if (live && c == h.src[r])
                v = -h.rate_dt[r];
            if (live && c == h.dst[r])
                v = h.rate_dt[r];
            if (dtype == SSLBM_F32)
                static_cast<float *>(rows)[r * MODEL_MAX_C + c] = (float)v;
            else
                static_cast<double *>(rows)[r * MODEL_MAX_C + c] = v;
        }
    }
}

}  // namespace sslbm
