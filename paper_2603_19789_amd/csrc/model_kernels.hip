// model_kernels.hip -- host side of the generic-model pass kernels: launch
// shape, dispatch over arithmetic type and lattice, and the device
// transition table. The kernels are in model_march.h.
#include <hip/hip_runtime_api.h>

#include "march_core.h"
#include "model_internal.h"

namespace sslbm {

ModelShape model_shape(int nx, int ny, int K) {
    // two workgroups of four wavefronts per CU (two wavefronts per SIMD hide
    // each other's LDS and memory waits), chunks of at least 2K and 8 rows;
    // measured at 4096 x 4096 with six compartments and one step per pass:
    // 56 GLUPS with one wavefront per SIMD, 73 with two, 66 with four
    // (shorter chunks, more halo rows)
    ModelShape s;
    const int wu = 64 - 2 * K;
    s.strips = (nx + wu - 1) / wu;
    long long chunks = (2 * 256 * WAVES_PER_BLOCK) / s.strips;
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
