// ensemble_kernels.hip -- one pass (K SSLBM steps) over many independent
// grids of different sizes in a single launch. Each wavefront takes one tile
// (instance, strip, rows) from a tile table and runs the same march as the
// single-grid kernel on that instance's buffer with that instance's
// coefficients; results are bit for bit those of the single-grid kernel.
#include <hip/hip_runtime.h>

#include "ensemble_internal.h"
#include "march_core.h"

namespace sslbm {

template <typename T>
struct EnsInstance {
    long long offset;  // elements from the start of the state buffer
    int nx, ny;
    Coef<T> k;
};

template <typename T, int K, bool DIFFUSE_D, int V>
__global__ __launch_bounds__(BLOCK_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
void ensemble_march_kernel(const T *__restrict__ in, T *__restrict__ out,
                           const EnsTile *__restrict__ tiles,
                           const EnsInstance<T> *__restrict__ insts, int ntiles, int bc) {
    const int wave = __builtin_amdgcn_readfirstlane(
        xcd_tile(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + (threadIdx.x >> 6));
    if (wave >= ntiles)
        return;  // whole wavefront leaves together
    const EnsTile t = tiles[wave];
    const EnsInstance<T> m = insts[t.inst];
    GridDesc g;
    g.nx = m.nx;
    g.ny = m.ny;
    g.plane = (long long)m.nx * m.ny;
    g.bc = bc;
    march_tile<T, K, DIFFUSE_D, V>(in + m.offset, out + m.offset, g, m.k, t.x0, t.y0, t.y1,
                                   t.up != 0);
}

template <typename T, int K, bool DD, int V>
static hipError_t launch_ek(const void *in, void *out, const EnsTile *tiles, int ntiles,
                            const void *insts, int bc, hipStream_t st) {
    if constexpr (!march_fits<T, K, V>()) {
        return hipErrorInvalidValue;
    } else {
        const int blocks = (ntiles + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
        hipLaunchKernelGGL((ensemble_march_kernel<T, K, DD, V>), dim3((unsigned)blocks),
                           dim3(BLOCK_THREADS), 0, st, static_cast<const T *>(in),
                           static_cast<T *>(out), tiles,
                           static_cast<const EnsInstance<T> *>(insts), ntiles, bc);
        return hipGetLastError();
    }
}

template <typename T, bool DD, int V>
static hipError_t dispatch_ek(const void *in, void *out, const EnsTile *tiles, int ntiles,
                              const void *insts, int bc, int K, hipStream_t st) {
    switch (K) {
    case 1: return launch_ek<T, 1, DD, V>(in, out, tiles, ntiles, insts, bc, st);
    case 2: return launch_ek<T, 2, DD, V>(in, out, tiles, ntiles, insts, bc, st);
    case 3: return launch_ek<T, 3, DD, V>(in, out, tiles, ntiles, insts, bc, st);
    case 4: return launch_ek<T, 4, DD, V>(in, out, tiles, ntiles, insts, bc, st);
    case 5: return launch_ek<T, 5, DD, V>(in, out, tiles, ntiles, insts, bc, st);
    case 6: return launch_ek<T, 6, DD, V>(in, out, tiles, ntiles, insts, bc, st);
    case 7: return launch_ek<T, 7, DD, V>(in, out, tiles, ntiles, insts, bc, st);
    case 8: return launch_ek<T, 8, DD, V>(in, out, tiles, ntiles, insts, bc, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ensemble(int dtype, const void *in, void *out, const EnsTile *tiles,
                           int ntiles, const void *insts, int bc, int K, int V, bool diffuse_d,
                           hipStream_t s) {
    if (ntiles <= 0)
        return hipSuccess;
    if (dtype == SSLBM_F32) {
        if (V == 2)
            return diffuse_d ? dispatch_ek<float, true, 2>(in, out, tiles, ntiles, insts, bc, K, s)
                             : dispatch_ek<float, false, 2>(in, out, tiles, ntiles, insts, bc, K, s);
        return diffuse_d ? dispatch_ek<float, true, 1>(in, out, tiles, ntiles, insts, bc, K, s)
                         : dispatch_ek<float, false, 1>(in, out, tiles, ntiles, insts, bc, K, s);
    }
    if (V == 2)
        return diffuse_d ? dispatch_ek<double, true, 2>(in, out, tiles, ntiles, insts, bc, K, s)
                         : dispatch_ek<double, false, 2>(in, out, tiles, ntiles, insts, bc, K, s);
    return diffuse_d ? dispatch_ek<double, true, 1>(in, out, tiles, ntiles, insts, bc, K, s)
                     : dispatch_ek<double, false, 1>(in, out, tiles, ntiles, insts, bc, K, s);
}

size_t ensemble_instance_bytes(int dtype) {
    return dtype == SSLBM_F32 ? sizeof(EnsInstance<float>) : sizeof(EnsInstance<double>);
}

void ensemble_pack_instance(int dtype, void *dst, long long offset, int nx, int ny,
                            const StepCoef &k) {
    if (dtype == SSLBM_F32) {
        EnsInstance<float> m;
        m.offset = offset;
        m.nx = nx;
        m.ny = ny;
        m.k = cast_coef<float>(k);
        *static_cast<EnsInstance<float> *>(dst) = m;
    } else {
        EnsInstance<double> m;
        m.offset = offset;
        m.nx = nx;
        m.ny = ny;
        m.k = cast_coef<double>(k);
        *static_cast<EnsInstance<double> *>(dst) = m;
    }
}

}  // namespace sslbm
