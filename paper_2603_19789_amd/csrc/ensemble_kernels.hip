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

// ---------------------------------------------------------------------------
// Instances small enough for the LDS of one workgroup (5 nx ny elements in
// ENS_LDS_BYTES: 64 x 64 in FP32) stay on chip for the whole run: one
// workgroup per instance reads it once, takes every step in LDS and writes it
// back once. A step: each thread forms the updates of its cells (cells
// tid, tid + 512, ...) into registers from the LDS values of the previous
// step, then, after a barrier, writes them over them. The neighbour sum is
// (north + south) + (east + west) and the update is seird_update, as in the
// pass kernels, so results are those of sslbm_run bit for bit.
constexpr int ENS_LDS_THREADS = 512;

template <typename T>
constexpr int lds_cells_per_thread() {
    return ENS_LDS_BYTES / (5 * (int)sizeof(T)) / ENS_LDS_THREADS;
}

// Eight wavefronts per workgroup, at most 256 VGPRs each (the updates of a
// thread's eight cells wait in registers for the barrier): one instance per
// CU at a time, which leaves the other half of the CU's LDS and most of its
// registers to other kernels.
template <typename T, bool DIFFUSE_D>
__global__ __launch_bounds__(ENS_LDS_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
void ensemble_lds_kernel(
    T *__restrict__ state, const int *__restrict__ lds_inst,
    const EnsInstance<T> *__restrict__ insts, int bc, long long nsteps) {
    extern __shared__ __align__(16) unsigned char lds_bytes[];
    T *s = reinterpret_cast<T *>(lds_bytes);
    const EnsInstance<T> m = insts[lds_inst[blockIdx.x]];
    const int nx = m.nx, ny = m.ny, n = nx * ny;
    T *g = state + m.offset;
    const int tid = threadIdx.x;
    for (int i = tid; i < 5 * n; i += ENS_LDS_THREADS)
        s[i] = g[i];

    constexpr int CPT = lds_cells_per_thread<T>();
    int nbr[CPT][4];  // north, south, east, west cell indices
#pragma unroll
    for (int j = 0; j < CPT; ++j) {
        const int cell = tid + j * ENS_LDS_THREADS;
        const int x = cell < n ? cell % nx : 0, y = cell < n ? cell / nx : 0;
        nbr[j][0] = map_index(y - 1, ny, bc) * nx + x;
        nbr[j][1] = map_index(y + 1, ny, bc) * nx + x;
        nbr[j][2] = y * nx + map_index(x + 1, nx, bc);
        nbr[j][3] = y * nx + map_index(x - 1, nx, bc);
    }
    __syncthreads();
    for (long long t = 0; t < nsteps; ++t) {
        T out[CPT][5];
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int cell = tid + j * ENS_LDS_THREADS;
            if (cell < n) {
                T cen[5], nb[5];
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    const T *f = s + c * n;
                    cen[c] = f[cell];
                    nb[c] = (c < 4 || DIFFUSE_D)
                                ? (f[nbr[j][0]] + f[nbr[j][1]]) + (f[nbr[j][2]] + f[nbr[j][3]])
                                : T(0);
                }
                seird_update<T, DIFFUSE_D>(cen, nb, m.k, out[j]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < CPT; ++j) {
            const int cell = tid + j * ENS_LDS_THREADS;
            if (cell < n) {
#pragma unroll
                for (int c = 0; c < 5; ++c)
                    s[c * n + cell] = out[j][c];
            }
        }
        __syncthreads();
    }
    for (int i = tid; i < 5 * n; i += ENS_LDS_THREADS)
        g[i] = s[i];
}

template <typename T, bool DD>
static hipError_t launch_lds_t(void *state, const int *lds_inst, int count, const void *insts,
                               int bc, long long nsteps, size_t lds_bytes, hipStream_t st) {
    hipLaunchKernelGGL((ensemble_lds_kernel<T, DD>), dim3((unsigned)count),
                       dim3(ENS_LDS_THREADS), lds_bytes, st, static_cast<T *>(state), lds_inst,
                       static_cast<const EnsInstance<T> *>(insts), bc, nsteps);
    return hipGetLastError();
}

hipError_t launch_ensemble_lds(int dtype, void *state, const int *lds_inst, int count,
                               const void *insts, int bc, long long nsteps, bool diffuse_d,
                               size_t lds_bytes, hipStream_t s) {
    if (count <= 0 || nsteps <= 0)
        return hipSuccess;
    if (lds_bytes > (size_t)ENS_LDS_BYTES)
        return hipErrorInvalidValue;
    if (dtype == SSLBM_F32)
        return diffuse_d ? launch_lds_t<float, true>(state, lds_inst, count, insts, bc, nsteps,
                                                     lds_bytes, s)
                         : launch_lds_t<float, false>(state, lds_inst, count, insts, bc, nsteps,
                                                      lds_bytes, s);
    return diffuse_d ? launch_lds_t<double, true>(state, lds_inst, count, insts, bc, nsteps,
                                                  lds_bytes, s)
                     : launch_lds_t<double, false>(state, lds_inst, count, insts, bc, nsteps,
                                                   lds_bytes, s);
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
