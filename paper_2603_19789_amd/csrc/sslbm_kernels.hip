// sslbm_kernels.hip -- the single-grid pass kernel (K steps of the SSLBM
// SEIRD step per pass over HBM) and its launch helpers. The pass itself is in
// march_core.h.
#include <hip/hip_runtime.h>

#include "march_core.h"

namespace sslbm {

// At least two wavefronts per SIMD (at most 256 VGPRs each): with one, a
// SIMD idles whenever its only wavefront waits for memory.
template <typename T, int K, bool DIFFUSE_D, int V>
__global__ __launch_bounds__(BLOCK_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
void sslbm_march_kernel(
    const T *__restrict__ in, T *__restrict__ out, GridDesc g, Coef<T> k, int rows_per_wave,
    int strips, int total_waves) {
    // wavefront-uniform from here on: keep it in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(
        xcd_tile(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + (threadIdx.x >> 6));
    if (wave >= total_waves)
        return;  // whole wavefront leaves together
    const int strip = wave % strips;
    const int chunk = wave / strips;
    const int y0 = chunk * rows_per_wave;
    march_tile<T, K, DIFFUSE_D, V>(in, out, g, k, strip * Strip<K, V>::WU, y0,
                                   min(y0 + rows_per_wave, g.ny), (chunk & 1) != 0);
}

// The same pass, writing the state after MID steps to `mid` as well: the
// checkpoints of a recorded run, two per pass over HBM.
template <typename T, int K, bool DIFFUSE_D, int V, int MID>
__global__ __launch_bounds__(BLOCK_THREADS) __attribute__((amdgpu_waves_per_eu(2)))
void sslbm_march_mid_kernel(
    const T *__restrict__ in, T *__restrict__ mid, T *__restrict__ out, GridDesc g, Coef<T> k,
    int rows_per_wave, int strips, int total_waves) {
    const int wave = __builtin_amdgcn_readfirstlane(
        xcd_tile(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + (threadIdx.x >> 6));
    if (wave >= total_waves)
        return;  // whole wavefront leaves together
    const int strip = wave % strips;
    const int chunk = wave / strips;
    const int y0 = chunk * rows_per_wave;
    march_tile<T, K, DIFFUSE_D, V, MID>(in, out, g, k, strip * Strip<K, V>::WU, y0,
                                        min(y0 + rows_per_wave, g.ny), (chunk & 1) != 0, mid);
}

template <typename T, int K, bool DD, int V>
static hipError_t launch_k(const void *in, void *out, const GridDesc &g, const StepCoef &s,
                           const MarchShape &shape, hipStream_t st) {
    if constexpr (!march_fits<T, K, V>()) {
        return hipErrorInvalidValue;
    } else {
        constexpr int WU = Strip<K, V>::WU;
        const int strips = (g.nx + WU - 1) / WU;
        const int chunks = (g.ny + shape.rows_per_wave - 1) / shape.rows_per_wave;
        const long long waves = (long long)strips * chunks;
        const long long blocks = (waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
        if (waves > 0x7fffffffll)
            return hipErrorInvalidConfiguration;
        hipLaunchKernelGGL((sslbm_march_kernel<T, K, DD, V>), dim3((unsigned)blocks),
                           dim3(BLOCK_THREADS), 0, st, static_cast<const T *>(in),
                           static_cast<T *>(out), g, cast_coef<T>(s), shape.rows_per_wave,
                           strips, (int)waves);
        return hipGetLastError();
    }
}

template <typename T, bool DD, int V>
static hipError_t dispatch_k(const void *in, void *out, const GridDesc &g, const StepCoef &s,
                             int K, const MarchShape &shape, hipStream_t st) {
    switch (K) {
    case 1: return launch_k<T, 1, DD, V>(in, out, g, s, shape, st);
    case 2: return launch_k<T, 2, DD, V>(in, out, g, s, shape, st);
    case 3: return launch_k<T, 3, DD, V>(in, out, g, s, shape, st);
    case 4: return launch_k<T, 4, DD, V>(in, out, g, s, shape, st);
    case 5: return launch_k<T, 5, DD, V>(in, out, g, s, shape, st);
    case 6: return launch_k<T, 6, DD, V>(in, out, g, s, shape, st);
    case 7: return launch_k<T, 7, DD, V>(in, out, g, s, shape, st);
    case 8: return launch_k<T, 8, DD, V>(in, out, g, s, shape, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, bool DD>
static hipError_t dispatch_v(const void *in, void *out, const GridDesc &g, const StepCoef &s,
                             int K, const MarchShape &shape, hipStream_t st) {
    if (shape.cols_per_lane == 2)
        return dispatch_k<T, DD, 2>(in, out, g, s, K, shape, st);
    return dispatch_k<T, DD, 1>(in, out, g, s, K, shape, st);
}

hipError_t launch_march(int dtype, const void *in, void *out, const GridDesc &g,
                        const StepCoef &k, int K, const MarchShape &shape, hipStream_t s) {
    if (dtype == SSLBM_F32)
        return k.diffuse_d ? dispatch_v<float, true>(in, out, g, k, K, shape, s)
                           : dispatch_v<float, false>(in, out, g, k, K, shape, s);
    return k.diffuse_d ? dispatch_v<double, true>(in, out, g, k, K, shape, s)
                       : dispatch_v<double, false>(in, out, g, k, K, shape, s);
}

template <typename T, bool DD, int V>
static hipError_t launch_mid_t(const void *in, void *mid, void *out, const GridDesc &g,
                               const StepCoef &s, const MarchShape &shape, hipStream_t st) {
    constexpr int K = 4, MID = 2;
    if constexpr (!march_fits<T, K, V>()) {
        return hipErrorInvalidValue;
    } else {
        constexpr int WU = Strip<K, V>::WU;
        const int strips = (g.nx + WU - 1) / WU;
        const int chunks = (g.ny + shape.rows_per_wave - 1) / shape.rows_per_wave;
        const long long waves = (long long)strips * chunks;
        const long long blocks = (waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
        if (waves > 0x7fffffffll)
            return hipErrorInvalidConfiguration;
        hipLaunchKernelGGL((sslbm_march_mid_kernel<T, K, DD, V, MID>), dim3((unsigned)blocks),
                           dim3(BLOCK_THREADS), 0, st, static_cast<const T *>(in),
                           static_cast<T *>(mid), static_cast<T *>(out), g, cast_coef<T>(s),
                           shape.rows_per_wave, strips, (int)waves);
        return hipGetLastError();
    }
}

hipError_t launch_march_mid(int dtype, const void *in, void *mid, void *out, const GridDesc &g,
                            const StepCoef &k, int K, int MID, const MarchShape &shape,
                            hipStream_t s) {
    if (K != 4 || MID != 2)
        return hipErrorNotSupported;
    const bool v2 = shape.cols_per_lane == 2;
    if (dtype == SSLBM_F32) {
        if (k.diffuse_d)
            return v2 ? launch_mid_t<float, true, 2>(in, mid, out, g, k, shape, s)
                      : launch_mid_t<float, true, 1>(in, mid, out, g, k, shape, s);
        return v2 ? launch_mid_t<float, false, 2>(in, mid, out, g, k, shape, s)
                  : launch_mid_t<float, false, 1>(in, mid, out, g, k, shape, s);
    }
    if (k.diffuse_d)
        return v2 ? launch_mid_t<double, true, 2>(in, mid, out, g, k, shape, s)
                  : launch_mid_t<double, true, 1>(in, mid, out, g, k, shape, s);
    return v2 ? launch_mid_t<double, false, 2>(in, mid, out, g, k, shape, s)
              : launch_mid_t<double, false, 1>(in, mid, out, g, k, shape, s);
}

int strip_width(int K, int cols_per_lane) {
    const int hx = (K + cols_per_lane - 1) / cols_per_lane * cols_per_lane;
    return 64 * cols_per_lane - 2 * hx;
}

template <typename T, bool DD, int V>
static const void *kernel_of(int K) {
    const void *f = nullptr;
    if constexpr (march_fits<T, 1, V>()) if (K == 1) f = (const void *)sslbm_march_kernel<T, 1, DD, V>;
    if constexpr (march_fits<T, 2, V>()) if (K == 2) f = (const void *)sslbm_march_kernel<T, 2, DD, V>;
    if constexpr (march_fits<T, 3, V>()) if (K == 3) f = (const void *)sslbm_march_kernel<T, 3, DD, V>;
    if constexpr (march_fits<T, 4, V>()) if (K == 4) f = (const void *)sslbm_march_kernel<T, 4, DD, V>;
    if constexpr (march_fits<T, 5, V>()) if (K == 5) f = (const void *)sslbm_march_kernel<T, 5, DD, V>;
    if constexpr (march_fits<T, 6, V>()) if (K == 6) f = (const void *)sslbm_march_kernel<T, 6, DD, V>;
    if constexpr (march_fits<T, 7, V>()) if (K == 7) f = (const void *)sslbm_march_kernel<T, 7, DD, V>;
    if constexpr (march_fits<T, 8, V>()) if (K == 8) f = (const void *)sslbm_march_kernel<T, 8, DD, V>;
    return f;
}

template <typename T, bool DD>
static const void *kernel_of_v(int K, int V) {
    return V == 2 ? kernel_of<T, DD, 2>(K) : kernel_of<T, DD, 1>(K);
}

int march_resident_waves(int dtype, int K, int cols_per_lane, bool diffuse_d) {
    // cached per (device, dtype, V, K, diffuse_d)
    static int cache[16][2][2][SSLBM_MAX_BLOCKING + 1][2] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16 || K < 1 ||
        K > SSLBM_MAX_BLOCKING || cols_per_lane < 1 || cols_per_lane > 2)
        return 0;
    int &slot = cache[dev][dtype == SSLBM_F64][cols_per_lane - 1][K][diffuse_d ? 1 : 0];
    if (slot)
        return slot;
    const void *f =
        dtype == SSLBM_F32
            ? (diffuse_d ? kernel_of_v<float, true>(K, cols_per_lane)
                         : kernel_of_v<float, false>(K, cols_per_lane))
            : (diffuse_d ? kernel_of_v<double, true>(K, cols_per_lane)
                         : kernel_of_v<double, false>(K, cols_per_lane));
    // occupancy from the kernel's register count: 512 VGPRs per SIMD lane,
    // allocated in granules of 8, at most 8 wavefronts per SIMD
    hipFuncAttributes attr;
    int cus = 0;
    if (!f || hipFuncGetAttributes(&attr, f) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    const int regs = (attr.numRegs + 7) / 8 * 8;
    int per_simd = regs > 0 ? 512 / regs : 8;
    if (per_simd > 8)
        per_simd = 8;
    if (per_simd < 1)
        per_simd = 1;
    slot = per_simd * 4 * cus;
    return slot;
}

template <typename T, int V>
static int max_depth() {
    int K = 0;
    if (march_fits<T, 1, V>()) K = 1;
    if (march_fits<T, 2, V>()) K = 2;
    if (march_fits<T, 3, V>()) K = 3;
    if (march_fits<T, 4, V>()) K = 4;
    if (march_fits<T, 5, V>()) K = 5;
    if (march_fits<T, 6, V>()) K = 6;
    if (march_fits<T, 7, V>()) K = 7;
    if (march_fits<T, 8, V>()) K = 8;
    return K;
}

int march_max_depth(int dtype, int cols_per_lane) {
    if (cols_per_lane == 2)
        return dtype == SSLBM_F32 ? max_depth<float, 2>() : max_depth<double, 2>();
    return dtype == SSLBM_F32 ? max_depth<float, 1>() : max_depth<double, 1>();
}

}  // namespace sslbm
