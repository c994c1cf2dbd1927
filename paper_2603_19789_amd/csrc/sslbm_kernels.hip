// sslbm_kernels.hip -- the SSLBM SEIRD step on gfx950: K time steps per pass
// over HBM with a y-marching wavefront.
//
// Layout: rho[5][ny][nx], structure of arrays, x fastest (one coalesced
// 64-lane row segment per field and row).
//
// Design. One wavefront owns a strip of 64 consecutive columns (one column
// per lane) and walks down a chunk of rows. For every level k = 0..K-1 it
// keeps the last three rows of that level in registers (a rolling window);
// level 0 is read from HBM one row ahead of use, levels 1..K are computed
// from the window of the level below, and level K is written to HBM. East and
// west neighbours come from the adjacent lanes through DPP wave shifts; north
// and south neighbours are in the lane's own window. No LDS and no barrier is
// needed: wavefronts are independent.
//
// Halos are recomputed rather than exchanged: after k levels only lanes at
// least k columns from the strip edge hold valid values, so a strip yields
// 64 - 2K output columns, and a chunk starts K rows above its first output
// row. Each pass therefore reads every field about once (plus halo rows and
// columns, which neighbouring strips of the same XCD share through L2) and
// writes it once, while doing K steps of arithmetic.
#include <hip/hip_runtime.h>

#include "seird_device.h"
#include "sslbm_internal.h"

namespace sslbm {

constexpr int WAVES_PER_BLOCK = 4;
constexpr int BLOCK_THREADS = 64 * WAVES_PER_BLOCK;

template <typename T, int K, bool DIFFUSE_D>
__global__ __launch_bounds__(BLOCK_THREADS) void sslbm_march_kernel(
    const T *__restrict__ in, T *__restrict__ out, GridDesc g, Coef<T> k, int rows_per_wave,
    int strips, int total_waves) {
    constexpr int WU = 64 - 2 * K;  // output columns per strip
    const int lane = threadIdx.x & 63;
    const int wave = xcd_tile(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + (threadIdx.x >> 6);
    if (wave >= total_waves)
        return;  // whole wavefront leaves together
    const int strip = wave % strips;
    const int chunk = wave / strips;

    const int xl = strip * WU - K + lane;           // logical column of this lane
    const int xm = map_index(xl, g.nx, g.bc);       // column in memory
    const bool out_lane = lane >= K && lane < 64 - K && xl < g.nx;
    const int y0 = chunk * rows_per_wave;
    const int y1 = min(y0 + rows_per_wave, g.ny);   // output rows [y0, y1)

    // win[l][r][C]: rows j-l-2, j-l-1, j-l of level l after iteration j
    T win[K][3][5];
#pragma unroll
    for (int l = 0; l < K; ++l)
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 5; ++c)
                win[l][r][c] = T(0);

    const long long plane = g.plane;
    auto load_row = [&](int j, T v[5]) {
        const long long base = (long long)map_index(j, g.ny, g.bc) * g.nx + xm;
#pragma unroll
        for (int c = 0; c < 5; ++c)
            v[c] = in[c * plane + base];
    };

    T pre[5];
    load_row(y0 - K, pre);
    for (int j = y0 - K; j < y1 + K; ++j) {
        // level 0: the prefetched row j enters the window; fetch row j + 1
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            win[0][0][c] = win[0][1][c];
            win[0][1][c] = win[0][2][c];
            win[0][2][c] = pre[c];
        }
        if (j + 1 < y1 + K)
            load_row(j + 1, pre);

#pragma unroll
        for (int l = 1; l <= K; ++l) {
            // level l produces row j - l; its first needed row is y0 - K + l
            if (j < y0 - K + 2 * l)
                continue;  // uniform across the wavefront
            T cen[5], nb[5], res[5];
#pragma unroll
            for (int c = 0; c < 5; ++c) {
                cen[c] = win[l - 1][1][c];
                if (c < 4 || DIFFUSE_D) {
                    const T west = lane_from_left(cen[c]);
                    const T east = lane_from_right(cen[c]);
                    nb[c] = (win[l - 1][0][c] + win[l - 1][2][c]) + (east + west);
                } else {
                    nb[c] = T(0);
                }
            }
            seird_update<T, DIFFUSE_D>(cen, nb, k, res);
            if (l < K) {
#pragma unroll
                for (int c = 0; c < 5; ++c) {
                    win[l][0][c] = win[l][1][c];
                    win[l][1][c] = win[l][2][c];
                    win[l][2][c] = res[c];
                }
            } else if (out_lane) {
                const long long base = (long long)(j - K) * g.nx + xl;
#pragma unroll
                for (int c = 0; c < 5; ++c)
                    out[c * plane + base] = res[c];
            }
        }
    }
}

template <typename T>
static Coef<T> cast_coef(const StepCoef &s) {
    Coef<T> k;
    for (int c = 0; c < 5; ++c)
        k.dl[c] = (T)s.dl[c];
    k.bdt = (T)s.bdt;
    k.kE = (T)s.kE;
    k.kI = (T)s.kI;
    k.kR = (T)s.kR;
    k.kD = (T)s.kD;
    return k;
}

template <typename T, int K, bool DD>
static hipError_t launch_k(const void *in, void *out, const GridDesc &g, const StepCoef &s,
                           const MarchShape &shape, hipStream_t st) {
    constexpr int WU = 64 - 2 * K;
    const int strips = (g.nx + WU - 1) / WU;
    const int chunks = (g.ny + shape.rows_per_wave - 1) / shape.rows_per_wave;
    const long long waves = (long long)strips * chunks;
    const long long blocks = (waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
    if (waves > 0x7fffffffll)
        return hipErrorInvalidConfiguration;
    hipLaunchKernelGGL((sslbm_march_kernel<T, K, DD>), dim3((unsigned)blocks),
                       dim3(BLOCK_THREADS), 0, st, static_cast<const T *>(in),
                       static_cast<T *>(out), g, cast_coef<T>(s), shape.rows_per_wave, strips,
                       (int)waves);
    return hipGetLastError();
}

template <typename T, bool DD>
static hipError_t dispatch_k(const void *in, void *out, const GridDesc &g, const StepCoef &s,
                             int K, const MarchShape &shape, hipStream_t st) {
    switch (K) {
    case 1: return launch_k<T, 1, DD>(in, out, g, s, shape, st);
    case 2: return launch_k<T, 2, DD>(in, out, g, s, shape, st);
    case 3: return launch_k<T, 3, DD>(in, out, g, s, shape, st);
    case 4: return launch_k<T, 4, DD>(in, out, g, s, shape, st);
    case 5: return launch_k<T, 5, DD>(in, out, g, s, shape, st);
    case 6: return launch_k<T, 6, DD>(in, out, g, s, shape, st);
    case 7: return launch_k<T, 7, DD>(in, out, g, s, shape, st);
    case 8: return launch_k<T, 8, DD>(in, out, g, s, shape, st);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_march(int dtype, const void *in, void *out, const GridDesc &g,
                        const StepCoef &k, int K, const MarchShape &shape, hipStream_t s) {
    if (dtype == SSLBM_F32)
        return k.diffuse_d ? dispatch_k<float, true>(in, out, g, k, K, shape, s)
                           : dispatch_k<float, false>(in, out, g, k, K, shape, s);
    return k.diffuse_d ? dispatch_k<double, true>(in, out, g, k, K, shape, s)
                       : dispatch_k<double, false>(in, out, g, k, K, shape, s);
}

}  // namespace sslbm
