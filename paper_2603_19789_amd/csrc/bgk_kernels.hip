// bgk_kernels.hip -- the BGK lattice Boltzmann comparison scheme on gfx950
// (Eq. pdf): per node, read the 20 populations of S, E, I, R and rho^D,
// collide with f^eq = w_i rho and the source w_i Psi dt, and push each
// post-collision population to x + c_i (periodic wrap, or half-way
// bounce-back at a no-flux wall). One thread per node, rows of the grid on
// blockIdx.y (grids taller than the 65535 rows a launch can span take rows
// y, y + 65535, ... in one workgroup), so every population plane is read and
// written in coalesced 256-node row segments (the pushed ones shifted by one
// node). Stores keep
// the default cache policy: the pushed rows are shifted by one node, and L2
// merges the partial lines (non-temporal stores measured 5% slower).
#include <hip/hip_runtime.h>

#include "seird_device.h"
#include "sslbm_internal.h"

namespace sslbm {

constexpr int BGK_THREADS = 256;

template <typename T>
struct BgkCoef {
    Coef<T> k;
    T omega[4];  // 1 / tau for S, E, I, R
};

// D2Q5 weights, Sec. II.B
template <typename T>
__device__ __forceinline__ T weight(int i) {
    return i == 0 ? T(1) / T(3) : T(1) / T(6);
}

// Most rows a launch spans (the grid's y dimension).
constexpr int BGK_MAX_GRID_ROWS = 65535;

// One node (x, y): collide and push.
template <typename T>
__device__ __forceinline__ void bgk_node(const T *__restrict__ f_in, const T *__restrict__ d_in,
                                         T *__restrict__ f_out, T *__restrict__ d_out,
                                         const GridDesc &g, const BgkCoef<T> &k, int x, int y) {
    const long long plane = g.plane;
    const long long cell = (long long)y * g.nx + x;

    T f[4][5], rho[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        T s = T(0);
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            f[c][i] = f_in[(c * 5 + i) * plane + cell];
            s += f[c][i];
        }
        rho[c] = s;
    }
    const T dead = d_in[cell];
    T fdt, rE, rI;
    seird_increments(rho[0], rho[1], rho[2], rho[3], k.k, fdt, rE, rI);
    const T src[4] = {-fdt, fdt - rE, rE - rI, k.k.kR * rho[2]};

    // destinations of the five links; at a no-flux wall the population
    // returns to this node in the opposite direction
    constexpr int CX[5] = {0, 1, 0, -1, 0};
    constexpr int CY[5] = {0, 0, 1, 0, -1};
    constexpr int OPP[5] = {0, 3, 4, 1, 2};
    long long dest[5];
    int dir[5];
#pragma unroll
    for (int i = 0; i < 5; ++i) {
        int xd = x + CX[i], yd = y + CY[i];
        dir[i] = i;
        const bool outside = xd < 0 || xd >= g.nx || yd < 0 || yd >= g.ny;
        if (outside && g.bc == SSLBM_NOFLUX) {
            xd = x;
            yd = y;
            dir[i] = OPP[i];
        } else if (outside) {
            xd = xd < 0 ? xd + g.nx : (xd >= g.nx ? xd - g.nx : xd);
            yd = yd < 0 ? yd + g.ny : (yd >= g.ny ? yd - g.ny : yd);
        }
        dest[i] = (long long)yd * g.nx + xd;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
        for (int i = 0; i < 5; ++i) {
            const T w = weight<T>(i);
            const T fs = f[c][i] + (w * rho[c] - f[c][i]) * k.omega[c] + w * src[c];
            f_out[(c * 5 + dir[i]) * plane + dest[i]] = fs;
        }
    }
    d_out[cell] = fma(k.k.kD, rho[2], dead);
}

template <typename T>
__global__ __launch_bounds__(BGK_THREADS) void bgk_step_kernel(const T *__restrict__ f_in,
                                                               const T *__restrict__ d_in,
                                                               T *__restrict__ f_out,
                                                               T *__restrict__ d_out, GridDesc g,
                                                               BgkCoef<T> k) {
    const int x = blockIdx.x * BGK_THREADS + threadIdx.x;
    if (x >= g.nx)
        return;
    for (int y = blockIdx.y; y < g.ny; y += gridDim.y)
        bgk_node(f_in, d_in, f_out, d_out, g, k, x, y);
}

template <typename T>
__global__ __launch_bounds__(BGK_THREADS) void bgk_init_kernel(const T *__restrict__ rho,
                                                               T *__restrict__ f,
                                                               T *__restrict__ rhoD, GridDesc g) {
    const long long plane = g.plane;
    const long long stride = (long long)gridDim.x * BGK_THREADS;
    for (long long cell = (long long)blockIdx.x * BGK_THREADS + threadIdx.x; cell < plane;
         cell += stride) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const T r = rho[c * plane + cell];
#pragma unroll
            for (int i = 0; i < 5; ++i)
                f[(c * 5 + i) * plane + cell] = weight<T>(i) * r;
        }
        rhoD[cell] = rho[4 * plane + cell];
    }
}

template <typename T>
__global__ __launch_bounds__(BGK_THREADS) void bgk_density_kernel(const T *__restrict__ f,
                                                                  const T *__restrict__ rhoD,
                                                                  T *__restrict__ rho, GridDesc g) {
    const long long plane = g.plane;
    const long long stride = (long long)gridDim.x * BGK_THREADS;
    for (long long cell = (long long)blockIdx.x * BGK_THREADS + threadIdx.x; cell < plane;
         cell += stride) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            T s = T(0);
#pragma unroll
            for (int i = 0; i < 5; ++i)
                s += f[(c * 5 + i) * plane + cell];
            rho[c * plane + cell] = s;
        }
        rho[4 * plane + cell] = rhoD[cell];
    }
}

template <typename T>
static BgkCoef<T> bgk_coef(const StepCoef &s) {
    BgkCoef<T> b;
    for (int c = 0; c < 5; ++c)
        b.k.dl[c] = (T)s.dl[c];
    b.k.bdt = (T)s.bdt;
    b.k.kE = (T)s.kE;
    b.k.kI = (T)s.kI;
    b.k.kR = (T)s.kR;
    b.k.kD = (T)s.kD;
    for (int c = 0; c < 4; ++c)
        b.omega[c] = (T)s.omega[c];
    return b;
}

// One thread per cell, at most 2^22 workgroups (2^30 work-items, within a
// launch's 32-bit work-item count); larger planes loop.
static dim3 plane_grid(const GridDesc &g) {
    const long long blocks = (g.plane + BGK_THREADS - 1) / BGK_THREADS;
    return dim3((unsigned)(blocks < (1ll << 22) ? blocks : (1ll << 22)));
}

hipError_t launch_bgk_step(int dtype, const void *f_in, const void *rhoD_in, void *f_out,
                           void *rhoD_out, const GridDesc &g, const StepCoef &k, hipStream_t s) {
    const dim3 grid((g.nx + BGK_THREADS - 1) / BGK_THREADS,
                    g.ny < BGK_MAX_GRID_ROWS ? g.ny : BGK_MAX_GRID_ROWS);
    if (dtype == SSLBM_F32)
        hipLaunchKernelGGL(bgk_step_kernel<float>, grid, dim3(BGK_THREADS), 0, s,
                           (const float *)f_in, (const float *)rhoD_in, (float *)f_out,
                           (float *)rhoD_out, g, bgk_coef<float>(k));
    else
        hipLaunchKernelGGL(bgk_step_kernel<double>, grid, dim3(BGK_THREADS), 0, s,
                           (const double *)f_in, (const double *)rhoD_in, (double *)f_out,
                           (double *)rhoD_out, g, bgk_coef<double>(k));
    return hipGetLastError();
}

hipError_t launch_bgk_init(int dtype, const void *rho, void *f, void *rhoD, const GridDesc &g,
                           hipStream_t s) {
    if (dtype == SSLBM_F32)
        hipLaunchKernelGGL(bgk_init_kernel<float>, plane_grid(g), dim3(BGK_THREADS), 0, s,
                           (const float *)rho, (float *)f, (float *)rhoD, g);
    else
        hipLaunchKernelGGL(bgk_init_kernel<double>, plane_grid(g), dim3(BGK_THREADS), 0, s,
                           (const double *)rho, (double *)f, (double *)rhoD, g);
    return hipGetLastError();
}

hipError_t launch_bgk_density(int dtype, const void *f, const void *rhoD, void *rho,
                              const GridDesc &g, hipStream_t s) {
    if (dtype == SSLBM_F32)
        hipLaunchKernelGGL(bgk_density_kernel<float>, plane_grid(g), dim3(BGK_THREADS), 0, s,
                           (const float *)f, (const float *)rhoD, (float *)rho, g);
    else
        hipLaunchKernelGGL(bgk_density_kernel<double>, plane_grid(g), dim3(BGK_THREADS), 0, s,
                           (const double *)f, (const double *)rhoD, (double *)rho, g);
    return hipGetLastError();
}

}  // namespace sslbm
