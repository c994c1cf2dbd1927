// fd4_kernels.hip -- the finite-difference reference solver of Sec. III on
// gfx950: fourth-order centred differences in space, the classic RK4 method
// in time, and the SEIRD reactions (Eqs. (EqSEIRD_S)-(EqSEIRD_D)) evaluated
// at every stage. It serves to validate the SSLBM on large grids and to
// time the comparison the paper makes; it is not on the SSLBM's path.
//
// With F the right-hand side and G = dt F, one step is
//   k1 = G(u), k2 = G(u + k1/2), k3 = G(u + k2/2), k4 = G(u + k3),
//   u' = u + (k1 + 2 k2 + 2 k3 + k4) / 6,
// G_C = (dl_C / 12) lap(rho_C) + Psi_C dt with dl = d dt / dx^2 and
// lap u = sum over the axes of -u(-2) + 16 u(-1) - 30 u + 16 u(+1) - u(+2).
// Each stage is one launch, because every stage reads its input two cells
// around each node: stage s reads its input y_s with the stencil and writes
// the next input y2 = u + k1/2, y3 = u + k2/2, y4 = u + k3. The stage inputs
// hold the k's (k1 = 2 (y2 - u), k2 = 2 (y3 - u), k3 = y4 - u), so the last
// stage needs no running sum: u' = (y2 + 2 y3 + y4 - u) / 3 + k4 / 6, written
// over u. Buffers: u (the state), y2, y3, y4. Per node and step the four
// stages move 13 state-sized arrays (stencil reads counted once), against 16
// with a running sum.
//
// A workgroup of 256 threads takes a tile of 64 columns x 16 rows: the tile
// and its two-cell halo of all five fields are staged in LDS (ghost cells by
// the boundary's index map: periodic wrap, or the even reflection about the
// wall of a no-flux boundary), then every thread computes four nodes of one
// column.
#include <hip/hip_runtime.h>

#include "fd4_internal.h"
#include "seird_device.h"

namespace sslbm {

namespace {

constexpr int FX = 64, FY = 16;               // tile: columns x rows
constexpr int GX = FX + 4, GY = FY + 4;       // with the two-cell halo
constexpr int FD4_THREADS = 256;
constexpr int ROWS_PER_THREAD = FY * FX / FD4_THREADS;

template <typename T, int STAGE>
__global__ __launch_bounds__(FD4_THREADS) void fd4_stage_kernel(
    const T *__restrict__ y_in, const T *u, const T *__restrict__ y2,
    const T *__restrict__ y3, T *out, GridDesc g, Coef<T> k, int tiles_x, int tiles) {
    __shared__ T tile[5][GY][GX];
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    if (t >= tiles)
        return;  // whole workgroup leaves together, before any barrier
    const int x0 = (t % tiles_x) * FX, y0 = (t / tiles_x) * FY;
    // stage the tile and its halo (ghost rows and columns folded into the grid)
    for (int e = threadIdx.x; e < GX * GY; e += FD4_THREADS) {
        const int ly = e / GX, lx = e - ly * GX;
        const long long cell =
            (long long)map_index(y0 + ly - 2, g.ny, g.bc) * g.nx + map_index(x0 + lx - 2, g.nx, g.bc);
#pragma unroll
        for (int c = 0; c < 5; ++c)
            tile[c][ly][lx] = y_in[c * g.plane + cell];
    }
    __syncthreads();

    const int lx = threadIdx.x % FX, ly0 = threadIdx.x / FX;
    const int x = x0 + lx;
    if (x >= g.nx)
        return;
    const T dl12[5] = {k.dl[0] / T(12), k.dl[1] / T(12), k.dl[2] / T(12), k.dl[3] / T(12),
                       k.dl[4] / T(12)};
#pragma unroll
    for (int r = 0; r < ROWS_PER_THREAD; ++r) {
        const int ly = ly0 + r * (FD4_THREADS / FX);
        const int y = y0 + ly;
        if (y >= g.ny)
            break;
        const int cx = lx + 2, cy = ly + 2;
        T cen[5];
#pragma unroll
        for (int c = 0; c < 5; ++c)
            cen[c] = tile[c][cy][cx];
        T fdt, rE, rI;
        seird_increments(cen[0], cen[1], cen[2], cen[3], k, fdt, rE, rI);
        const T src[5] = {-fdt, fdt - rE, rE - rI, k.kR * cen[2], k.kD * cen[2]};
        const long long cell = (long long)y * g.nx + x;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            const T(*f)[GX] = tile[c];
            const T along_x = (T(16) * (f[cy][cx - 1] + f[cy][cx + 1]) -
                               (f[cy][cx - 2] + f[cy][cx + 2])) - T(30) * cen[c];
            const T along_y = (T(16) * (f[cy - 1][cx] + f[cy + 1][cx]) -
                               (f[cy - 2][cx] + f[cy + 2][cx])) - T(30) * cen[c];
            const T kc = fma(dl12[c], along_x + along_y, src[c]);
            const long long i = c * g.plane + cell;
            if constexpr (STAGE == 1) {
                out[i] = fma(kc, T(0.5), cen[c]);  // y_in is u
            } else if constexpr (STAGE == 2) {
                out[i] = fma(kc, T(0.5), u[i]);
            } else if constexpr (STAGE == 3) {
                out[i] = kc + u[i];
            } else {
                // out is u: the new state (each node read, then written, by
                // its own thread; the stencil reads y4, not u)
                const T s = ((y2[i] + T(2) * y3[i]) + cen[c]) - u[i];
                out[i] = fma(kc, T(1) / T(6), s / T(3));
            }
        }
    }
}

template <typename T>
hipError_t launch_t(void *rho, void *work, const GridDesc &g, const StepCoef &s, long long n,
                    hipStream_t st) {
    T *u = static_cast<T *>(rho);
    T *y2 = static_cast<T *>(work);
    T *y3 = y2 + 5 * g.plane;
    T *y4 = y3 + 5 * g.plane;
    Coef<T> k;
    for (int c = 0; c < 5; ++c)
        k.dl[c] = (T)s.dl[c];
    k.bdt = (T)s.bdt;
    k.kE = (T)s.kE;
    k.kI = (T)s.kI;
    k.kR = (T)s.kR;
    k.kD = (T)s.kD;
    const int tiles_x = (g.nx + FX - 1) / FX;
    const int tiles = tiles_x * ((g.ny + FY - 1) / FY);
    const dim3 grid((unsigned)tiles), block(FD4_THREADS);
    for (long long step = 0; step < n; ++step) {
        hipLaunchKernelGGL((fd4_stage_kernel<T, 1>), grid, block, 0, st, u, u, y2, y3, y2, g, k,
                           tiles_x, tiles);
        hipLaunchKernelGGL((fd4_stage_kernel<T, 2>), grid, block, 0, st, y2, u, y2, y3, y3, g, k,
                           tiles_x, tiles);
        hipLaunchKernelGGL((fd4_stage_kernel<T, 3>), grid, block, 0, st, y3, u, y2, y3, y4, g, k,
                           tiles_x, tiles);
        hipLaunchKernelGGL((fd4_stage_kernel<T, 4>), grid, block, 0, st, y4, u, y2, y3, u, g, k,
                           tiles_x, tiles);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_fd4(int dtype, void *rho, void *work, const GridDesc &g, const StepCoef &k,
                      long long nsteps, hipStream_t s) {
    return dtype == SSLBM_F32 ? launch_t<float>(rho, work, g, k, nsteps, s)
                              : launch_t<double>(rho, work, g, k, nsteps, s);
}

}  // namespace sslbm
