// reduce_kernels.hip -- per-compartment totals sum_x rho[C](x) in FP64, the
// quantity whose sum over C is conserved (Eq. mass_conservation).
// Two deterministic passes: a fixed number of blocks each reduce a fixed
// slice of every plane into 5 partial sums, then one block adds the partials
// in a fixed order. The same input always gives the same bits.
#include <hip/hip_runtime.h>

#include "sslbm_internal.h"

namespace sslbm {

constexpr int RED_THREADS = 256;
constexpr int RED_MAX_BLOCKS = 1024;

// Sum of v over the block in a fixed tree order; result valid in thread 0.
__device__ double block_sum(double v, double *lds) {
    lds[threadIdx.x] = v;
    __syncthreads();
    for (int s = RED_THREADS / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            lds[threadIdx.x] += lds[threadIdx.x + s];
        __syncthreads();
    }
    const double r = lds[0];
    __syncthreads();
    return r;
}

template <typename T>
__global__ __launch_bounds__(RED_THREADS) void total_partial_kernel(const T *__restrict__ rho,
                                                                    long long plane,
                                                                    double *__restrict__ partial) {
    __shared__ double lds[RED_THREADS];
    const long long per_block = (plane + gridDim.x - 1) / gridDim.x;
    const long long lo = (long long)blockIdx.x * per_block;
    const long long hi = lo + per_block < plane ? lo + per_block : plane;
    for (int c = 0; c < 5; ++c) {
        double acc = 0.0;
        for (long long i = lo + threadIdx.x; i < hi; i += RED_THREADS)
            acc += (double)rho[c * plane + i];
        const double s = block_sum(acc, lds);
        if (threadIdx.x == 0)
            partial[blockIdx.x * 5 + c] = s;
    }
}

__global__ __launch_bounds__(RED_THREADS) void total_final_kernel(const double *__restrict__ partial,
                                                                  int blocks,
                                                                  double *__restrict__ out5) {
    __shared__ double lds[RED_THREADS];
    for (int c = 0; c < 5; ++c) {
        double acc = 0.0;
        for (int b = threadIdx.x; b < blocks; b += RED_THREADS)
            acc += partial[b * 5 + c];
        const double s = block_sum(acc, lds);
        if (threadIdx.x == 0)
            out5[c] = s;
    }
}

int total_blocks(const GridDesc &g) {
    const long long want = (g.plane + 4095) / 4096;
    return (int)(want < 1 ? 1 : (want > RED_MAX_BLOCKS ? RED_MAX_BLOCKS : want));
}

hipError_t launch_total(int dtype, const void *rho, const GridDesc &g, double *partials,
                        int blocks, double *out5_device, hipStream_t s) {
    if (dtype == SSLBM_F32)
        hipLaunchKernelGGL(total_partial_kernel<float>, dim3(blocks), dim3(RED_THREADS), 0, s,
                           (const float *)rho, g.plane, partials);
    else
        hipLaunchKernelGGL(total_partial_kernel<double>, dim3(blocks), dim3(RED_THREADS), 0, s,
                           (const double *)rho, g.plane, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(total_final_kernel, dim3(1), dim3(RED_THREADS), 0, s, partials, blocks,
                       out5_device);
    return hipGetLastError();
}

}  // namespace sslbm
