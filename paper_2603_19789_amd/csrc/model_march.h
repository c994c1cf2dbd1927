// model_march.h -- the generic-model pass kernel, templated on the
// arithmetic type, the lattice, the compartment count and the steps per
// pass; each (type, lattice) pair is instantiated in a translation unit of
// its own (model_kernels_<type>_d2q<Q>.hip) so that they compile in parallel.
//
// K SSLBM steps per pass of a generic compartmental model (Eq. (generic_pde)) on the D2Q5 or the D2Q9 lattice, for up to 8
// compartments whose sources are a list of transitions.
//
// Update. Eq. (sslbm_final_clean) with rho_f = rho_b = sum_i w_i rho(x + c_i)
// (both lattices are symmetric) reduces to rho + (2 tau - 1)(sum_i w_i
// rho(x + c_i) - rho) + Psi dt:
//   D2Q5: rho + dl L5,        L5 = (N + S + E + W) - 4 rho
//   D2Q9: rho + (dl / 6) L9,  L9 = 4 (N + S + E + W) + (NE + NW + SE + SW) - 20 rho
// with dl = d dt / dx^2 (weights 1/3, 1/6 on D2Q5; 4/9, 1/9, 1/36 on D2Q9).
// No-flux walls are mirror images (map_index), periodic walls wrap.
//
// Sources. Transition r moves rate_r dt C[src] (C[cat] if cat >= 0)
// (/ N if frequency-dependent, 0 where N <= 0) from src to dst (dst < 0:
// out of the system); N sums the compartments flagged as counted. The table
// is the same for every node and sits in LDS; each lane also keeps its
// compartment vector in LDS slots, so a lookup by table index is a single
// LDS access rather than a select over all compartments.
//
// Traversal: the y-march of the SEIRD pass kernel with K steps per pass
// (one wavefront per strip of 64 - 2K output columns plus K halo columns
// per side; for every level the recent rows in a 4-slot register ring with
// compile-time slots; east/west through DPP). Level 0 is read from HBM one
// row ahead of use, levels 1..K are computed from the level below, level K
// is written: per pass every compartment is read and written about once for
// K steps. Odd chunks march up the rows, so that two chunks meeting at a
// row boundary read its halo rows at about the same time. Every level runs
// the same per-node code, so every K gives the same bits.
#pragma once

#include <hip/hip_runtime.h>

#include "march_core.h"
#include "model_internal.h"

namespace sslbm {
namespace model_detail {

constexpr int MODEL_GROUP = 4;  // transitions looked up together (divides MODEL_MAX_T)

template <int K>
struct ModelStrip {
    static constexpr int HX = K, WU = 64 - 2 * K;
};

template <typename T, int K>
struct ModelRows {
    T ring[K][RING][MODEL_MAX_C];
};

template <typename T>
struct ModelArgs {
    const T *__restrict__ in;
    T *__restrict__ out;
    GridDesc g;
    unsigned xoff, xo;
    bool out_col;
    int j0;    // first level-0 row (y0 - K marching down, y1 - 1 + K marching up)
    int dir;   // +1: rows in increasing order, -1: decreasing
    int tend;  // number of level-0 rows
};

// Level-0 row j0 + dir t into ring slot SL. The compartment count is a
// template parameter, so every load is unconditional straight-line code and
// the next row's loads stay in flight while the current row is computed.
// Rows past the chunk are still in range (the index map folds every integer
// into the grid).
template <typename T, int K, int M, int SL>
__device__ __forceinline__ void fetch_rows(ModelRows<T, K> &st, const ModelArgs<T> &a, int t) {
    const long long row = (long long)map_index(a.j0 + a.dir * t, a.g.ny, a.g.bc) * a.g.nx;
#pragma unroll
    for (int c = 0; c < M; ++c)
        st.ring[0][SL][c] =
            buf_load(row_resource(a.in + (c * a.g.plane + row), a.g.nx), a.xoff, T(0));
}

// A lane's view of its workgroup's LDS: the transition table (shared) and
// the lane's own compartment and increment slots.
template <typename T>
struct LaneLds {
    const int4 *itab;
    const T *stoich;
    T *vals;
};

// Level L (1..K) at phase P: the row of level L from three rows of level
// L-1 (slots P-L-1, P-L, P-L+1 mod 4), into slot P-L of level L, or to HBM
// for L = K.
template <typename T, int Q, int M, int K, int P, int L>
__device__ __forceinline__ void model_level(ModelRows<T, K> &st, const ModelArgs<T> &a,
                                            const ModelCoef<T> &k, const LaneLds<T> &lds, int t) {
    constexpr int su = ((P - L - 1) % RING + RING) % RING;
    constexpr int sm = ((P - L) % RING + RING) % RING;
    constexpr int sd = ((P - L + 1) % RING + RING) % RING;
    T cen[MODEL_MAX_C], out[MODEL_MAX_C];
    T total = T(0);
#pragma unroll
    for (int c = 0; c < MODEL_MAX_C; ++c) {
        cen[c] = c < M ? st.ring[L - 1][sm][c] : T(0);
        out[c] = T(0);
        if (c < M) {
            const T up = st.ring[L - 1][su][c], dn = st.ring[L - 1][sd][c];
            const T axis = (up + dn) + add_right_to(cen[c], lane_from_left(cen[c]));
            if constexpr (Q == 5) {
                out[c] = fma(k.dl[c], fma(T(-4), cen[c], axis), cen[c]);
            } else {
                const T diag = add_right_to(up, lane_from_left(up)) +
                               add_right_to(dn, lane_from_left(dn));
                out[c] = fma(k.dl[c], fma(T(-20), cen[c], fma(T(4), axis, diag)), cen[c]);
            }
            total += ((k.counted >> c) & 1u) ? cen[c] : T(0);
        }
    }
    // transitions: each lane keeps its compartment vector in LDS (slot c at
    // element c * 64 + lane), so a lookup by a table index is one LDS
    // access; slot M holds the constant 1 (no catalyst)
#pragma unroll
    for (int c = 0; c < M; ++c)
        lds.vals[c * 64] = cen[c];
    // 1 / N once per node (0 where N is not a positive normal number: no
    // frequency-dependent flow)
    const T inv_total = recip_or_zero(total);
    // MODEL_GROUP transitions at a time: their lookups are issued together,
    // so a group costs one LDS latency; increments go straight into the
    // output registers through the stoichiometry rows (rate dt (delta_dst -
    // delta_src), uniform LDS broadcasts). The table is padded with
    // zero-rate transitions to a multiple of MODEL_GROUP.
    for (int r0 = 0; r0 < k.ntrans; r0 += MODEL_GROUP) {
        int4 d[MODEL_GROUP];
        T sv[MODEL_GROUP], cv[MODEL_GROUP];
#pragma unroll
        for (int j = 0; j < MODEL_GROUP; ++j)
            d[j] = lds.itab[r0 + j];  // src, catalyst slot, destination, frequency
#pragma unroll
        for (int j = 0; j < MODEL_GROUP; ++j) {
            sv[j] = lds.vals[d[j].x * 64];
            cv[j] = lds.vals[d[j].y * 64];
        }
#pragma unroll
        for (int j = 0; j < MODEL_GROUP; ++j) {
            const T flow = sv[j] * cv[j] * (d[j].w ? inv_total : T(1));
            const T *row = lds.stoich + (r0 + j) * MODEL_MAX_C;
#pragma unroll
            for (int c = 0; c < M; ++c)
                out[c] = fma(row[c], flow, out[c]);
        }
    }
    if constexpr (L < K) {
#pragma unroll
        for (int c = 0; c < M; ++c)
            st.ring[L][sm][c] = out[c];
    } else if (a.out_col) {
        const long long row = (long long)(a.j0 + a.dir * (t - K)) * a.g.nx;
#pragma unroll
        for (int c = 0; c < M; ++c)
            buf_store(row_resource(a.out + (c * a.g.plane + row), a.g.nx), a.xo, out[c]);
    }
}

template <typename T, int Q, int M, int K, int P, int L, int LMAX>
__device__ __forceinline__ void model_levels(ModelRows<T, K> &st, const ModelArgs<T> &a,
                                             const ModelCoef<T> &k, const LaneLds<T> &lds,
                                             int t) {
    if constexpr (L <= LMAX) {
        model_level<T, Q, M, K, P, L>(st, a, k, lds, t);
        model_levels<T, Q, M, K, P, L + 1, LMAX>(st, a, k, lds, t);
    }
}

// Warm-up rows t = TC < 2K: fetch row t + 1, then the levels that already
// have three rows below them (l <= t/2). Nothing is stored yet.
template <typename T, int Q, int M, int K, int TC>
__device__ __forceinline__ void model_warm_up(ModelRows<T, K> &st, const ModelArgs<T> &a,
                                              const ModelCoef<T> &k, const LaneLds<T> &lds) {
    if constexpr (TC < 2 * K) {
        fetch_rows<T, K, M, (TC + 1) % RING>(st, a, TC + 1);
        model_levels<T, Q, M, K, TC % RING, 1, TC / 2>(st, a, k, lds, TC);
        model_warm_up<T, Q, M, K, TC + 1>(st, a, k, lds);
    }
}

// Steady-state row t (phase P): fetch row t + 1, all K levels, one output row.
template <typename T, int Q, int M, int K, int P>
__device__ __forceinline__ void model_steady(ModelRows<T, K> &st, const ModelArgs<T> &a,
                                             const ModelCoef<T> &k, const LaneLds<T> &lds,
                                             int t) {
    fetch_rows<T, K, M, (P + 1) % RING>(st, a, t + 1);
    model_levels<T, Q, M, K, P, 1, K>(st, a, k, lds, t);
}

template <typename T, int Q, int M, int K>
__global__ __launch_bounds__(BLOCK_THREADS) void model_kernel(const T *__restrict__ in,
                                                              T *__restrict__ out, GridDesc g,
                                                              ModelCoef<T> k,
                                                              const T *__restrict__ table,
                                                              int strips, int chunks, int rows) {
    // the transition table, copied to LDS by the whole workgroup before any
    // wavefront may leave; per-lane slots for the source lookups
    __shared__ int4 itab[MODEL_MAX_T];
    __shared__ T stoich[MODEL_MAX_T * MODEL_MAX_C];
    __shared__ T vals[WAVES_PER_BLOCK][(MODEL_MAX_C + 1) * 64];
    if (threadIdx.x < (unsigned)MODEL_MAX_T) {
        const int *row = reinterpret_cast<const int *>(table) + 4 * threadIdx.x;
        itab[threadIdx.x] = make_int4(row[0], row[1], row[2], row[3]);
    }
    if (threadIdx.x < (unsigned)(MODEL_MAX_T * MODEL_MAX_C))
        stoich[threadIdx.x] = reinterpret_cast<const T *>(reinterpret_cast<const int *>(table) +
                                                          4 * MODEL_MAX_T)[threadIdx.x];
    {
        const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
        vals[w][M * 64 + l] = T(1);
    }
    __syncthreads();
    const int wave = __builtin_amdgcn_readfirstlane(
        xcd_tile(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + (threadIdx.x >> 6));
    if (wave >= strips * chunks)
        return;  // whole wavefront leaves together
    using Geo = ModelStrip<K>;
    const int strip = wave / chunks, chunk = wave - strip * chunks;
    const int y0 = chunk * rows;
    const int y1 = min(y0 + rows, g.ny);
    const bool up = (chunk & 1) != 0;
    const int lane = threadIdx.x & 63;
    const int xl = strip * Geo::WU - Geo::HX + lane;
    ModelArgs<T> a;
    a.in = in;
    a.out = out;
    a.g = g;
    a.xoff = (unsigned)map_index(xl, g.nx, g.bc) * (unsigned)sizeof(T);
    a.xo = (unsigned)xl * (unsigned)sizeof(T);
    a.out_col = lane >= Geo::HX && lane < Geo::HX + Geo::WU && xl < g.nx;
    a.dir = up ? -1 : 1;
    a.j0 = up ? y1 - 1 + K : y0 - K;
    a.tend = y1 - y0 + 2 * K;

    LaneLds<T> lds;
    lds.itab = itab;
    lds.stoich = stoich;
    lds.vals = &vals[threadIdx.x >> 6][lane];

    ModelRows<T, K> st;
#pragma unroll
    for (int l = 0; l < K; ++l)
#pragma unroll
        for (int s = 0; s < RING; ++s)
#pragma unroll
            for (int c = 0; c < MODEL_MAX_C; ++c)
                st.ring[l][s][c] = T(0);
    // rows 0 .. 2K-1 fill the levels; from row 2K on every row yields output
    fetch_rows<T, K, M, 0>(st, a, 0);
    model_warm_up<T, Q, M, K, 0>(st, a, k, lds);
    constexpr int P0 = (2 * K) % RING;
    int t = 2 * K;
    for (; t + RING <= a.tend; t += RING) {
        model_steady<T, Q, M, K, P0>(st, a, k, lds, t);
        model_steady<T, Q, M, K, (P0 + 1) % RING>(st, a, k, lds, t + 1);
        model_steady<T, Q, M, K, (P0 + 2) % RING>(st, a, k, lds, t + 2);
        model_steady<T, Q, M, K, (P0 + 3) % RING>(st, a, k, lds, t + 3);
    }
    // last partial group of rows, nested so that no older ring value stays
    // live through the loop for a tail row that might read it
    if (t < a.tend) {
        model_steady<T, Q, M, K, P0>(st, a, k, lds, t);
        if (t + 1 < a.tend) {
            model_steady<T, Q, M, K, (P0 + 1) % RING>(st, a, k, lds, t + 1);
            if (t + 2 < a.tend)
                model_steady<T, Q, M, K, (P0 + 2) % RING>(st, a, k, lds, t + 2);
        }
    }
}

// Wavefronts of model_kernel<T, Q, M, K> that fit on one SIMD at once (512
// VGPRs per lane, allocated in granules of 8), from the built kernel's
// register count; queried once per device.
template <typename T, int Q, int M, int K>
int resident_waves_per_simd() {
    static int cached[16] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) {
        (void)hipGetLastError();
        return 1;
    }
    if (cached[dev])
        return cached[dev];
    hipFuncAttributes attr;
    if (hipFuncGetAttributes(&attr, (const void *)model_kernel<T, Q, M, K>) != hipSuccess) {
        (void)hipGetLastError();
        return 1;
    }
    const int regs = (attr.numRegs + 7) / 8 * 8;
    int per = regs > 0 ? 512 / regs : 8;
    per = per < 1 ? 1 : (per > 8 ? 8 : per);
    cached[dev] = per;
    return per;
}

template <typename T, int Q, int M, int K>
hipError_t launch_mk(const void *in, void *out, const GridDesc &g, const ModelCoef<T> &k,
                     const void *table, hipStream_t s) {
    const ModelShape sh = model_shape(g.nx, g.ny, K, resident_waves_per_simd<T, Q, M, K>());
    const int waves = sh.strips * sh.chunks;
    hipLaunchKernelGGL((model_kernel<T, Q, M, K>), dim3((unsigned)((waves + 3) / 4)),
                       dim3(BLOCK_THREADS), 0, s, static_cast<const T *>(in),
                       static_cast<T *>(out), g, k, static_cast<const T *>(table), sh.strips,
                       sh.chunks, sh.rows);
    return hipGetLastError();
}

template <typename T, int Q, int M>
hipError_t launch_m(const void *in, void *out, const GridDesc &g, const ModelCoef<T> &k,
                    const void *table, int K, hipStream_t s) {
    switch (K) {
    case 1: return launch_mk<T, Q, M, 1>(in, out, g, k, table, s);
    case 2: return launch_mk<T, Q, M, 2>(in, out, g, k, table, s);
    case 3: return launch_mk<T, Q, M, 3>(in, out, g, k, table, s);
    case 4: return launch_mk<T, Q, M, 4>(in, out, g, k, table, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int Q>
hipError_t launch_t(const void *in, void *out, const GridDesc &g, const ModelCoefHost &h,
                    const void *table, int K, hipStream_t s) {
    ModelCoef<T> k;
    k.m = h.m;
    k.ntrans = h.ntrans;
    k.counted = h.counted;
    for (int c = 0; c < MODEL_MAX_C; ++c)
        k.dl[c] = (T)(Q == 5 ? h.dl[c] : h.dl[c] / 6.0);
    switch (h.m) {
    case 1: return launch_m<T, Q, 1>(in, out, g, k, table, K, s);
    case 2: return launch_m<T, Q, 2>(in, out, g, k, table, K, s);
    case 3: return launch_m<T, Q, 3>(in, out, g, k, table, K, s);
    case 4: return launch_m<T, Q, 4>(in, out, g, k, table, K, s);
    case 5: return launch_m<T, Q, 5>(in, out, g, k, table, K, s);
    case 6: return launch_m<T, Q, 6>(in, out, g, k, table, K, s);
    case 7: return launch_m<T, Q, 7>(in, out, g, k, table, K, s);
    case 8: return launch_m<T, Q, 8>(in, out, g, k, table, K, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace model_detail
}  // namespace sslbm
