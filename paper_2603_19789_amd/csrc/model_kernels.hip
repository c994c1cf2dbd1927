// model_kernels.hip -- one SSLBM step of a generic compartmental model
// (Eq. (generic_pde)) on the D2Q5 or the D2Q9 lattice, for up to 8
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
// compartment vector and its increments in LDS slots, so a lookup by table
// index is a single LDS access rather than a select over all compartments.
//
// Traversal: the y-march of the single-step kernels (one wavefront per strip
// of 62 output columns plus one halo column per side, rows in a 4-slot
// register ring with compile-time slots, east/west through DPP). Per output
// row: one row of every compartment read, one written.
#include <hip/hip_runtime.h>

#include "march_core.h"
#include "model_internal.h"

namespace sslbm {

namespace {

constexpr int MHX = 1, MWU = 64 - 2 * MHX;
constexpr int MODEL_GROUP = 4;  // transitions looked up together (divides MODEL_MAX_T)

template <typename T>
struct ModelRows {
    T ring[RING][MODEL_MAX_C];
};

template <typename T>
struct ModelArgs {
    const T *__restrict__ in;
    T *__restrict__ out;
    GridDesc g;
    unsigned xoff, xo;
    bool out_col;
    int j0;
};

// The compartment count is a template parameter, so every load is
// unconditional straight-line code and the next row's loads stay in flight
// while the current row is computed.
template <typename T, int M, int SL>
__device__ __forceinline__ void fetch_rows(ModelRows<T> &st, const ModelArgs<T> &a, int t) {
    const long long row = (long long)map_index(a.j0 + t, a.g.ny, a.g.bc) * a.g.nx;
#pragma unroll
    for (int c = 0; c < M; ++c)
        st.ring[SL][c] =
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

template <typename T, int Q, int M, int P>
__device__ __forceinline__ void model_row(ModelRows<T> &st, const ModelArgs<T> &a,
                                          const ModelCoef<T> &k, const LaneLds<T> &lds, int t) {
    constexpr int su = (P + 2) % RING, sm = (P + 3) % RING, sd = P % RING;
    T cen[MODEL_MAX_C], out[MODEL_MAX_C];
    T total = T(0);
#pragma unroll
    for (int c = 0; c < MODEL_MAX_C; ++c) {
        cen[c] = c < M ? st.ring[sm][c] : T(0);
        out[c] = T(0);
        if (c < M) {
            const T up = st.ring[su][c], dn = st.ring[sd][c];
            const T axis = (up + dn) + (lane_from_right(cen[c]) + lane_from_left(cen[c]));
            if constexpr (Q == 5) {
                out[c] = fma(k.dl[c], fma(T(-4), cen[c], axis), cen[c]);
            } else {
                const T diag = (lane_from_right(up) + lane_from_left(up)) +
                               (lane_from_right(dn) + lane_from_left(dn));
                out[c] = fma(k.dl[c], fma(T(-20), cen[c], fma(T(4), axis, diag)), cen[c]);
            }
            total += ((k.counted >> c) & 1u) ? cen[c] : T(0);
        }
    }
    // transitions: each lane keeps its compartment vector and its source
    // increments in LDS (slot c at element c * 64 + lane), so a lookup by a
    // table index is one LDS access; slot M of vals holds the constant 1 (no
    // catalyst), slot M of psi absorbs flows out of the system
#pragma unroll
    for (int c = 0; c < M; ++c)
        lds.vals[c * 64] = cen[c];
    // 1 / N once per node (0 where N <= 0: no frequency-dependent flow)
    const T inv_total = total > T(0) ? quotient(T(1), total) : T(0);
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
    if (a.out_col) {
        const long long row = (long long)(a.j0 + t - 1) * a.g.nx;
#pragma unroll
        for (int c = 0; c < M; ++c)
            buf_store(row_resource(a.out + (c * a.g.plane + row), a.g.nx), a.xo, out[c]);
    }
}

template <typename T, int Q, int M, int P>
__device__ __forceinline__ void model_steady(ModelRows<T> &st, const ModelArgs<T> &a,
                                             const ModelCoef<T> &k, const LaneLds<T> &lds,
                                             int t) {
    fetch_rows<T, M, (P + 1) % RING>(st, a, t + 1);
    model_row<T, Q, M, P>(st, a, k, lds, t);
}

template <typename T, int Q, int M>
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
    const int strip = wave / chunks, chunk = wave - strip * chunks;
    const int y0 = chunk * rows;
    const int y1 = min(y0 + rows, g.ny);
    const int lane = threadIdx.x & 63;
    const int xl = strip * MWU - MHX + lane;
    ModelArgs<T> a;
    a.in = in;
    a.out = out;
    a.g = g;
    a.xoff = (unsigned)map_index(xl, g.nx, g.bc) * (unsigned)sizeof(T);
    a.xo = (unsigned)xl * (unsigned)sizeof(T);
    a.out_col = lane >= MHX && lane < MHX + MWU && xl < g.nx;
    a.j0 = y0 - 1;

    LaneLds<T> lds;
    lds.itab = itab;
    lds.stoich = stoich;
    lds.vals = &vals[threadIdx.x >> 6][lane];

    ModelRows<T> st;
#pragma unroll
    for (int s = 0; s < RING; ++s)
#pragma unroll
        for (int c = 0; c < MODEL_MAX_C; ++c)
            st.ring[s][c] = T(0);
    // rows j0 .. y1 (t = 0 .. tend); the output row of t is j0 + t - 1
    const int tend = y1 - y0 + 2;
    fetch_rows<T, M, 0>(st, a, 0);
    fetch_rows<T, M, 1>(st, a, 1);
    fetch_rows<T, M, 2>(st, a, 2);
    int t = 2;
    for (; t + RING <= tend; t += RING) {
        model_steady<T, Q, M, 2>(st, a, k, lds, t);
        model_steady<T, Q, M, 3>(st, a, k, lds, t + 1);
        model_steady<T, Q, M, 0>(st, a, k, lds, t + 2);
        model_steady<T, Q, M, 1>(st, a, k, lds, t + 3);
    }
    if (t < tend)
        model_steady<T, Q, M, 2>(st, a, k, lds, t);
    if (t + 1 < tend)
        model_steady<T, Q, M, 3>(st, a, k, lds, t + 1);
    if (t + 2 < tend)
        model_steady<T, Q, M, 0>(st, a, k, lds, t + 2);
}

template <typename T, int Q, int M>
hipError_t launch_m(const void *in, void *out, const GridDesc &g, const ModelCoef<T> &k,
                    const void *table, hipStream_t s) {
    const ModelShape sh = model_shape(g.nx, g.ny);
    const int waves = sh.strips * sh.chunks;
    hipLaunchKernelGGL((model_kernel<T, Q, M>), dim3((unsigned)((waves + 3) / 4)),
                       dim3(BLOCK_THREADS), 0, s, static_cast<const T *>(in),
                       static_cast<T *>(out), g, k, static_cast<const T *>(table), sh.strips,
                       sh.chunks, sh.rows);
    return hipGetLastError();
}

template <typename T, int Q>
hipError_t launch_t(const void *in, void *out, const GridDesc &g, const ModelCoefHost &h,
                    const void *table, hipStream_t s) {
    ModelCoef<T> k;
    k.m = h.m;
    k.ntrans = h.ntrans;
    k.counted = h.counted;
    for (int c = 0; c < MODEL_MAX_C; ++c)
        k.dl[c] = (T)(Q == 5 ? h.dl[c] : h.dl[c] / 6.0);
    switch (h.m) {
    case 1: return launch_m<T, Q, 1>(in, out, g, k, table, s);
    case 2: return launch_m<T, Q, 2>(in, out, g, k, table, s);
    case 3: return launch_m<T, Q, 3>(in, out, g, k, table, s);
    case 4: return launch_m<T, Q, 4>(in, out, g, k, table, s);
    case 5: return launch_m<T, Q, 5>(in, out, g, k, table, s);
    case 6: return launch_m<T, Q, 6>(in, out, g, k, table, s);
    case 7: return launch_m<T, Q, 7>(in, out, g, k, table, s);
    case 8: return launch_m<T, Q, 8>(in, out, g, k, table, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

ModelShape model_shape(int nx, int ny) {
    // two workgroups of four wavefronts per CU (two wavefronts per SIMD hide
    // each other's LDS and memory waits), chunks of at least 8 rows; measured
    // at 4096 x 4096 with six compartments: 56 GLUPS with one wavefront per
    // SIMD, 73 with two, 66 with four (shorter chunks, more halo rows)
    ModelShape s;
    s.strips = (nx + MWU - 1) / MWU;
    long long chunks = (2 * 256 * WAVES_PER_BLOCK) / s.strips;
    if (chunks < 1)
        chunks = 1;
    long long rows = (ny + chunks - 1) / chunks;
    if (rows < 8)
        rows = 8;
    if (rows > ny)
        rows = ny;
    s.rows = (int)rows;
    s.chunks = (int)((ny + rows - 1) / rows);
    return s;
}

hipError_t launch_model(int dtype, int lattice, const void *in, void *out, const GridDesc &g,
                        const ModelCoefHost &h, const void *table, hipStream_t s) {
    if (dtype == SSLBM_F32)
        return lattice == 9 ? launch_t<float, 9>(in, out, g, h, table, s)
                            : launch_t<float, 5>(in, out, g, h, table, s);
    return lattice == 9 ? launch_t<double, 9>(in, out, g, h, table, s)
                        : launch_t<double, 5>(in, out, g, h, table, s);
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
