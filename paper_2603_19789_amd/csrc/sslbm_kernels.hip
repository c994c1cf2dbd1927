// sslbm_kernels.hip -- the SSLBM SEIRD step on gfx950: K time steps per pass
// over HBM with a y-marching wavefront.
//
// Layout: rho[5][ny][nx], structure of arrays, x fastest.
//
// Design. One wavefront owns a strip of 64 consecutive columns (one per
// lane) and walks down a chunk of rows. For every level l = 0..K-1 it keeps
// the recent rows of that level in registers; level 0 is read from HBM one
// row ahead of use, levels 1..K are computed from the rows of the level
// below, and level K is written to HBM. East and west neighbours come from
// the adjacent lanes through DPP wave shifts; north and south neighbours are
// the lane's own rows. No LDS and no barrier is needed: wavefronts are
// independent. Each field row is one coalesced 64-lane segment (256 B in
// FP32); rows are addressed through buffer descriptors held in scalar
// registers, so lanes carry 32-bit offsets only.
//
// Every level keeps its rows in a ring of 4 slots and the row loop is
// unrolled by 4, so the slot of a row is a compile-time constant (row r of
// every level lives in slot (r - j0) mod 4, j0 the first row read) and a
// loaded row lands directly in its slot: no row ever moves between
// registers. Everything that depends only on the row is wavefront-uniform
// and runs on the scalar unit.
//
// Halos are recomputed rather than exchanged: after l levels only columns at
// least l from the strip edge hold valid values, so a strip of 64 columns
// yields 64 - 2K output columns, and a chunk starts K rows above its first
// output row. Each pass reads every field about once (plus halo rows and
// columns, which neighbouring strips of the same XCD share through L2) and
// writes it once, while doing K steps of arithmetic.
#include <hip/hip_runtime.h>

#include "seird_device.h"
#include "sslbm_internal.h"

namespace sslbm {

constexpr int WAVES_PER_BLOCK = 4;
constexpr int BLOCK_THREADS = 64 * WAVES_PER_BLOCK;
constexpr int RING = 4;  // row slots per level: 3 in use + 1 being loaded

// Register budget: the rows a wavefront keeps live (3 per level plus the one
// in flight, 5 fields) must fit in 256 VGPRs with room for the arithmetic;
// larger depths are not instantiated.
template <typename T, int K>
constexpr bool march_fits() {
    return (3 * K + 1) * 5 * (int)(sizeof(T) / 4) + 48 <= 256;
}

// Row access through buffer instructions: the resource (base address and
// byte length of one row) is wavefront-uniform and lives in scalar
// registers; each lane supplies a 32-bit byte offset. An offset past the row
// end would read 0 / drop the store instead of touching other memory
// (offsets are in range by construction). Descriptor word 3 is the gfx9
// raw-buffer format (32-bit data).
constexpr int BUF_FORMAT_WORD = 0x00020000;

template <typename T>
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_resource(const T *row, int nx) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<T *>(row), (short)0,
                                             nx * (int)sizeof(T), BUF_FORMAT_WORD);
}

__device__ __forceinline__ float buf_load(__amdgpu_buffer_rsrc_t r, unsigned off, float) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double buf_load(__amdgpu_buffer_rsrc_t r, unsigned off, double) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned off, double v) {
    using U2 = unsigned __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, off, 0, 0);
}

template <typename T, int K>
struct MarchState {
    T ring[K][RING][5];  // [level][slot][compartment]
};

template <typename T>
struct MarchArgs {
    const T *__restrict__ in;
    T *__restrict__ out;
    GridDesc g;
    Coef<T> k;
    unsigned xoff;  // byte offset of this lane's memory column within a row
    int xl;         // logical column of this lane
    bool out_lane;  // lane holds an output column of the strip
    int y0;         // first output row of the chunk
    int j0;         // first level-0 row (y0 - K)
    int tend;       // number of level-0 rows
};

// Level-0 row j0 + t into its ring slot SL. Rows past the chunk are still
// in range (the index map folds every integer into the grid), so the fetch
// needs no guard.
template <typename T, int K, int SL>
__device__ __forceinline__ void fetch_row(MarchState<T, K> &st, const MarchArgs<T> &a, int t) {
    const long long row = (long long)map_index(a.j0 + t, a.g.ny, a.g.bc) * a.g.nx;
#pragma unroll
    for (int c = 0; c < 5; ++c)
        st.ring[0][SL][c] = buf_load(row_resource(a.in + (c * a.g.plane + row), a.g.nx), a.xoff,
                                     T(0));
}

// Level l (1..K) at phase P: the row j - l from rows j-l-1, j-l, j-l+1 of
// level l-1 (slots (P-l-1), (P-l), (P-l+1) mod RING); the result goes to slot
// (P-l) mod RING of level l, or to HBM for l = K (output row j - K).
template <typename T, int K, bool DIFFUSE_D, int P, int L>
__device__ __forceinline__ void level(MarchState<T, K> &st, const MarchArgs<T> &a, int t) {
    constexpr int s_up = ((P - L - 1) % RING + RING) % RING;
    constexpr int s_mid = ((P - L) % RING + RING) % RING;
    constexpr int s_dn = ((P - L + 1) % RING + RING) % RING;
    T cen[5], nb[5], res[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        cen[c] = st.ring[L - 1][s_mid][c];
        if (c < 4 || DIFFUSE_D) {
            const T ew = lane_from_right(cen[c]) + lane_from_left(cen[c]);
            nb[c] = (st.ring[L - 1][s_up][c] + st.ring[L - 1][s_dn][c]) + ew;
        } else {
            nb[c] = T(0);
        }
    }
    seird_update<T, DIFFUSE_D>(cen, nb, a.k, res);
    if constexpr (L < K) {
#pragma unroll
        for (int c = 0; c < 5; ++c)
            st.ring[L][s_mid][c] = res[c];
    } else {
        const long long row = (long long)(a.j0 + t - K) * a.g.nx;
        const unsigned xo = (unsigned)a.xl * (unsigned)sizeof(T);
        if (a.out_lane) {
#pragma unroll
            for (int c = 0; c < 5; ++c)
                buf_store(row_resource(a.out + (c * a.g.plane + row), a.g.nx), xo, res[c]);
        }
    }
}

// Levels L..LMAX at phase P.
template <typename T, int K, bool DIFFUSE_D, int P, int L, int LMAX>
__device__ __forceinline__ void levels(MarchState<T, K> &st, const MarchArgs<T> &a, int t) {
    if constexpr (L <= LMAX) {
        level<T, K, DIFFUSE_D, P, L>(st, a, t);
        levels<T, K, DIFFUSE_D, P, L + 1, LMAX>(st, a, t);
    }
}

// Warm-up rows t = TC < 2K (compile time): fetch row t + 1, then the levels
// that already have three rows below them (l <= t/2). Nothing is stored yet.
template <typename T, int K, bool DIFFUSE_D, int TC>
__device__ __forceinline__ void warm_up(MarchState<T, K> &st, const MarchArgs<T> &a) {
    if constexpr (TC < 2 * K) {
        fetch_row<T, K, (TC + 1) % RING>(st, a, TC + 1);
        levels<T, K, DIFFUSE_D, TC % RING, 1, TC / 2>(st, a, TC);
        warm_up<T, K, DIFFUSE_D, TC + 1>(st, a);
    }
}

// Steady-state row t (phase P): fetch row t + 1, all K levels, one output row.
// Straight-line code, so the memory counters stay exact and the wait for row
// t's data lets the row t + 1 loads stay in flight.
template <typename T, int K, bool DIFFUSE_D, int P>
__device__ __forceinline__ void steady_row(MarchState<T, K> &st, const MarchArgs<T> &a, int t) {
    fetch_row<T, K, (P + 1) % RING>(st, a, t + 1);
    levels<T, K, DIFFUSE_D, P, 1, K>(st, a, t);
}

template <typename T, int K, bool DIFFUSE_D>
__global__ __launch_bounds__(BLOCK_THREADS) void sslbm_march_kernel(
    const T *__restrict__ in, T *__restrict__ out, GridDesc g, Coef<T> k, int rows_per_wave,
    int strips, int total_waves) {
    constexpr int WU = 64 - 2 * K;  // output columns per strip
    const int lane = threadIdx.x & 63;
    // wavefront-uniform from here on: keep it in scalar registers
    const int wave = __builtin_amdgcn_readfirstlane(
        xcd_tile(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + (threadIdx.x >> 6));
    if (wave >= total_waves)
        return;  // whole wavefront leaves together
    const int strip = wave % strips;
    const int chunk = wave / strips;

    MarchArgs<T> a;
    a.in = in;
    a.out = out;
    a.g = g;
    a.k = k;
    a.y0 = chunk * rows_per_wave;
    const int y1 = min(a.y0 + rows_per_wave, g.ny);  // output rows [y0, y1)
    a.j0 = a.y0 - K;
    a.tend = y1 - a.y0 + 2 * K;
    a.xl = strip * WU - K + lane;
    a.xoff = (unsigned)map_index(a.xl, g.nx, g.bc) * (unsigned)sizeof(T);
    a.out_lane = lane >= K && lane < 64 - K && a.xl < g.nx;

    MarchState<T, K> st;
#pragma unroll
    for (int l = 0; l < K; ++l)
#pragma unroll
        for (int r = 0; r < RING; ++r)
#pragma unroll
            for (int c = 0; c < 5; ++c)
                st.ring[l][r][c] = T(0);

    // rows 0 .. 2K-1: fill the levels; from row 2K on every row yields output
    fetch_row<T, K, 0>(st, a, 0);
    warm_up<T, K, DIFFUSE_D, 0>(st, a);
    constexpr int P0 = (2 * K) % RING;
    int t = 2 * K;
    for (; t + RING <= a.tend; t += RING) {
        steady_row<T, K, DIFFUSE_D, P0>(st, a, t);
        steady_row<T, K, DIFFUSE_D, (P0 + 1) % RING>(st, a, t + 1);
        steady_row<T, K, DIFFUSE_D, (P0 + 2) % RING>(st, a, t + 2);
        steady_row<T, K, DIFFUSE_D, (P0 + 3) % RING>(st, a, t + 3);
    }
    // last partial group of rows (only when the chunk height is not a multiple of 4)
    if (t < a.tend)
        steady_row<T, K, DIFFUSE_D, P0>(st, a, t);
    if (t + 1 < a.tend)
        steady_row<T, K, DIFFUSE_D, (P0 + 1) % RING>(st, a, t + 1);
    if (t + 2 < a.tend)
        steady_row<T, K, DIFFUSE_D, (P0 + 2) % RING>(st, a, t + 2);
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
    if constexpr (!march_fits<T, K>()) {
        return hipErrorInvalidValue;
    } else {
        constexpr int WU = 64 - 2 * K;
        const int strips = (g.nx + WU - 1) / WU;
        const int chunks = (g.ny + shape.rows_per_wave - 1) / shape.rows_per_wave;
        const long long waves = (long long)strips * chunks;
        const long long blocks = (waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
        if (waves > 0x7fffffffll)
            return hipErrorInvalidConfiguration;
        hipLaunchKernelGGL((sslbm_march_kernel<T, K, DD>), dim3((unsigned)blocks),
                           dim3(BLOCK_THREADS), 0, st, static_cast<const T *>(in),
                           static_cast<T *>(out), g, cast_coef<T>(s), shape.rows_per_wave,
                           strips, (int)waves);
        return hipGetLastError();
    }
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

int strip_width(int K) { return 64 - 2 * K; }

template <typename T>
static int max_depth() {
    int K = 0;
    if (march_fits<T, 1>()) K = 1;
    if (march_fits<T, 2>()) K = 2;
    if (march_fits<T, 3>()) K = 3;
    if (march_fits<T, 4>()) K = 4;
    if (march_fits<T, 5>()) K = 5;
    if (march_fits<T, 6>()) K = 6;
    if (march_fits<T, 7>()) K = 7;
    if (march_fits<T, 8>()) K = 8;
    return K;
}

int march_max_depth(int dtype) {
    return dtype == SSLBM_F32 ? max_depth<float>() : max_depth<double>();
}

}  // namespace sslbm
