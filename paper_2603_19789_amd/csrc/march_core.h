// march_core.h -- the y-marching pass of the SSLBM SEIRD step on gfx950,
// shared by the single-grid and the ensemble kernels: K time steps per pass
// over HBM.
//
// Layout: rho[5][ny][nx], structure of arrays, x fastest.
//
// Design. One wavefront owns a strip of 64 V consecutive columns (V = 1 or
// 2 adjacent columns per lane) and walks down a chunk of rows. For every
// level l = 0..K-1 it keeps the recent rows of that level in registers;
// level 0 is read from HBM one row ahead of use, levels 1..K are computed
// from the rows of the level below, and level K is written to HBM. East and
// west neighbours come from the neighbouring register of the lane or, across
// lanes, from DPP wave shifts; north and south neighbours are the lane's own
// rows. No LDS and no barrier is needed: wavefronts are independent. A
// lane's V elements of a field row are one 32/64/128-bit access; rows are
// addressed through buffer descriptors held in scalar registers, so lanes
// carry 32-bit offsets only.
//
// Every level keeps its rows in a ring of 4 slots and the row loop is
// unrolled by 4, so the slot of a row is a compile-time constant (row r of
// every level lives in slot (r - j0) mod 4, j0 the first row read) and a
// loaded row lands directly in its slot: no row ever moves between
// registers. The first 2K rows (filling the levels) are unrolled at compile
// time; after them the loop body is straight-line code, so the memory
// counters stay exact and the next rows' loads stay in flight while the
// current row is computed. Everything that depends only on the row is
// wavefront-uniform and runs on the scalar unit.
//
// Halos are recomputed rather than exchanged: after l levels only columns at
// least l from the strip edge hold valid values, so a strip yields
// 64 V - 2 HX output columns (HX = K rounded up to a multiple of V), and a
// chunk starts K rows above its first output row. Each pass reads every
// field about once (plus halo rows and columns, which neighbouring strips of
// the same XCD share through L2) and writes it once, while doing K steps of
// arithmetic.
#pragma once

#include <hip/hip_runtime.h>

#include "seird_device.h"
#include "sslbm_internal.h"

namespace sslbm {

constexpr int WAVES_PER_BLOCK = 4;
constexpr int BLOCK_THREADS = 64 * WAVES_PER_BLOCK;
constexpr int RING = 4;  // row slots per level: 3 in use + 1 being loaded

// Register budget: the rows a wavefront keeps live (3 per level plus the one
// in flight, 5 fields, V columns) plus the arithmetic's temporaries must fit
// in 256 VGPRs (two wavefronts per SIMD); larger combinations would spill and
// are not instantiated.
template <typename T, int K, int V>
constexpr bool march_fits() {
    constexpr int words = (int)(sizeof(T) / 4);
    return (3 * K + 1) * 5 * V * words + 48 * words <= 256;
}

// Strip geometry: 64 lanes x V columns, of which HX on each side are halo
// (K rounded up to a multiple of V so that every strip starts at an even
// column for V = 2).
template <int K, int V>
struct Strip {
    static constexpr int HX = (K + V - 1) / V * V;
    static constexpr int WU = 64 * V - 2 * HX;  // output columns
};

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
// Stores go through L2 with the default policy: strips are not aligned to
// 128-byte lines, and L2 merges the partial lines that neighbouring strips
// write (streaming them past the cache measured slower).
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned off, float v) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, unsigned off, double v) {
    using U2 = unsigned __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, off, 0, 0);
}

// Two consecutive elements at an aligned byte offset, one vector access.
// The loaded vector is reinterpreted as one wide integer and split with
// shifts: taking its elements one by one lets this compiler narrow the load
// to half its width (the upper half is then never read).
__device__ __forceinline__ void buf_load_pair(__amdgpu_buffer_rsrc_t r, unsigned off, float &a,
                                              float &b) {
    const unsigned long long w = __builtin_bit_cast(
        unsigned long long, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
    a = __builtin_bit_cast(float, (unsigned)w);
    b = __builtin_bit_cast(float, (unsigned)(w >> 32));
}
__device__ __forceinline__ void buf_load_pair(__amdgpu_buffer_rsrc_t r, unsigned off, double &a,
                                              double &b) {
    const unsigned __int128 w = __builtin_bit_cast(
        unsigned __int128, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0));
    a = __builtin_bit_cast(double, (unsigned long long)w);
    b = __builtin_bit_cast(double, (unsigned long long)(w >> 64));
}
__device__ __forceinline__ void buf_store_pair(__amdgpu_buffer_rsrc_t r, unsigned off, float a,
                                               float b) {
    using U2 = unsigned __attribute__((ext_vector_type(2)));
    const U2 w = {__builtin_bit_cast(unsigned, a), __builtin_bit_cast(unsigned, b)};
    __builtin_amdgcn_raw_buffer_store_b64(w, r, off, 0, 0);
}
__device__ __forceinline__ void buf_store_pair(__amdgpu_buffer_rsrc_t r, unsigned off, double a,
                                               double b) {
    using U4 = unsigned __attribute__((ext_vector_type(4)));
    const unsigned long long x = __builtin_bit_cast(unsigned long long, a);
    const unsigned long long y = __builtin_bit_cast(unsigned long long, b);
    const U4 w = {(unsigned)x, (unsigned)(x >> 32), (unsigned)y, (unsigned)(y >> 32)};
    __builtin_amdgcn_raw_buffer_store_b128(w, r, off, 0, 0);
}

template <typename T, int K, int V>
struct MarchState {
    T ring[K][RING][5][V];  // [level][slot][compartment][column of the lane]
};

template <typename T, int V>
struct MarchArgs {
    const T *__restrict__ in;
    T *__restrict__ out;
    T *__restrict__ mid_out;  // the state after MID steps (MID > 0 only)
    GridDesc g;
    Coef<T> k;
    unsigned xoff[V];  // byte offsets of this lane's memory columns within a row
    bool swap;         // V = 2: the lane's pair lies reversed in memory (mirror image)
    int xl;            // logical column of this lane's first column
    bool out_col[V];   // the column is an output column of the strip
    int j0;            // first level-0 row (y0 - K marching down, y1 - 1 + K marching up)
    int dir;           // +1: rows in increasing order, -1: decreasing
    int tend;          // number of level-0 rows
};

// Level-0 row j0 + t into its ring slot SL. Rows past the chunk are still
// in range (the index map folds every integer into the grid), so the fetch
// needs no guard.
template <typename T, int K, int V, bool SW, int SL>
__device__ __forceinline__ void fetch_row(MarchState<T, K, V> &st, const MarchArgs<T, V> &a,
                                          int t) {
    const long long row = (long long)map_index(a.j0 + a.dir * t, a.g.ny, a.g.bc) * a.g.nx;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        const __amdgpu_buffer_rsrc_t r = row_resource(a.in + (c * a.g.plane + row), a.g.nx);
        if constexpr (V == 1) {
            st.ring[0][SL][c][0] = buf_load(r, a.xoff[0], T(0));
        } else {
            // the pair is one aligned vector in memory, possibly mirrored
            // (only strips with a lane across a no-flux wall take the select)
            T lo, hi;
            buf_load_pair(r, a.xoff[0], lo, hi);
            if constexpr (SW) {
                st.ring[0][SL][c][0] = a.swap ? hi : lo;
                st.ring[0][SL][c][1] = a.swap ? lo : hi;
            } else {
                st.ring[0][SL][c][0] = lo;
                st.ring[0][SL][c][1] = hi;
            }
        }
    }
}

// East + west neighbours of column v of this lane at level-(L-1) slot S:
// the adjacent column inside the lane, or the next lane's edge column
// through a DPP wave shift.
template <typename T, int V, typename Row>
__device__ __forceinline__ T east_west(const Row &m, int v) {
    static_assert(V == 1 || V == 2, "one or two columns per lane");
    if constexpr (V == 1) {
        return add_right_to(m[0], lane_from_left(m[0]));
    } else {
        if (v == 0)
            return add_from_left(m[V - 1]);  // m[1] + the left lane's m[1] (V = 2)
        if (v == V - 1)
            return add_from_right(m[0]);  // the right lane's m[0] + m[0] (V = 2)
        return m[v + 1] + m[v - 1];
    }
}

// Level l (1..K) at phase P: the row j - l from rows j-l-1, j-l, j-l+1 of
// level l-1 (slots (P-l-1), (P-l), (P-l+1) mod RING); the result goes to slot
// (P-l) mod RING of level l, or to HBM for l = K (output row j - K).
// Row r (counted from j0 in the marching direction) of the five results of
// this lane into dst, at the strip's output columns.
template <typename T, int V>
__device__ __forceinline__ void store_row(T *__restrict__ dst, const MarchArgs<T, V> &a, int r,
                                          const T (&res)[5][V]) {
    const long long row = (long long)(a.j0 + a.dir * r) * a.g.nx;
    const unsigned xo = (unsigned)a.xl * (unsigned)sizeof(T);
    if constexpr (V == 1) {
        if (a.out_col[0]) {
#pragma unroll
            for (int c = 0; c < 5; ++c)
                buf_store(row_resource(dst + (c * a.g.plane + row), a.g.nx), xo, res[c][0]);
        }
    } else {
        // strips start at even columns and nx is even, so a pair is either
        // entirely output or entirely halo
        if (a.out_col[0]) {
#pragma unroll
            for (int c = 0; c < 5; ++c)
                buf_store_pair(row_resource(dst + (c * a.g.plane + row), a.g.nx), xo, res[c][0],
                               res[c][1]);
        }
    }
}

// MID > 0: level MID's rows that are output rows of the chunk also go to
// a.mid_out, the state after MID steps (the same bits as a pass of MID
// steps: the output rows and columns hold exact values at every level).
template <typename T, int K, bool DIFFUSE_D, int V, int P, int L, int MID = 0>
__device__ __forceinline__ void level(MarchState<T, K, V> &st, const MarchArgs<T, V> &a, int t) {
    constexpr int s_up = ((P - L - 1) % RING + RING) % RING;
    constexpr int s_mid = ((P - L) % RING + RING) % RING;
    constexpr int s_dn = ((P - L + 1) % RING + RING) % RING;
    T res[5][V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
        T cen[5], nb[5], o[5];
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            cen[c] = st.ring[L - 1][s_mid][c][v];
            if (c < 4 || DIFFUSE_D) {
                const T ew = east_west<T, V>(st.ring[L - 1][s_mid][c], v);
                nb[c] = (st.ring[L - 1][s_up][c][v] + st.ring[L - 1][s_dn][c][v]) + ew;
            } else {
                nb[c] = T(0);
            }
        }
        seird_update<T, DIFFUSE_D>(cen, nb, a.k, o);
#pragma unroll
        for (int c = 0; c < 5; ++c)
            res[c][v] = o[c];
    }
    if constexpr (L < K) {
#pragma unroll
        for (int c = 0; c < 5; ++c)
#pragma unroll
            for (int v = 0; v < V; ++v)
                st.ring[L][s_mid][c][v] = res[c][v];
        if constexpr (L == MID) {
            // the level's row t - L is an output row for t - L in [K, tend - K)
            if (t - L >= K && t - L < a.tend - K)
                store_row<T, V>(a.mid_out, a, t - L, res);
        }
    } else {
        store_row<T, V>(a.out, a, t - K, res);
    }
}

// Levels L..LMAX at phase P.
template <typename T, int K, bool DIFFUSE_D, int V, int P, int L, int LMAX, int MID = 0>
__device__ __forceinline__ void levels(MarchState<T, K, V> &st, const MarchArgs<T, V> &a, int t) {
    if constexpr (L <= LMAX) {
        level<T, K, DIFFUSE_D, V, P, L, MID>(st, a, t);
        levels<T, K, DIFFUSE_D, V, P, L + 1, LMAX, MID>(st, a, t);
    }
}

// Warm-up rows t = TC < 2K (compile time): fetch row t + 1, then the levels
// that already have three rows below them (l <= t/2). Nothing is stored yet.
template <typename T, int K, bool DIFFUSE_D, int V, bool SW, int TC, int MID = 0>
__device__ __forceinline__ void warm_up(MarchState<T, K, V> &st, const MarchArgs<T, V> &a) {
    if constexpr (TC < 2 * K) {
        fetch_row<T, K, V, SW, (TC + 1) % RING>(st, a, TC + 1);
        levels<T, K, DIFFUSE_D, V, TC % RING, 1, TC / 2, MID>(st, a, TC);
        warm_up<T, K, DIFFUSE_D, V, SW, TC + 1, MID>(st, a);
    }
}

// Steady-state row t (phase P): fetch row t + 1, all K levels, one output row.
// Straight-line code, so the memory counters stay exact and the wait for row
// t's data lets the row t + 1 loads stay in flight.
template <typename T, int K, bool DIFFUSE_D, int V, bool SW, int P, int MID = 0>
__device__ __forceinline__ void steady_row(MarchState<T, K, V> &st, const MarchArgs<T, V> &a,
                                           int t) {
    fetch_row<T, K, V, SW, (P + 1) % RING>(st, a, t + 1);
    levels<T, K, DIFFUSE_D, V, P, 1, K, MID>(st, a, t);
}

// The rows of one wavefront's chunk: fill the levels, then one output row
// per level-0 row. SW: some lane's column pair is mirrored in memory.
template <typename T, int K, bool DIFFUSE_D, int V, bool SW, int MID = 0>
__device__ __forceinline__ void march_rows(const MarchArgs<T, V> &a) {
    MarchState<T, K, V> st;
#pragma unroll
    for (int l = 0; l < K; ++l)
#pragma unroll
        for (int r = 0; r < RING; ++r)
#pragma unroll
            for (int c = 0; c < 5; ++c)
#pragma unroll
                for (int v = 0; v < V; ++v)
                    st.ring[l][r][c][v] = T(0);

    // rows 0 .. 2K-1: fill the levels; from row 2K on every row yields output
    fetch_row<T, K, V, SW, 0>(st, a, 0);
    warm_up<T, K, DIFFUSE_D, V, SW, 0, MID>(st, a);
    constexpr int P0 = (2 * K) % RING;
    int t = 2 * K;
    for (; t + RING <= a.tend; t += RING) {
        steady_row<T, K, DIFFUSE_D, V, SW, P0, MID>(st, a, t);
        steady_row<T, K, DIFFUSE_D, V, SW, (P0 + 1) % RING, MID>(st, a, t + 1);
        steady_row<T, K, DIFFUSE_D, V, SW, (P0 + 2) % RING, MID>(st, a, t + 2);
        steady_row<T, K, DIFFUSE_D, V, SW, (P0 + 3) % RING, MID>(st, a, t + 3);
    }
    // last partial group of rows (only when the chunk height is not a multiple
    // of 4), nested so that no ring slot's older value stays live through the
    // loop for a tail row that might read it
    if (t < a.tend) {
        steady_row<T, K, DIFFUSE_D, V, SW, P0, MID>(st, a, t);
        if (t + 1 < a.tend) {
            steady_row<T, K, DIFFUSE_D, V, SW, (P0 + 1) % RING, MID>(st, a, t + 1);
            if (t + 2 < a.tend)
                steady_row<T, K, DIFFUSE_D, V, SW, (P0 + 2) % RING, MID>(st, a, t + 2);
        }
    }
}

// One wavefront: the strip whose first output column is x0, output rows
// [y0, y1), of the grid g with coefficients k; K steps from in to out,
// marching down the rows (up = false) or up. The stencil is symmetric in y,
// so both directions give the same bits. Chunks that meet at a row boundary
// march towards it (or away from it) together, so the K halo rows on each
// side of it are read by both wavefronts at about the same time and the
// second read is served from cache rather than HBM.
template <typename T, int K, bool DIFFUSE_D, int V, int MID = 0>
__device__ __forceinline__ void march_tile(const T *__restrict__ in, T *__restrict__ out,
                                           const GridDesc &g, const Coef<T> &k, int x0, int y0,
                                           int y1, bool up, T *__restrict__ mid_out = nullptr) {
    static_assert(MID >= 0 && MID < K, "the middle state is one of levels 1 .. K-1");
    using Geo = Strip<K, V>;
    const int lane = threadIdx.x & 63;
    MarchArgs<T, V> a;
    a.in = in;
    a.out = out;
    a.mid_out = mid_out;
    a.g = g;
    a.k = k;
    a.dir = up ? -1 : 1;
    a.j0 = up ? y1 - 1 + K : y0 - K;
    a.tend = y1 - y0 + 2 * K;
    a.xl = x0 - Geo::HX + lane * V;
#pragma unroll
    for (int v = 0; v < V; ++v) {
        a.xoff[v] = (unsigned)map_index(a.xl + v, g.nx, g.bc) * (unsigned)sizeof(T);
        const int pos = lane * V + v;
        a.out_col[v] = pos >= Geo::HX && pos < Geo::HX + Geo::WU && a.xl + v < g.nx;
    }
    a.swap = false;
    if constexpr (V == 2) {
        // xl is even and nx is even, so the pair maps onto one aligned pair of
        // memory columns, in order or (across a mirror) reversed
        a.swap = a.xoff[1] < a.xoff[0];
        if (a.swap)
            a.xoff[0] = a.xoff[1];
    }

    // Every strip but the few with a lane across a no-flux wall runs the
    // loop without the pair select (a wavefront-uniform branch).
    if constexpr (V == 2) {
        if (__builtin_amdgcn_ballot_w64(a.swap) != 0) {
            march_rows<T, K, DIFFUSE_D, V, true, MID>(a);
            return;
        }
    }
    march_rows<T, K, DIFFUSE_D, V, false, MID>(a);
}

template <typename T>
inline Coef<T> cast_coef(const StepCoef &s) {
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

}  // namespace sslbm
