// adjoint_kernels.hip -- reverse (adjoint) SSLBM step on gfx950.
//
// For a loss J of the state at the end of a run, the adjoint field
// lam(t) = dJ/d rho(t) obeys lam(t) = A(rho(t))^T lam(t + dt), A the Jacobian
// of one step (Eq. sslbm_final_clean with the sources of Eq. (sources) and
// Eq. (rhoD)). On D2Q5 the transport part of the step is c + dl L c, L the
// five-point Laplacian with periodic wrap or mirror (no-flux) ghosts; L is
// symmetric on both, so its transpose is the same stencil applied to lam.
// The source part is pointwise: its transpose multiplies lam(x) by the
// transposed 5x5 Jacobian of Psi dt at rho(x, t).
//
// Parameter gradients of one step, summed over the grid (dt and the factors
// that do not vary in space are applied once, at the end of a run):
//   dJ/dbeta  += dt sum (lamE - lamS) S I / Nc
//   dJ/dalpha += dt sum (lamI - lamE) E
//   dJ/dgamma += dt sum (-lamI + (1 - phi) lamR + phi lamD) I
//   dJ/dphi   += gamma dt sum (lamD - lamR) I
//   dJ/dd^C   += dt/dx^2 sum lam^C L rho^C = dt/dx^2 sum rho^C L lam^C
// (the last by the symmetry of L: the kernel needs rho only at the node).
//
// Layout and traversal are those of the forward pass at one step per pass:
// one wavefront per strip of 64 columns (62 output columns and one halo
// column on each side) walking down a chunk of rows; lam rows sit in a
// 4-slot register ring unrolled so that slots are compile-time constants,
// east/west neighbours come through DPP lane shifts, rows are addressed by
// buffer descriptors. Per output row the wavefront reads one row of lam and
// one row of rho (5 fields each) and writes one row of the new lam.
//
// The nine sums are kept per lane in FP64, reduced across the wavefront at
// the end of its chunk and added to the wavefront's own slot of a partials
// buffer; the same wavefront owns the same slot at every step, so a run's
// sums are deterministic. A final one-block kernel adds the slots in a fixed
// order and applies the factors.
#include <hip/hip_runtime.h>

#include "adjoint_internal.h"
#include "march_core.h"

namespace sslbm {

namespace {

constexpr int ADJ_HX = 1;                 // halo columns per strip side
constexpr int ADJ_WU = 64 - 2 * ADJ_HX;   // output columns per strip

template <typename T>
struct AdjState {
    T lam[RING][5];  // lam(t + dt) rows, ring slot = row mod 4
    T rho[2][5];     // rho(t) of the output row (and of the next one, in flight)
};

template <typename T>
struct AdjArgs {
    const T *__restrict__ rho;
    const T *__restrict__ lam;
    T *__restrict__ out;
    GridDesc g;
    Coef<T> k;
    unsigned xoff;  // byte offset of the lane's memory column within a row
    unsigned xo;    // byte offset of the lane's output column
    bool out_col;   // the lane's column is an output column
    int j0;         // first lam row read (one above the first output row)
};

template <typename T, int SL>
__device__ __forceinline__ void fetch_lam(AdjState<T> &st, const AdjArgs<T> &a, int t) {
    const long long row = (long long)map_index(a.j0 + t, a.g.ny, a.g.bc) * a.g.nx;
#pragma unroll
    for (int c = 0; c < 5; ++c)
        st.lam[SL][c] =
            buf_load(row_resource(a.lam + (c * a.g.plane + row), a.g.nx), a.xoff, T(0));
}

template <typename T, int SR>
__device__ __forceinline__ void fetch_rho(AdjState<T> &st, const AdjArgs<T> &a, int y) {
    const long long row = (long long)map_index(y, a.g.ny, a.g.bc) * a.g.nx;
#pragma unroll
    for (int c = 0; c < 5; ++c)
        st.rho[SR][c] =
            buf_load(row_resource(a.rho + (c * a.g.plane + row), a.g.nx), a.xoff, T(0));
}

// The reverse update of one node: o = A(rho)^T lam at the node, from the
// adjoint field at the node (lc), its five-point Laplacian (lap) and the
// state at the node (rho).
// Populations below `below` are scaled by `scale` (and S I / Nc back by
// `unscale`) in the reverse step: every positive subnormal Nc then becomes
// a normal number.
template <typename T>
struct TinyPopulation;
template <>
struct TinyPopulation<float> {
    static constexpr float below = 0x1p-100f, scale = 0x1p64f, unscale = 0x1p-64f;
};
template <>
struct TinyPopulation<double> {
    static constexpr double below = 0x1p-960, scale = 0x1p512, unscale = 0x1p-512;
};

template <typename T, bool DIFFUSE_D>
__device__ __forceinline__ void adjoint_node(const T lc[5], const T lap[5], const T rho[5],
                                             const Coef<T> &k, T o[5], T &g, T &de, T &sir) {
#pragma unroll
    for (int c = 0; c < 4; ++c)
        o[c] = fma(k.dl[c], lap[c], lc[c]);
    o[4] = DIFFUSE_D ? fma(k.dl[4], lap[4], lc[4]) : lc[4];

    const T S = rho[0], E = rho[1], I = rho[2], R = rho[3];
    const T nc = (S + E) + (I + R);
    // F = beta S I / Nc is homogeneous of degree one in (S, E, I, R), so its
    // derivatives keep their size as the population shrinks to zero. A tiny
    // population is first scaled up by an exact power of two (which leaves
    // every ratio below unchanged) so that 1 / Nc stays a normal number; at
    // ordinary sizes the scale is 1 and changes no bit.
    const bool tiny = nc < TinyPopulation<T>::below;
    const T up = tiny ? TinyPopulation<T>::scale : T(1);
    const T Su = S * up, Iu = I * up;
    const T r = recip_or_zero(nc * up);            // 1 / (up Nc), or 0 where F = 0
    const T siru = (Su * Iu) * r;                  // up S I / Nc
    sir = siru * (tiny ? TinyPopulation<T>::unscale : T(1));  // S I / Nc = F / beta
    const T qi = k.bdt * (Iu * r);                 // dt dF/dS + dt F/Nc
    const T qs = k.bdt * (Su * r);                 // dt dF/dI + dt F/Nc
    const T w = k.bdt * (siru * r);                // dt F / Nc
    g = lc[1] - lc[0];                             // F moves S -> E
    de = lc[2] - lc[1];                            // alpha E moves E -> I
    o[0] = fma(g, qi - w, o[0]);
    o[1] = fma(de, k.kE, fma(-g, w, o[1]));
    o[2] = fma(g, qs - w, o[2]) + (fma(lc[3], k.kR, lc[4] * k.kD) - lc[2] * k.kI);
    o[3] = fma(-g, w, o[3]);
}

// The node's contributions to the nine parameter-gradient sums.
template <typename T>
__device__ __forceinline__ void adjoint_sums(const T lc[5], const T lap[5], const T rho[5], T g,
                                             T de, T sir, double acc[ADJ_SUMS]) {
    acc[0] += (double)(g * sir);
    acc[1] += (double)(de * rho[1]);
    acc[2] += (double)(lc[2] * rho[2]);
    acc[3] += (double)(lc[3] * rho[2]);
    acc[4] += (double)(lc[4] * rho[2]);
#pragma unroll
    for (int c = 0; c < 5; ++c)
        acc[5 + c] += (double)(rho[c] * lap[c]);
}

// Output row j0 + t - 1 at phase P = t mod 4: lam rows t-2, t-1, t are in
// slots P-2, P-1, P; rho of the row is in slot P mod 2.
template <typename T, bool DIFFUSE_D, int P>
__device__ __forceinline__ void adjoint_row(AdjState<T> &st, const AdjArgs<T> &a, int t,
                                            double acc[ADJ_SUMS]) {
    constexpr int su = (P + 2) % RING, sm = (P + 3) % RING, sd = P % RING, sr = P % 2;
    T lc[5], lap[5], o[5], g, de, sir;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        lc[c] = st.lam[sm][c];
        const T nb = (st.lam[su][c] + st.lam[sd][c]) +
                     add_right_to(lc[c], lane_from_left(lc[c]));
        lap[c] = fma(T(-4), lc[c], nb);
    }
    adjoint_node<T, DIFFUSE_D>(lc, lap, st.rho[sr], a.k, o, g, de, sir);
    if (a.out_col) {
        const long long row = (long long)(a.j0 + t - 1) * a.g.nx;
#pragma unroll
        for (int c = 0; c < 5; ++c)
            buf_store(row_resource(a.out + (c * a.g.plane + row), a.g.nx), a.xo, o[c]);
        adjoint_sums(lc, lap, st.rho[sr], g, de, sir, acc);
    }
}

// Steady row t at phase P: fetch lam row t + 1 and the rho row of the next
// output row, then the output row of t.
template <typename T, bool DIFFUSE_D, int P>
__device__ __forceinline__ void adjoint_steady(AdjState<T> &st, const AdjArgs<T> &a, int t,
                                               double acc[ADJ_SUMS]) {
    fetch_lam<T, (P + 1) % RING>(st, a, t + 1);
    fetch_rho<T, (P + 1) % 2>(st, a, a.j0 + t);
    adjoint_row<T, DIFFUSE_D, P>(st, a, t, acc);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        v += __shfl_xor(v, m, 64);
    return v;
}

template <typename T, bool DIFFUSE_D>
__global__ __launch_bounds__(BLOCK_THREADS) void adjoint_kernel(
    const T *__restrict__ rho, const T *__restrict__ lam, T *__restrict__ out, GridDesc g,
    Coef<T> k, int strips, int chunks, int rows, double *__restrict__ partials, int first) {
    const int wave = __builtin_amdgcn_readfirstlane(
        xcd_tile(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + (threadIdx.x >> 6));
    if (wave >= strips * chunks)
        return;  // whole wavefront leaves together
    const int strip = wave / chunks, chunk = wave - strip * chunks;
    const int y0 = chunk * rows;
    const int y1 = min(y0 + rows, g.ny);
    const int lane = threadIdx.x & 63;
    const int xl = strip * ADJ_WU - ADJ_HX + lane;

    AdjArgs<T> a;
    a.rho = rho;
    a.lam = lam;
    a.out = out;
    a.g = g;
    a.k = k;
    a.xoff = (unsigned)map_index(xl, g.nx, g.bc) * (unsigned)sizeof(T);
    a.xo = (unsigned)xl * (unsigned)sizeof(T);
    a.out_col = lane >= ADJ_HX && lane < ADJ_HX + ADJ_WU && xl < g.nx;
    a.j0 = y0 - 1;

    AdjState<T> st;
#pragma unroll
    for (int s = 0; s < RING; ++s)
#pragma unroll
        for (int c = 0; c < 5; ++c)
            st.lam[s][c] = T(0);
    double acc[ADJ_SUMS];
#pragma unroll
    for (int j = 0; j < ADJ_SUMS; ++j)
        acc[j] = 0.0;

    // lam rows j0 .. y1 (t = 0 .. tend); the output row of t is j0 + t - 1
    const int tend = y1 - y0 + 2;
    fetch_lam<T, 0>(st, a, 0);
    fetch_lam<T, 1>(st, a, 1);
    fetch_lam<T, 2>(st, a, 2);
    fetch_rho<T, 0>(st, a, y0);
    int t = 2;
    for (; t + RING <= tend; t += RING) {
        adjoint_steady<T, DIFFUSE_D, 2>(st, a, t, acc);
        adjoint_steady<T, DIFFUSE_D, 3>(st, a, t + 1, acc);
        adjoint_steady<T, DIFFUSE_D, 0>(st, a, t + 2, acc);
        adjoint_steady<T, DIFFUSE_D, 1>(st, a, t + 3, acc);
    }
    if (t < tend)
        adjoint_steady<T, DIFFUSE_D, 2>(st, a, t, acc);
    if (t + 1 < tend)
        adjoint_steady<T, DIFFUSE_D, 3>(st, a, t + 1, acc);
    if (t + 2 < tend)
        adjoint_steady<T, DIFFUSE_D, 0>(st, a, t + 2, acc);

#pragma unroll
    for (int j = 0; j < ADJ_SUMS; ++j)
        acc[j] = wave_sum(acc[j]);
    if (lane == 0) {
        double *slot = partials + (long long)wave * ADJ_SLOT;
#pragma unroll
        for (int j = 0; j < ADJ_SUMS; ++j)
            slot[j] = first ? acc[j] : slot[j] + acc[j];
    }
}

// --------------------------------------------------- two steps per pass
// lam(n) from lam(n + 2) and the state rho(n): the state of step n + 1 is
// recomputed in registers by one forward level (the SSLBM update of the
// pass kernels), the reverse level n + 1 follows it one row behind and the
// reverse level n one row behind that. Per output row the wavefront reads
// one row of rho(n) and one of lam(n + 2) and writes one of lam(n): the
// bytes of one single step for two steps of work. A strip has two halo
// columns per side (60 output columns); a chunk reads two halo rows above
// and below.
constexpr int F_HX = 2, F_WU = 64 - 2 * F_HX;

template <typename T>
struct Fused2State {
    T rho0[RING][5];  // rho(n) rows, ring slot = row mod 4
    T lam2[RING][5];  // lam(n + 2) rows
    T lam1[RING][5];  // lam(n + 1) rows (computed)
};

template <typename T>
struct Fused2Args {
    const T *__restrict__ rho;
    const T *__restrict__ lam;
    T *__restrict__ out;
    GridDesc g;
    Coef<T> k;
    unsigned xoff, xo;
    bool out_col;
    int j0;    // first row read: y0 - 2 marching down, y1 + 1 marching up
    int dir;   // +1: rows in increasing order, -1: decreasing
    int tend;  // rows read: y1 - y0 + 4
};

template <typename T, int SL>
__device__ __forceinline__ void fused_fetch(Fused2State<T> &st, const Fused2Args<T> &a, int t) {
    const long long row = (long long)map_index(a.j0 + a.dir * t, a.g.ny, a.g.bc) * a.g.nx;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        st.rho0[SL][c] =
            buf_load(row_resource(a.rho + (c * a.g.plane + row), a.g.nx), a.xoff, T(0));
        st.lam2[SL][c] =
            buf_load(row_resource(a.lam + (c * a.g.plane + row), a.g.nx), a.xoff, T(0));
    }
}

// Row t at phase P = t mod 4 (rows j0 + t - 2 .. j0 + t are in slots
// P + 2, P + 3, P): forward level and reverse level n + 1 for row t - 1,
// then (OUT) reverse level n for row t - 2.
template <typename T, bool DIFFUSE_D, int P, bool OUT>
__device__ __forceinline__ void fused_row(Fused2State<T> &st, const Fused2Args<T> &a, int t,
                                          double acc[ADJ_SUMS]) {
    constexpr int su = (P + 2) % RING, sm = (P + 3) % RING, sd = P % RING;
    fused_fetch<T, (P + 1) % RING>(st, a, t + 1);
    // rho(n + 1) at row t - 1
    T cen[5], nb[5], r1[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
        cen[c] = st.rho0[sm][c];
        nb[c] = (c < 4 || DIFFUSE_D) ? (st.rho0[su][c] + st.rho0[sd][c]) +
                                           add_right_to(cen[c], lane_from_left(cen[c]))
                                     : T(0);
    }
    seird_update<T, DIFFUSE_D>(cen, nb, a.k, r1);
    // lam(n + 1) at row t - 1
    {
        T lc[5], lap[5], o[5], g, de, sir;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            lc[c] = st.lam2[sm][c];
            const T n2 = (st.lam2[su][c] + st.lam2[sd][c]) +
                         add_right_to(lc[c], lane_from_left(lc[c]));
            lap[c] = fma(T(-4), lc[c], n2);
        }
        adjoint_node<T, DIFFUSE_D>(lc, lap, r1, a.k, o, g, de, sir);
#pragma unroll
        for (int c = 0; c < 5; ++c)
            st.lam1[sm][c] = o[c];
        // rows y0 .. y1 - 1 only: the halo rows belong to the neighbouring chunks
        if (a.out_col && t >= 3 && t < a.tend - 1)
            adjoint_sums(lc, lap, r1, g, de, sir, acc);
    }
    if constexpr (OUT) {
        // lam(n) at row t - 2, from lam(n + 1) rows t - 3 .. t - 1
        constexpr int lu = (P + 1) % RING, lm = (P + 2) % RING, ld = (P + 3) % RING;
        T lc[5], lap[5], o[5], g, de, sir;
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            lc[c] = st.lam1[lm][c];
            const T n1 = (st.lam1[lu][c] + st.lam1[ld][c]) +
                         add_right_to(lc[c], lane_from_left(lc[c]));
            lap[c] = fma(T(-4), lc[c], n1);
        }
        adjoint_node<T, DIFFUSE_D>(lc, lap, st.rho0[lm], a.k, o, g, de, sir);
        if (a.out_col) {
            const long long row = (long long)(a.j0 + a.dir * (t - 2)) * a.g.nx;
#pragma unroll
            for (int c = 0; c < 5; ++c)
                buf_store(row_resource(a.out + (c * a.g.plane + row), a.g.nx), a.xo, o[c]);
            adjoint_sums(lc, lap, st.rho0[lm], g, de, sir, acc);
        }
    }
}

template <typename T, bool DIFFUSE_D>
__global__ __launch_bounds__(BLOCK_THREADS) void adjoint2_kernel(
    const T *__restrict__ rho, const T *__restrict__ lam, T *__restrict__ out, GridDesc g,
    Coef<T> k, int strips, int chunks, int rows, double *__restrict__ partials) {
    const int wave = __builtin_amdgcn_readfirstlane(
        xcd_tile(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + (threadIdx.x >> 6));
    if (wave >= strips * chunks)
        return;  // whole wavefront leaves together
    const int strip = wave / chunks, chunk = wave - strip * chunks;
    const int y0 = chunk * rows;
    const int y1 = min(y0 + rows, g.ny);
    const int lane = threadIdx.x & 63;
    const int xl = strip * F_WU - F_HX + lane;

    Fused2Args<T> a;
    a.rho = rho;
    a.lam = lam;
    a.out = out;
    a.g = g;
    a.k = k;
    a.xoff = (unsigned)map_index(xl, g.nx, g.bc) * (unsigned)sizeof(T);
    a.xo = (unsigned)xl * (unsigned)sizeof(T);
    a.out_col = lane >= F_HX && lane < F_HX + F_WU && xl < g.nx;
    // odd chunks march up the rows, so that two chunks meeting at a row
    // boundary read the halo rows around it at about the same time (the
    // second read then comes from cache); the stencil is symmetric in y
    const bool up = (chunk & 1) != 0;
    a.dir = up ? -1 : 1;
    a.j0 = up ? y1 + 1 : y0 - 2;
    a.tend = y1 - y0 + 4;

    Fused2State<T> st;
#pragma unroll
    for (int s = 0; s < RING; ++s)
#pragma unroll
        for (int c = 0; c < 5; ++c) {
            st.rho0[s][c] = T(0);
            st.lam2[s][c] = T(0);
            st.lam1[s][c] = T(0);
        }
    double acc[ADJ_SUMS];
#pragma unroll
    for (int j = 0; j < ADJ_SUMS; ++j)
        acc[j] = 0.0;

    fused_fetch<T, 0>(st, a, 0);
    fused_fetch<T, 1>(st, a, 1);
    fused_fetch<T, 2>(st, a, 2);
    fused_row<T, DIFFUSE_D, 2, false>(st, a, 2, acc);
    fused_row<T, DIFFUSE_D, 3, false>(st, a, 3, acc);
    int t = 4;
    for (; t + RING <= a.tend; t += RING) {
        fused_row<T, DIFFUSE_D, 0, true>(st, a, t, acc);
        fused_row<T, DIFFUSE_D, 1, true>(st, a, t + 1, acc);
        fused_row<T, DIFFUSE_D, 2, true>(st, a, t + 2, acc);
        fused_row<T, DIFFUSE_D, 3, true>(st, a, t + 3, acc);
    }
    // tail rows nested, so that no older ring value stays live through the
    // loop for a tail row that might read it
    if (t < a.tend) {
        fused_row<T, DIFFUSE_D, 0, true>(st, a, t, acc);
        if (t + 1 < a.tend) {
            fused_row<T, DIFFUSE_D, 1, true>(st, a, t + 1, acc);
            if (t + 2 < a.tend)
                fused_row<T, DIFFUSE_D, 2, true>(st, a, t + 2, acc);
        }
    }

#pragma unroll
    for (int j = 0; j < ADJ_SUMS; ++j)
        acc[j] = wave_sum(acc[j]);
    if (lane == 0) {
        double *slot = partials + (long long)wave * ADJ_SLOT;
#pragma unroll
        for (int j = 0; j < ADJ_SUMS; ++j)
            slot[j] += acc[j];
    }
}

__global__ __launch_bounds__(256) void zero_kernel(double *__restrict__ p, long long n) {
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e < n)
        p[e] = 0.0;
}

// Sum of the slots in a fixed order (slot-strided per thread, then a fixed
// tree), scaled into the nine parameter gradients and added to grad. Each
// thread reads whole slots, so its loads are independent and contiguous.
constexpr int FINISH_THREADS = 512;

__global__ __launch_bounds__(FINISH_THREADS) void adjoint_finish_kernel(
    const double *__restrict__ partials, int slots, AdjFactors f, double *__restrict__ grad) {
    __shared__ double part[ADJ_SUMS][FINISH_THREADS];
    const int tid = threadIdx.x;
    double s[ADJ_SUMS];
#pragma unroll
    for (int j = 0; j < ADJ_SUMS; ++j)
        s[j] = 0.0;
    for (int i = tid; i < slots; i += FINISH_THREADS) {
        const double *slot = partials + (long long)i * ADJ_SLOT;
#pragma unroll
        for (int j = 0; j < ADJ_SUMS; ++j)
            s[j] += slot[j];
    }
#pragma unroll
    for (int j = 0; j < ADJ_SUMS; ++j)
        part[j][tid] = s[j];
    __syncthreads();
    for (int h = FINISH_THREADS / 2; h >= 1; h >>= 1) {
        if (tid < h) {
#pragma unroll
            for (int j = 0; j < ADJ_SUMS; ++j)
                part[j][tid] += part[j][tid + h];
        }
        __syncthreads();
    }
    if (tid < 9) {
        double v;
        switch (tid) {
        case 0: v = f.dt * part[0][0]; break;
        case 1: v = f.dt * part[1][0]; break;
        case 2: v = f.dt * ((1.0 - f.phi) * part[3][0] + f.phi * part[4][0] - part[2][0]); break;
        case 3: v = f.gamma_dt * (part[4][0] - part[3][0]); break;
        default: v = f.dt_dx2 * part[5 + (tid - 4)][0]; break;
        }
        grad[tid] += v;
    }
}

template <typename T, bool DD>
hipError_t launch_t(const void *rho, const void *lam, void *out, const GridDesc &g,
                    const StepCoef &k, const AdjShape &s, double *partials, bool first,
                    hipStream_t st) {
    const int waves = s.strips * s.chunks;
    const int blocks = (waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
    hipLaunchKernelGGL((adjoint_kernel<T, DD>), dim3((unsigned)blocks), dim3(BLOCK_THREADS), 0,
                       st, static_cast<const T *>(rho), static_cast<const T *>(lam),
                       static_cast<T *>(out), g, cast_coef<T>(k), s.strips, s.chunks, s.rows,
                       partials, first ? 1 : 0);
    return hipGetLastError();
}

}  // namespace

AdjShape adjoint_shape(int nx, int ny) {
    AdjShape s;
    s.strips = (nx + ADJ_WU - 1) / ADJ_WU;
    // The shortest chunks (at least 8 rows) for which the grid fits in one
    // workgroup of 4 wavefronts per CU of the 256 of an MI355X: measured at
    // 1024 x 1024 in FP64, one wavefront per SIMD on long chunks beats more
    // wavefronts on short ones (25.5 us per step at 24 rows, 31 us at 16 rows
    // when 16 CUs get a second workgroup, 29 us at 3 rows), since every chunk
    // re-reads two halo rows and restarts its row pipeline.
    const long long target = 256 * WAVES_PER_BLOCK;
    long long chunks = target / s.strips;
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

hipError_t launch_adjoint(int dtype, const void *rho, const void *lam, void *out,
                          const GridDesc &g, const StepCoef &k, const AdjShape &s,
                          double *partials, bool first, hipStream_t st) {
    if (dtype == SSLBM_F32)
        return k.diffuse_d ? launch_t<float, true>(rho, lam, out, g, k, s, partials, first, st)
                           : launch_t<float, false>(rho, lam, out, g, k, s, partials, first, st);
    return k.diffuse_d ? launch_t<double, true>(rho, lam, out, g, k, s, partials, first, st)
                       : launch_t<double, false>(rho, lam, out, g, k, s, partials, first, st);
}

AdjShape adjoint2_shape(int nx, int ny) {
    AdjShape s;
    s.strips = (nx + F_WU - 1) / F_WU;
    // as adjoint_shape: one workgroup of four wavefronts per CU, chunks of
    // at least 8 rows
    const long long target = 256 * WAVES_PER_BLOCK;
    long long chunks = target / s.strips;
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

template <typename T, bool DD>
static hipError_t launch2_t(const void *rho, const void *lam, void *out, const GridDesc &g,
                            const StepCoef &k, const AdjShape &s, double *partials,
                            hipStream_t st) {
    const int waves = s.strips * s.chunks;
    const int blocks = (waves + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
    hipLaunchKernelGGL((adjoint2_kernel<T, DD>), dim3((unsigned)blocks), dim3(BLOCK_THREADS), 0,
                       st, static_cast<const T *>(rho), static_cast<const T *>(lam),
                       static_cast<T *>(out), g, cast_coef<T>(k), s.strips, s.chunks, s.rows,
                       partials);
    return hipGetLastError();
}

hipError_t launch_adjoint2(int dtype, const void *rho, const void *lam, void *out,
                           const GridDesc &g, const StepCoef &k, const AdjShape &s,
                           double *partials, hipStream_t st) {
    if (dtype == SSLBM_F32)
        return k.diffuse_d ? launch2_t<float, true>(rho, lam, out, g, k, s, partials, st)
                           : launch2_t<float, false>(rho, lam, out, g, k, s, partials, st);
    return k.diffuse_d ? launch2_t<double, true>(rho, lam, out, g, k, s, partials, st)
                       : launch2_t<double, false>(rho, lam, out, g, k, s, partials, st);
}

hipError_t launch_zero(double *p, long long n, hipStream_t st) {
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
    return hipGetLastError();
}

hipError_t launch_adjoint_finish(const double *partials, int slots, const AdjFactors &f,
                                 double *grad, hipStream_t st) {
    hipLaunchKernelGGL(adjoint_finish_kernel, dim3(1), dim3(FINISH_THREADS), 0, st, partials,
                       slots, f, grad);
    return hipGetLastError();
}

}  // namespace sslbm
