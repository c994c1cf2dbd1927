// seird_device.h -- device-side building blocks of the SSLBM SEIRD step on
// gfx950: the per-node update, boundary index maps, the XCD-aware workgroup
// order and whole-wavefront lane shifts.
#pragma once

#include <hip/hip_runtime.h>

#include "sslbm.h"

namespace sslbm {

template <typename T>
struct Coef {
    T dl[5];
    T bdt, kE, kI, kR, kD;
};

// ---------------------------------------------------------------------------
// 1 / n where n is a positive normal number, else 0.
//
// FP32: the hardware reciprocal v_rcp_f32 (within 1 ulp for normal inputs,
// a fifth of the cost of the rounded division). It is not valid for
// subnormal inputs (it returns inf there), so positive subnormal n takes
// the zero branch with n <= 0.
// FP64: the rounded division, taken unconditionally and then selected (a
// division under the select measured slower: the compiler branches around
// it); 1 / n overflows for the smallest subnormal n, hence the same
// normal-number condition.
__device__ __forceinline__ float recip_or_zero(float n) {
    return n >= 0x1p-126f ? __builtin_amdgcn_rcpf(n) : 0.0f;
}
__device__ __forceinline__ double recip_or_zero(double n) {
    const double r = 1.0 / n;
    return n >= 0x1p-1022 ? r : 0.0;
}

// a / n where n > 0, else 0 (the force of infection is zero on cells with
// no contact-eligible population). FP32: a times the reciprocal, so a
// positive subnormal n also gives 0; the quotient dropped there is below
// 2^-126 beta dt, since a = dt beta S I with S, I <= n. FP64: the rounded
// quotient, exact for subnormal n too.
__device__ __forceinline__ float quotient_or_zero(float a, float n) {
    return a * recip_or_zero(n);
}
__device__ __forceinline__ double quotient_or_zero(double a, double n) {
    const double q = a / n;
    return n > 0.0 ? q : 0.0;
}

// SEIRD source increments Psi^C dt of one node, Eq. (sources) and Eq. (rhoD),
// from the node's densities at time t. The force of infection is zero where
// the contact-eligible population S + E + I + R is not positive.
template <typename T>
__device__ __forceinline__ void seird_increments(T S, T E, T I, T R, const Coef<T> &k, T &fdt,
                                                 T &rE, T &rI) {
    const T nc = (S + E) + (I + R);
    fdt = quotient_or_zero((k.bdt * S) * I, nc);
    rE = k.kE * E;
    rI = k.kI * I;
}

// One SSLBM update of the five compartments of one node.
//   c[C]  : densities at the node, time t
//   nb[C] : (north + south) + (east + west) neighbour densities, time t
// Eq. (sslbm_final_clean) on D2Q5 has rho_f = rho_b = c + (1/6) L c with
// L c = nb - 4 c, so rho(t+dt) = c + dl L c + Psi dt with dl = (2 tau - 1)/6.
// The diffusion part is evaluated as c + dl (nb - 4 c): its rounding errors
// have no preferred sign, so the total population only random-walks. (The
// cheaper dl nb + (1 - 4 dl) c rounds 1 - 4 dl once per launch, and that
// error shifts the total the same way every step.) The I balance folds
// k.kI * I into one fused multiply-add. The grouping of nb makes the result
// invariant, bit for bit, under every symmetry of the square lattice. Every
// kernel uses this function, so every launch shape gives the same bits.
template <typename T, bool DIFFUSE_D>
__device__ __forceinline__ void seird_update(const T c[5], const T nb[5], const Coef<T> &k,
                                             T out[5]) {
    T fdt, rE, rI;
    seird_increments(c[0], c[1], c[2], c[3], k, fdt, rE, rI);
    (void)rI;
    // nb - 4c with one rounding (4c is exact, so this equals nb - (4c))
    T diff[5];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        diff[q] = fma(k.dl[q], fma(T(-4), c[q], nb[q]), c[q]);
    diff[4] = DIFFUSE_D ? fma(k.dl[4], fma(T(-4), c[4], nb[4]), c[4]) : c[4];
    out[0] = diff[0] - fdt;
    out[1] = diff[1] + (fdt - rE);
    out[2] = diff[2] + fma(-k.kI, c[2], rE);
    out[3] = fma(k.kR, c[2], diff[3]);
    out[4] = fma(k.kD, c[2], diff[4]);
}

// ---------------------------------------------------------------------------
// Boundary handling by index map. A no-flux wall (neighbour outside := centre)
// is the same as extending the field by its mirror image about the wall: the
// mirrored field stays mirrored under the step, so several steps can be taken
// on the extended lattice and stay exact. Periodic wraps. Any integer i maps
// into [0, n).
__device__ __forceinline__ int map_index(int i, int n, int bc) {
    if ((unsigned)i < (unsigned)n)
        return i;
    if (bc == SSLBM_PERIODIC) {
        int m = i % n;
        return m < 0 ? m + n : m;
    }
    const int p = 2 * n;
    int m = i % p;
    if (m < 0)
        m += p;
    return m < n ? m : p - 1 - m;
}

// ---------------------------------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X, each
// with its own L2. Renumber them so that every XCD works on one contiguous
// range of tiles; neighbouring tiles then share halo rows in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    constexpr int X = 8;
    const int q = nb / X, r = nb % X;
    const int xcd = b % X, l = b / X;
    return xcd < r ? xcd * (q + 1) + l : r * (q + 1) + (xcd - r) * q + l;
}

// ---------------------------------------------------------------------------
// Whole-wavefront lane shifts by one (DPP wave_shr:1 / wave_shl:1). Lane 0
// (resp. 63) receives zero; those edge lanes are halo lanes whose results are
// never stored. With a zero fill the shift needs no copy of an old value and
// folds into the add that consumes it.
__device__ __forceinline__ int lane_from_left_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ int lane_from_right_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, true);
}
__device__ __forceinline__ float lane_from_left(float v) {
    return __int_as_float(lane_from_left_i(__float_as_int(v)));
}
__device__ __forceinline__ float lane_from_right(float v) {
    return __int_as_float(lane_from_right_i(__float_as_int(v)));
}
__device__ __forceinline__ double lane_from_left(double v) {
    long long b = __double_as_longlong(v);
    int lo = lane_from_left_i((int)(b & 0xffffffffll));
    int hi = lane_from_left_i((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane_from_right(double v) {
    long long b = __double_as_longlong(v);
    int lo = lane_from_right_i((int)(b & 0xffffffffll));
    int hi = lane_from_right_i((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sums of a value and its neighbour lane's, each one v_add_f32_dpp. This
// compiler fuses a DPP move into the add that consumes it only part of the
// time, so these write the fused instruction. The compiler does not see the
// DPP read inside the asm, so each one starts with s_nop 1: the two wait
// states gfx9 requires between a VALU write of a register and its DPP read.
// Lanes without a neighbour read 0 (bound_ctrl), as lane_from_left/right.
//   x + lane_from_left(x)
__device__ __forceinline__ float add_from_left(float x) {
    float r;
    asm("s_nop 1\n\tv_add_f32_dpp %0, %1, %1 wave_shr:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=v"(r)
        : "v"(x));
    return r;
}
//   lane_from_right(x) + x
__device__ __forceinline__ float add_from_right(float x) {
    float r;
    asm("s_nop 1\n\tv_add_f32_dpp %0, %1, %1 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=v"(r)
        : "v"(x));
    return r;
}
//   lane_from_right(x) + y
__device__ __forceinline__ float add_right_to(float x, float y) {
    float r;
    asm("s_nop 1\n\tv_add_f32_dpp %0, %1, %2 wave_shl:1 row_mask:0xf bank_mask:0xf bound_ctrl:1"
        : "=v"(r)
        : "v"(x), "v"(y));
    return r;
}
__device__ __forceinline__ double add_from_left(double x) { return x + lane_from_left(x); }
__device__ __forceinline__ double add_from_right(double x) { return lane_from_right(x) + x; }
__device__ __forceinline__ double add_right_to(double x, double y) {
    return lane_from_right(x) + y;
}

}  // namespace sslbm
