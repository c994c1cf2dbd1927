// model_api.cpp -- host side of the generic-model entry points of sslbm.h:
// validation of the model (lattice, compartments, transitions, stability)
// before any HIP call, derived constants, and the step and run loops.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <new>

#include "model_internal.h"
#include "sslbm.h"

struct sslbm_model {
    int nx = 0, ny = 0, dtype = 0, bc = 0, lattice = 5;
    sslbm::ModelCoefHost coef{};
    int last_hip = 0;
    void *table = nullptr;  // device transition table, uploaded on first use
    int table_device = -1;
    int blocking = 0;  // steps per pass of sslbm_model_run (0: automatic)
};

namespace {

constexpr int MAX_SIDE = 1 << 20;

sslbm_status hip_status(sslbm_model *m, hipError_t e) {
    if (e == hipSuccess)
        return SSLBM_OK;
    m->last_hip = (int)e;
    return SSLBM_E_HIP;
}

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

// Steps per pass of sslbm_model_run: the caller's choice, else 3. Measured
// at 4096 x 4096 with the six-compartment model, each depth at the
// wavefronts per SIMD its registers allow: FP32 D2Q5 71 / 140 / 165 / 162
// GLUPS and D2Q9 73 / 138 / 156 / 153 at 1 / 2 / 3 / 4 steps per pass;
// FP64 D2Q5 97 and D2Q9 87 at 3 steps, 77 and 69 at 4 (two wavefronts per
// SIMD).
constexpr int MODEL_AUTO_K = 3;

int resolved_blocking(const sslbm_model *m) {
    return m->blocking > 0 ? m->blocking : MODEL_AUTO_K;
}

size_t state_bytes(const sslbm_model *m) {
    return (size_t)m->coef.m * m->nx * m->ny * (m->dtype == SSLBM_F32 ? 4 : 8);
}

// The device transition table on the current device (uploaded once; a
// model stays on the device it first ran on).
sslbm_status ensure_table(sslbm_model *m) {
    int dev = 0;
    sslbm_status st = hip_status(m, hipGetDevice(&dev));
    if (st != SSLBM_OK)
        return st;
    if (m->table)
        return m->table_device == dev ? SSLBM_OK : SSLBM_E_UNSUPPORTED;
    const size_t bytes = sslbm::model_table_bytes(m->dtype);
    alignas(16) unsigned char host[sslbm::model_table_bytes(SSLBM_F64)] = {};
    sslbm::model_table(m->coef, m->dtype, host);
    st = hip_status(m, hipMalloc(&m->table, bytes));
    if (st != SSLBM_OK)
        return st;
    st = hip_status(m, hipMemcpy(m->table, host, bytes, hipMemcpyHostToDevice));
    if (st != SSLBM_OK) {
        (void)hipFree(m->table);
        m->table = nullptr;
        return st;
    }
    m->table_device = dev;
    return SSLBM_OK;
}

sslbm::GridDesc grid_of(const sslbm_model *m) {
    sslbm::GridDesc g;
    g.nx = m->nx;
    g.ny = m->ny;
    g.plane = (long long)m->nx * m->ny;
    g.bc = m->bc;
    return g;
}

}  // namespace

extern "C" {

sslbm_status sslbm_model_create(sslbm_model **out, int nx, int ny, int dtype, int bc,
                                int lattice, int compartments, const double *d, const int *counted,
                                double dx, double dt, int ntransitions, const sslbm_transition *t) {
    if (!out)
        return SSLBM_E_ARG;
    *out = nullptr;
    if (nx < 1 || ny < 1 || nx > MAX_SIDE || ny > MAX_SIDE || (long long)nx * ny > (1ll << 33) ||
        (dtype != SSLBM_F32 && dtype != SSLBM_F64) || (bc != SSLBM_PERIODIC && bc != SSLBM_NOFLUX) ||
        (lattice != 5 && lattice != 9) || compartments < 1 ||
        compartments > SSLBM_MAX_COMPARTMENTS || !d || !counted || ntransitions < 0 ||
        ntransitions > SSLBM_MAX_TRANSITIONS || (ntransitions && !t) || !std::isfinite(dx) ||
        !std::isfinite(dt) || dx <= 0.0 || dt <= 0.0)
        return SSLBM_E_ARG;
    sslbm::ModelCoefHost k{};
    k.m = compartments;
    k.ntrans = ntransitions;
    double outflow[SSLBM_MAX_COMPARTMENTS] = {};
    for (int c = 0; c < compartments; ++c) {
        if (!std::isfinite(d[c]) || d[c] < 0.0)
            return SSLBM_E_ARG;
        k.dl[c] = d[c] * dt / (dx * dx);
        if (counted[c])
            k.counted |= 1u << c;
    }
    for (int r = 0; r < ntransitions; ++r) {
        const sslbm_transition &x = t[r];
        if (x.src < 0 || x.src >= compartments || x.dst < -1 || x.dst >= compartments ||
            x.dst == x.src || x.catalyst < -1 || x.catalyst >= compartments ||
            (x.frequency != 0 && x.frequency != 1) || !std::isfinite(x.rate) || x.rate < 0.0)
            return SSLBM_E_ARG;
        k.src[r] = x.src;
        k.dst[r] = x.dst;
        k.cat[r] = x.catalyst;
        k.freq[r] = x.frequency;
        k.rate_dt[r] = x.rate * dt;
        // per-node outflow rate of src: bounded by rate when the catalyst is
        // absent, or is a counted compartment of a frequency-dependent term
        // (C_cat / N <= 1); density-dependent catalysis is left unbounded
        if (x.catalyst < 0 || (x.frequency && counted[x.catalyst]))
            outflow[x.src] += x.rate;
    }
    // linear stability of the explicit update, as for the SEIRD step:
    // (2 tau - 1) max(1 - Lambda) + dt * outflow <= 2, with
    // max(1 - Lambda) = 4/3 on D2Q5 and 8/9 on D2Q9, 2 tau - 1 = 6 dl
    const double spread = lattice == 5 ? 8.0 : 16.0 / 3.0;
    for (int c = 0; c < compartments; ++c)
        if (spread * k.dl[c] + dt * outflow[c] > 2.0 * (1.0 + 1e-12))
            return SSLBM_E_UNSTABLE;
    sslbm_model *m = new (std::nothrow) sslbm_model();
    if (!m)
        return SSLBM_E_NOMEM;
    m->nx = nx;
    m->ny = ny;
    m->dtype = dtype;
    m->bc = bc;
    m->lattice = lattice;
    m->coef = k;
    *out = m;
    return SSLBM_OK;
}

sslbm_status sslbm_model_step(sslbm_model *m, const void *rho_in, void *rho_out, void *hip_stream) {
    if (!m || !rho_in || !rho_out)
        return SSLBM_E_ARG;
    const size_t bytes = state_bytes(m);
    if (overlap(rho_in, bytes, rho_out, bytes))
        return SSLBM_E_ALIAS;
    const sslbm_status st = ensure_table(m);
    if (st != SSLBM_OK)
        return st;
    return hip_status(m, sslbm::launch_model(m->dtype, m->lattice, rho_in, rho_out, grid_of(m),
                                             m->coef, m->table, 1, (hipStream_t)hip_stream));
}

sslbm_status sslbm_model_run(sslbm_model *m, void *rho, void *scratch, long long nsteps,
                             void *hip_stream) {
    if (!m || !rho || !scratch || nsteps < 0)
        return SSLBM_E_ARG;
    const size_t bytes = state_bytes(m);
    if (overlap(rho, bytes, scratch, bytes))
        return SSLBM_E_ALIAS;
    if (nsteps == 0)
        return SSLBM_OK;
    const sslbm_status tst = ensure_table(m);
    if (tst != SSLBM_OK)
        return tst;
    const hipStream_t s = (hipStream_t)hip_stream;
    const int K = resolved_blocking(m);
    void *src = rho, *dst = scratch;
    for (long long n = 0; n < nsteps;) {
        const int k = nsteps - n < K ? (int)(nsteps - n) : K;
        const sslbm_status st = hip_status(m, sslbm::launch_model(m->dtype, m->lattice, src, dst,
                                                         grid_of(m), m->coef, m->table, k, s));
        if (st != SSLBM_OK)
            return st;
        void *tmp = src;
        src = dst;
        dst = tmp;
        n += k;
    }
    if (src != rho)
        return hip_status(m, hipMemcpyAsync(rho, src, bytes, hipMemcpyDeviceToDevice, s));
    return SSLBM_OK;
}

sslbm_status sslbm_model_set_blocking(sslbm_model *m, int steps_per_pass) {
    if (!m || steps_per_pass < 0 || steps_per_pass > SSLBM_MODEL_MAX_BLOCKING)
        return SSLBM_E_ARG;
    m->blocking = steps_per_pass;
    return SSLBM_OK;
}

sslbm_status sslbm_model_get_blocking(const sslbm_model *m, int *steps_per_pass) {
    if (!m || !steps_per_pass)
        return SSLBM_E_ARG;
    *steps_per_pass = resolved_blocking(m);
    return SSLBM_OK;
}

int sslbm_model_last_hip_error(const sslbm_model *m) { return m ? m->last_hip : 0; }

void sslbm_model_destroy(sslbm_model *m) {
    if (!m)
        return;
    if (m->table)
        (void)hipFree(m->table);
    delete m;
}

}  // extern "C"
