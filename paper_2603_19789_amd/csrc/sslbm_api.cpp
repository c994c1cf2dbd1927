// sslbm_api.cpp -- host side of libsslbm.so: argument validation, derived
// constants, launch planning and the extern "C" entry points of sslbm.h.
// Every check runs before the first HIP call, so rejected calls need no GPU.
#include <hip/hip_runtime_api.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <new>
#include <vector>

#include "fd4_internal.h"
#include "sslbm.h"
#include "sslbm_internal.h"

namespace {

constexpr int MAX_SIDE = 1 << 20;
constexpr long long MAX_CELLS = 1ll << 33;

size_t elem_size(const sslbm_ctx *c) { return c->dtype == SSLBM_F32 ? 4 : 8; }
size_t plane_elems(const sslbm_ctx *c) { return (size_t)c->nx * (size_t)c->ny; }

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + nb && y < x + na;
}

sslbm::GridDesc grid_of(const sslbm_ctx *c) {
    sslbm::GridDesc g;
    g.nx = c->nx;
    g.ny = c->ny;
    g.plane = (long long)c->nx * c->ny;
    g.bc = c->bc;
    return g;
}

sslbm_status hip_status(sslbm_ctx *c, hipError_t e) {
    if (e == hipSuccess)
        return SSLBM_OK;
    c->last_hip = (int)e;
    return SSLBM_E_HIP;
}

// Steps per pass and columns per lane when the caller has not chosen: the
// fastest shapes measured on MI355X for large grids (the pass turns from
// HBM-bound to ALU-bound around there).
int auto_depth(const sslbm_ctx *c) { return c->dtype == SSLBM_F32 ? 6 : 5; }
int auto_cols(const sslbm_ctx *c) { return c->dtype == SSLBM_F32 ? 2 : 1; }

// Rows per wavefront when the caller has not chosen: the shortest chunks for
// which all wavefronts of the pass are resident at once (one round, no tail),
// but at least 2K rows so the halo rows stay a minority. Without a device to
// query, a fixed estimate of three resident wavefronts per SIMD is used.
long long round_rows(const sslbm_ctx *c, int K, int V) {
    const int w = sslbm::strip_width(K, V);
    const long long strips = (c->nx + w - 1) / w;
    long long resident = sslbm::march_resident_waves(c->dtype, K, V, c->coef.diffuse_d);
    if (resident <= 0)
        resident = 3 * 4 * 256;
    long long chunks = resident / strips;
    if (chunks < 1)
        chunks = 1;
    return (c->ny + chunks - 1) / chunks;
}

int auto_rows(const sslbm_ctx *c, int K, int V) {
    long long h = round_rows(c, K, V);
    // One step per pass: a wavefront's work is so short that several rounds
    // of 8-row chunks stream better than one round of taller ones (4096^2:
    // FP32 4.44 -> 4.68 TB/s, FP64 4.54 -> 4.71 TB/s).
    if (K == 1 && h > 8)
        h = 8;
    if (h < 2 * K)
        h = 2 * K;
    if (h > 65536)
        h = 65536;
    return (int)h;
}

// Pass shape actually used: requested fields, automatic ones filled in.
sslbm_launch resolve(const sslbm_ctx *c) {
    sslbm_launch r = c->launch;
    if (r.steps_per_pass == 0)
        r.steps_per_pass = auto_depth(c);
    if (r.cols_per_lane == 0) {
        r.cols_per_lane = auto_cols(c);
        // A grid too small to give one round of resident two-column strips
        // chunks of 2K rows takes one column per lane: twice the strips, and
        // the narrower kernel keeps more wavefronts resident (1024^2 FP32:
        // 259 -> about 305 GLUPS at six steps per pass).
        const int K = r.steps_per_pass;
        if (r.cols_per_lane == 2 && K <= sslbm::march_max_depth(c->dtype, 1) &&
            round_rows(c, K, 2) < 2 * K)
            r.cols_per_lane = 1;
    }
    if (r.rows_per_wave == 0)
        r.rows_per_wave = auto_rows(c, r.steps_per_pass, r.cols_per_lane);
    return r;
}

// Shape of one pass of k steps (the last pass of a run may be shorter). Two
// columns per lane read and write aligned element pairs: that needs an even
// row length and pair-aligned buffers, else the pass takes one column per lane.
sslbm::MarchShape shape_for(const sslbm_ctx *c, int k, const void *in, const void *out) {
    const sslbm_launch r = resolve(c);
    sslbm::MarchShape s;
    s.cols_per_lane = r.cols_per_lane;
    const uintptr_t pair = 2 * elem_size(c);
    if (s.cols_per_lane == 2 &&
        (c->nx % 2 != 0 || (uintptr_t)in % pair != 0 || (uintptr_t)out % pair != 0 ||
         k > sslbm::march_max_depth(c->dtype, 2)))
        s.cols_per_lane = 1;
    s.rows_per_wave =
        c->launch.rows_per_wave > 0 ? c->launch.rows_per_wave : auto_rows(c, k, s.cols_per_lane);
    return s;
}

}  // namespace

namespace sslbm {

// One pass of k steps, in -> out, with the context's pass shape.
sslbm_status run_pass(sslbm_ctx *c, const void *in, void *out, int k, hipStream_t s) {
    return hip_status(c, launch_march(c->dtype, in, out, grid_of(c), c->coef, k,
                                      shape_for(c, k, in, out), s));
}

sslbm_status run_pass_mid2(sslbm_ctx *c, const void *in, void *mid, void *out, hipStream_t s) {
    // both outputs pair-aligned for two columns per lane
    MarchShape shape = shape_for(c, 4, in, out);
    if ((uintptr_t)mid % (2 * elem_size(c)) != 0)
        shape.cols_per_lane = 1;
    return hip_status(c, launch_march_mid(c->dtype, in, mid, out, grid_of(c), c->coef, 4, 2,
                                          shape, s));
}

static bool finite_nonneg(double v) { return std::isfinite(v) && v >= 0.0; }

// Validation of sslbm_params and the derived per-step constants.
sslbm_status derive_coef(const sslbm_params *p, StepCoef *k) {
    if (!p)
        return SSLBM_E_ARG;
    if (!finite_nonneg(p->beta) || !finite_nonneg(p->alpha) || !finite_nonneg(p->gamma) ||
        !finite_nonneg(p->phi) || p->phi > 1.0)
        return SSLBM_E_ARG;
    if (!(std::isfinite(p->dx) && p->dx > 0.0) || !(std::isfinite(p->dt) && p->dt > 0.0))
        return SSLBM_E_ARG;
    for (int c = 0; c < 5; ++c)
        if (!finite_nonneg(p->d[c]))
            return SSLBM_E_ARG;

    StepCoef out{};
    const double scale = p->dt / (p->dx * p->dx);
    for (int c = 0; c < 5; ++c) {
        out.dl[c] = p->d[c] * scale;
        // |G(k)| <= 1 for every k iff 0 <= d_lu <= 1/4 (G = 1 - 2 d_lu (2 - cos kx - cos ky))
        if (!(out.dl[c] <= 0.25))
            return SSLBM_E_UNSTABLE;
    }
    // Linearisation at the disease-free equilibrium, Eq. (eigenvalues): the
    // decaying E-I eigenvalue lambda_2 plus the most negative diffusion factor
    // must stay >= -1, i.e. dt |lambda_2| + 8 max(d_lu^E, d_lu^I) <= 2.
    const double a = p->alpha, g = p->gamma, b = p->beta;
    const double lambda2 = 0.5 * (-(a + g) - std::sqrt((a - g) * (a - g) + 4.0 * a * b));
    const double dmax = out.dl[1] > out.dl[2] ? out.dl[1] : out.dl[2];
    if (p->dt * std::fabs(lambda2) + 8.0 * dmax > 2.0)
        return SSLBM_E_UNSTABLE;

    out.bdt = p->beta * p->dt;
    out.kE = p->alpha * p->dt;
    out.kI = p->gamma * p->dt;
    out.kR = (1.0 - p->phi) * p->gamma * p->dt;
    out.kD = p->phi * p->gamma * p->dt;
    for (int c = 0; c < 4; ++c)
        out.omega[c] = 1.0 / (0.5 + 3.0 * out.dl[c]);
    out.diffuse_d = p->d[4] != 0.0;
    *k = out;
    return SSLBM_OK;
}

PassPlan plan_passes(long long nsteps, int K) {
    PassPlan p;
    if (nsteps <= 0 || K < 1)
        return p;
    p.count = (nsteps + K - 1) / K;
    // one more pass only while every pass keeps at least one step (K = 1 and
    // an odd nsteps stay odd: the run then ends with a copy)
    if (p.count % 2 == 1 && p.count < nsteps)
        ++p.count;
    p.base = (int)(nsteps / p.count);
    p.longer = nsteps - (long long)p.base * p.count;
    return p;
}

}  // namespace sslbm

extern "C" {

sslbm_status sslbm_init(sslbm_ctx **out, int nx, int ny, int dtype, int bc,
                        const sslbm_params *p) {
    if (!out || !p)
        return SSLBM_E_ARG;
    *out = nullptr;
    if (nx < 1 || ny < 1 || nx > MAX_SIDE || ny > MAX_SIDE || (long long)nx * ny > MAX_CELLS)
        return SSLBM_E_ARG;
    if (dtype != SSLBM_F32 && dtype != SSLBM_F64)
        return SSLBM_E_ARG;
    if (bc != SSLBM_PERIODIC && bc != SSLBM_NOFLUX)
        return SSLBM_E_ARG;
    sslbm::StepCoef k;
    const sslbm_status st = sslbm::derive_coef(p, &k);
    if (st != SSLBM_OK)
        return st;
    sslbm_ctx *c = new (std::nothrow) sslbm_ctx();
    if (!c)
        return SSLBM_E_NOMEM;
    c->nx = nx;
    c->ny = ny;
    c->dtype = dtype;
    c->bc = bc;
    c->p = *p;
    c->coef = k;
    *out = c;
    return SSLBM_OK;
}

sslbm_status sslbm_params_from_rates(double beta, double sigma, double gamma, double mu,
                                     const double d[5], double dx, double dt, sslbm_params *out) {
    const double rates[4] = {beta, sigma, gamma, mu};
    if (!out || !d)
        return SSLBM_E_ARG;
    for (double r : rates)
        if (!std::isfinite(r) || r < 0.0)
            return SSLBM_E_ARG;
    const double removal = gamma + mu;
    if (!(removal > 0.0))
        return SSLBM_E_ARG;
    sslbm_params p;
    p.beta = beta;
    p.alpha = sigma;
    p.gamma = removal;
    p.phi = mu / removal;
    for (int c = 0; c < 5; ++c)
        p.d[c] = d[c];
    p.dx = dx;
    p.dt = dt;
    *out = p;
    return SSLBM_OK;
}

sslbm_status sslbm_rate_gradients(const double grad_params[4], double gamma, double mu,
                                  double grad_rates[4]) {
    if (!grad_params || !grad_rates || !std::isfinite(gamma) || !std::isfinite(mu) ||
        gamma < 0.0 || mu < 0.0 || !(gamma + mu > 0.0))
        return SSLBM_E_ARG;
    const double removal = gamma + mu, r2 = removal * removal;
    const double g_beta = grad_params[0], g_alpha = grad_params[1];
    const double g_removal = grad_params[2], g_phi = grad_params[3];
    grad_rates[0] = g_beta;
    grad_rates[1] = g_alpha;
    grad_rates[2] = g_removal - g_phi * (mu / r2);
    grad_rates[3] = g_removal + g_phi * (gamma / r2);
    return SSLBM_OK;
}

sslbm_status sslbm_set_params(sslbm_ctx *c, const sslbm_params *p) {
    if (!c)
        return SSLBM_E_ARG;
    sslbm::StepCoef k;
    const sslbm_status st = sslbm::derive_coef(p, &k);
    if (st != SSLBM_OK)
        return st;
    c->p = *p;
    c->coef = k;
    return SSLBM_OK;
}

sslbm_status sslbm_set_launch(sslbm_ctx *c, const sslbm_launch *shape) {
    if (!c || !shape)
        return SSLBM_E_ARG;
    const sslbm_launch &r = *shape;
    if (r.steps_per_pass < 0 || r.steps_per_pass > SSLBM_MAX_BLOCKING || r.rows_per_wave < 0 ||
        r.rows_per_wave > 65536 || r.cols_per_lane < 0 || r.cols_per_lane > 2)
        return SSLBM_E_ARG;
    sslbm_ctx probe = *c;
    probe.partials = nullptr;
    probe.launch = r;
    const sslbm_launch full = resolve(&probe);
    if (full.steps_per_pass > sslbm::march_max_depth(c->dtype, full.cols_per_lane))
        return SSLBM_E_UNSUPPORTED;
    c->launch = r;
    return SSLBM_OK;
}

sslbm_status sslbm_get_launch(const sslbm_ctx *c, sslbm_launch *shape) {
    if (!c || !shape)
        return SSLBM_E_ARG;
    *shape = resolve(c);
    return SSLBM_OK;
}

sslbm_status sslbm_tune(sslbm_ctx *c, const void *rho, void *scratch, void *hip_stream,
                        sslbm_launch *best) {
    if (!c || !rho || !scratch)
        return SSLBM_E_ARG;
    const size_t bytes = 5 * plane_elems(c) * elem_size(c);
    if (overlap(rho, bytes, scratch, bytes))
        return SSLBM_E_ALIAS;
    const hipStream_t s = (hipStream_t)hip_stream;
    sslbm_status st = hip_status(c, hipStreamSynchronize(s));
    if (st != SSLBM_OK)
        return st;
    hipEvent_t t0, t1;
    st = hip_status(c, hipEventCreate(&t0));
    if (st != SSLBM_OK)
        return st;
    st = hip_status(c, hipEventCreate(&t1));
    if (st != SSLBM_OK) {
        (void)hipEventDestroy(t0);
        return st;
    }
    const uintptr_t pair = 2 * elem_size(c);
    const bool pairs_ok =
        c->nx % 2 == 0 && (uintptr_t)rho % pair == 0 && (uintptr_t)scratch % pair == 0;
    const sslbm_launch saved = c->launch;
    sslbm_launch best_shape = resolve(c);
    double best_ns = 1e300;
    for (int V = 1; V <= (pairs_ok ? 2 : 1) && st == SSLBM_OK; ++V) {
        for (int K = 1; K <= sslbm::march_max_depth(c->dtype, V) && st == SSLBM_OK; ++K) {
            const int cands[] = {0, 8, 16, 32, 64, 128};
            for (int H : cands) {
                if (H != 0 && H < 2 * K)
                    continue;
                c->launch = sslbm_launch{K, H, V};
                // one untimed pass, then three timed ones, all rho -> scratch
                for (int rep = 0; rep < 4 && st == SSLBM_OK; ++rep) {
                    if (rep == 1)
                        st = hip_status(c, hipEventRecord(t0, s));
                    if (st == SSLBM_OK)
                        st = sslbm::run_pass(c, rho, scratch, K, s);
                }
                if (st == SSLBM_OK)
                    st = hip_status(c, hipEventRecord(t1, s));
                if (st == SSLBM_OK)
                    st = hip_status(c, hipEventSynchronize(t1));
                float ms = 0.f;
                if (st == SSLBM_OK)
                    st = hip_status(c, hipEventElapsedTime(&ms, t0, t1));
                if (st != SSLBM_OK)
                    break;
                const double ns_per_step = 1e6 * ms / (3.0 * K);
                if (ns_per_step < best_ns) {
                    best_ns = ns_per_step;
                    best_shape = resolve(c);
                }
            }
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (st != SSLBM_OK) {
        c->launch = saved;
        return st;
    }
    c->launch = best_shape;
    if (best)
        *best = best_shape;
    return SSLBM_OK;
}

sslbm_status sslbm_plan_run(const sslbm_ctx *c, long long nsteps, long long *passes, int *longest,
                            int *shortest) {
    if (!c || nsteps < 0 || !passes)
        return SSLBM_E_ARG;
    const sslbm::PassPlan p = sslbm::plan_passes(nsteps, resolve(c).steps_per_pass);
    *passes = p.count;
    if (longest)
        *longest = p.count == 0 ? 0 : p.steps(0);
    if (shortest)
        *shortest = p.count == 0 ? 0 : p.steps(p.count - 1);
    return SSLBM_OK;
}

sslbm_status sslbm_set_blocking(sslbm_ctx *c, int steps_per_pass) {
    if (!c)
        return SSLBM_E_ARG;
    sslbm_launch r = c->launch;
    r.steps_per_pass = steps_per_pass;
    return sslbm_set_launch(c, &r);
}

int sslbm_get_blocking(const sslbm_ctx *c) {
    if (!c)
        return SSLBM_E_ARG;
    return resolve(c).steps_per_pass;
}

sslbm_status sslbm_step(sslbm_ctx *c, const void *rho_in, void *rho_out, void *hip_stream) {
    if (!c || !rho_in || !rho_out)
        return SSLBM_E_ARG;
    const size_t bytes = 5 * plane_elems(c) * elem_size(c);
    if (overlap(rho_in, bytes, rho_out, bytes))
        return SSLBM_E_ALIAS;
    return hip_status(c, sslbm::launch_march(c->dtype, rho_in, rho_out, grid_of(c), c->coef, 1,
                                             shape_for(c, 1, rho_in, rho_out),
                                             (hipStream_t)hip_stream));
}

sslbm_status sslbm_run(sslbm_ctx *c, void *rho, void *scratch, long long nsteps, void *hip_stream) {
    if (!c || !rho || !scratch || nsteps < 0)
        return SSLBM_E_ARG;
    const size_t bytes = 5 * plane_elems(c) * elem_size(c);
    if (overlap(rho, bytes, scratch, bytes))
        return SSLBM_E_ALIAS;
    if (nsteps == 0)
        return SSLBM_OK;
    const int K = resolve(c).steps_per_pass;
    const hipStream_t s = (hipStream_t)hip_stream;
    const sslbm::GridDesc g = grid_of(c);
    void *src = rho, *dst = scratch;
    const sslbm::PassPlan plan = sslbm::plan_passes(nsteps, K);
    for (long long i = 0; i < plan.count; ++i) {
        const int k = plan.steps(i);
        const sslbm_status st =
            hip_status(c, sslbm::launch_march(c->dtype, src, dst, g, c->coef, k,
                                              shape_for(c, k, src, dst), s));
        if (st != SSLBM_OK)
            return st;
        void *t = src;
        src = dst;
        dst = t;
    }
    if (src != rho)
        return hip_status(c, hipMemcpyAsync(rho, src, bytes, hipMemcpyDeviceToDevice, s));
    return SSLBM_OK;
}

static sslbm_status bgk_check(const sslbm_ctx *c) {
    if (!c)
        return SSLBM_E_ARG;
    if (c->p.d[4] != 0.0)
        return SSLBM_E_UNSUPPORTED;
    return SSLBM_OK;
}

sslbm_status bgk_init(sslbm_ctx *c, const void *rho, void *f, void *rhoD, void *hip_stream) {
    sslbm_status st = bgk_check(c);
    if (st != SSLBM_OK)
        return st;
    if (!rho || !f || !rhoD)
        return SSLBM_E_ARG;
    const size_t pb = plane_elems(c) * elem_size(c);
    if (overlap(rho, 5 * pb, f, 20 * pb) || overlap(rho, 5 * pb, rhoD, pb) ||
        overlap(f, 20 * pb, rhoD, pb))
        return SSLBM_E_ALIAS;
    return hip_status(c, sslbm::launch_bgk_init(c->dtype, rho, f, rhoD, grid_of(c),
                                                (hipStream_t)hip_stream));
}

sslbm_status bgk_step(sslbm_ctx *c, const void *f_in, const void *rhoD_in, void *f_out,
                      void *rhoD_out, void *hip_stream) {
    sslbm_status st = bgk_check(c);
    if (st != SSLBM_OK)
        return st;
    if (!f_in || !rhoD_in || !f_out || !rhoD_out)
        return SSLBM_E_ARG;
    const size_t pb = plane_elems(c) * elem_size(c);
    const void *ins[2] = {f_in, rhoD_in};
    const void *outs[2] = {f_out, rhoD_out};
    const size_t sz[2] = {20 * pb, pb};
    for (int i = 0; i < 2; ++i)
        for (int j = 0; j < 2; ++j)
            if (overlap(ins[i], sz[i], outs[j], sz[j]))
                return SSLBM_E_ALIAS;
    if (overlap(f_out, 20 * pb, rhoD_out, pb))
        return SSLBM_E_ALIAS;
    return hip_status(c, sslbm::launch_bgk_step(c->dtype, f_in, rhoD_in, f_out, rhoD_out,
                                                grid_of(c), c->coef, (hipStream_t)hip_stream));
}

sslbm_status bgk_run(sslbm_ctx *c, void *f, void *rhoD, void *f_scratch, void *rhoD_scratch,
                     long long nsteps, void *hip_stream) {
    sslbm_status st = bgk_check(c);
    if (st != SSLBM_OK)
        return st;
    if (!f || !rhoD || !f_scratch || !rhoD_scratch || nsteps < 0)
        return SSLBM_E_ARG;
    const size_t pb = plane_elems(c) * elem_size(c);
    void *bufs[4] = {f, rhoD, f_scratch, rhoD_scratch};
    const size_t sz[4] = {20 * pb, pb, 20 * pb, pb};
    for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j)
            if (overlap(bufs[i], sz[i], bufs[j], sz[j]))
                return SSLBM_E_ALIAS;
    const hipStream_t s = (hipStream_t)hip_stream;
    const sslbm::GridDesc g = grid_of(c);
    void *fa = f, *da = rhoD, *fb = f_scratch, *db = rhoD_scratch;
    for (long long n = 0; n < nsteps; ++n) {
        st = hip_status(c, sslbm::launch_bgk_step(c->dtype, fa, da, fb, db, g, c->coef, s));
        if (st != SSLBM_OK)
            return st;
        void *t = fa;
        fa = fb;
        fb = t;
        t = da;
        da = db;
        db = t;
    }
    if (fa != f) {
        st = hip_status(c, hipMemcpyAsync(f, fa, 20 * pb, hipMemcpyDeviceToDevice, s));
        if (st != SSLBM_OK)
            return st;
        return hip_status(c, hipMemcpyAsync(rhoD, da, pb, hipMemcpyDeviceToDevice, s));
    }
    return SSLBM_OK;
}

sslbm_status bgk_density(sslbm_ctx *c, const void *f, const void *rhoD, void *rho,
                         void *hip_stream) {
    sslbm_status st = bgk_check(c);
    if (st != SSLBM_OK)
        return st;
    if (!f || !rhoD || !rho)
        return SSLBM_E_ARG;
    const size_t pb = plane_elems(c) * elem_size(c);
    if (overlap(rho, 5 * pb, f, 20 * pb) || overlap(rho, 5 * pb, rhoD, pb))
        return SSLBM_E_ALIAS;
    return hip_status(c, sslbm::launch_bgk_density(c->dtype, f, rhoD, rho, grid_of(c),
                                                   (hipStream_t)hip_stream));
}

size_t sslbm_fd4_workspace_bytes(const sslbm_ctx *c) {
    return c ? 3 * 5 * plane_elems(c) * elem_size(c) : 0;
}

sslbm_status sslbm_fd4_run(sslbm_ctx *c, void *rho, void *work, size_t work_bytes, long long nsteps,
                           void *hip_stream) {
    if (!c || !rho || !work || nsteps < 0)
        return SSLBM_E_ARG;
    const size_t bytes = 5 * plane_elems(c) * elem_size(c);
    if (work_bytes < 3 * bytes || (uintptr_t)rho % elem_size(c) || (uintptr_t)work % elem_size(c))
        return SSLBM_E_ARG;
    if (overlap(rho, bytes, work, 3 * bytes))
        return SSLBM_E_ALIAS;
    if (nsteps == 0)
        return SSLBM_OK;
    return hip_status(c, sslbm::launch_fd4(c->dtype, rho, work, grid_of(c), c->coef, nsteps,
                                           (hipStream_t)hip_stream));
}

sslbm_status sslbm_total(sslbm_ctx *c, const void *rho, double out_totals[5], void *hip_stream) {
    if (!c || !rho || !out_totals)
        return SSLBM_E_ARG;
    const sslbm::GridDesc g = grid_of(c);
    const int blocks = sslbm::total_blocks(g);
    int dev = 0;
    sslbm_status st = hip_status(c, hipGetDevice(&dev));
    if (st != SSLBM_OK)
        return st;
    if (!c->partials || c->partial_blocks < blocks || c->partial_device != dev) {
        if (c->partials)
            (void)hipFree(c->partials);
        c->partials = nullptr;
        st = hip_status(c, hipMalloc((void **)&c->partials, sizeof(double) * (5 * blocks + 5)));
        if (st != SSLBM_OK)
            return st;
        c->partial_blocks = blocks;
        c->partial_device = dev;
    }
    const hipStream_t s = (hipStream_t)hip_stream;
    double *out_dev = c->partials + 5 * c->partial_blocks;
    st = hip_status(c, sslbm::launch_total(c->dtype, rho, g, c->partials, blocks, out_dev, s));
    if (st != SSLBM_OK)
        return st;
    st = hip_status(c, hipMemcpyAsync(out_totals, out_dev, 5 * sizeof(double),
                                      hipMemcpyDeviceToHost, s));
    if (st != SSLBM_OK)
        return st;
    return hip_status(c, hipStreamSynchronize(s));
}

void sslbm_destroy(sslbm_ctx *c) {
    if (!c)
        return;
    if (c->partials)
        (void)hipFree(c->partials);
    if (c->adj_partials)
        (void)hipFree(c->adj_partials);
    delete c;
}

const char *sslbm_strerror(int status) {
    switch (status) {
    case SSLBM_OK: return "success";
    case SSLBM_E_ARG: return "invalid argument";
    case SSLBM_E_UNSTABLE: return "parameters outside the linear stability region";
    case SSLBM_E_UNSUPPORTED: return "unsupported request";
    case SSLBM_E_ALIAS: return "input and output buffers overlap";
    case SSLBM_E_HIP: return "HIP runtime error";
    case SSLBM_E_NOMEM: return "out of host memory";
    case SSLBM_E_LIMIT: return "request exceeds a fixed-size buffer of the library";
    default: return "unknown status";
    }
}

int sslbm_last_hip_error(const sslbm_ctx *c) { return c ? c->last_hip : 0; }

}  // extern "C"
