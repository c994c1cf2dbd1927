// adjoint_api.cpp -- host side of the reverse-mode entry points of sslbm.h:
// one adjoint step, a forward run that stores checkpoints, and the
// checkpointed reverse sweep over a whole run.
//
// Reverse sweep. The forward run stores the state every `every` steps. The
// sweep takes the segments from the last to the first: it recomputes the
// states of a segment from its checkpoint with single forward steps (each
// state is needed by one adjoint step), then runs the segment's adjoint
// steps backwards. Work: about two forward steps and one adjoint step per
// step of the run; memory: the checkpoints plus one segment of states.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <utility>

#include "adjoint_internal.h"
#include "sslbm.h"
#include "sslbm_internal.h"

namespace {

size_t elem_size(const sslbm_ctx *c) { return c->dtype == SSLBM_F32 ? 4 : 8; }
size_t state_bytes(const sslbm_ctx *c) {
    return 5 * (size_t)c->nx * (size_t)c->ny * elem_size(c);
}
size_t align256(size_t n) { return (n + 255) & ~(size_t)255; }

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return na && nb && x < y + nb && y < x + na;
}

sslbm_status hip_status(sslbm_ctx *c, hipError_t e) {
    if (e == hipSuccess)
        return SSLBM_OK;
    c->last_hip = (int)e;
    return SSLBM_E_HIP;
}

sslbm::GridDesc grid_of(const sslbm_ctx *c) {
    sslbm::GridDesc g;
    g.nx = c->nx;
    g.ny = c->ny;
    g.plane = (long long)c->nx * c->ny;
    g.bc = c->bc;
    return g;
}

sslbm::AdjFactors factors_of(const sslbm_ctx *c) {
    sslbm::AdjFactors f;
    f.dt = c->p.dt;
    f.gamma_dt = c->p.gamma * c->p.dt;
    f.phi = c->p.phi;
    f.dt_dx2 = c->p.dt / (c->p.dx * c->p.dx);
    return f;
}

size_t partials_bytes(const sslbm::AdjShape &s) {
    return (size_t)s.slots() * sslbm::ADJ_SLOT * sizeof(double);
}

sslbm_status step_args(const sslbm_ctx *c, const void *rho, const void *lam_next,
                       const void *lam_out, const double *grad) {
    if (!c || !rho || !lam_next || !lam_out || !grad)
        return SSLBM_E_ARG;
    const size_t bytes = state_bytes(c);
    if (overlap(lam_out, bytes, lam_next, bytes) || overlap(lam_out, bytes, rho, bytes) ||
        overlap(grad, 9 * sizeof(double), lam_out, bytes))
        return SSLBM_E_ALIAS;
    return SSLBM_OK;
}

// The reverse step and the sum of its wavefront slots into grad.
sslbm_status step_into(sslbm_ctx *c, const void *rho, const void *lam_next, void *lam_out,
                       double *grad, const sslbm::AdjShape &shape, double *partials,
                       hipStream_t s) {
    const sslbm_status st = hip_status(c, sslbm::launch_adjoint(c->dtype, rho, lam_next, lam_out,
                                                       grid_of(c), c->coef, shape, partials,
                                                       true, s));
    if (st != SSLBM_OK)
        return st;
    return hip_status(c, sslbm::launch_adjoint_finish(partials, (int)shape.slots(),
                                                      factors_of(c), grad, s));
}

}  // namespace

// ---- the allocation-free adjoint step -------------------------------------
// The wavefront slots of sslbm_adjoint_step_noalloc: a file-scope device
// array, one copy per GPU. Host code never passes `scratch` itself to a
// kernel (on the host it only names the symbol): its device address is
// looked up once per device with that device current, and kept.
static __device__ __align__(256) double scratch[SSLBM_ADJ_NOALLOC_SLOTS * sslbm::ADJ_SLOT];

namespace {

constexpr long long NOALLOC_SLOTS = SSLBM_ADJ_NOALLOC_SLOTS;
constexpr int MAX_DEVICES = 64;
std::mutex scratch_lock;
double *scratch_of_device[MAX_DEVICES] = {};

sslbm_status scratch_address(sslbm_ctx *c, double **out) {
    int dev = 0;
    sslbm_status st = hip_status(c, hipGetDevice(&dev));
    if (st != SSLBM_OK)
        return st;
    if (dev < 0 || dev >= MAX_DEVICES)
        return SSLBM_E_UNSUPPORTED;
    std::lock_guard<std::mutex> guard(scratch_lock);
    if (!scratch_of_device[dev]) {
        void *p = nullptr;
        st = hip_status(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (st != SSLBM_OK)
            return st;
        if (!p)
            return hip_status(c, hipErrorInvalidSymbol);
        scratch_of_device[dev] = static_cast<double *>(p);
    }
    *out = scratch_of_device[dev];
    return SSLBM_OK;
}

}  // namespace

extern "C" {

sslbm_status sslbm_adjoint_step_noalloc(sslbm_ctx *c, const void *rho, const void *lam_next,
                                        void *lam_out, double *grad, void *hip_stream) {
    sslbm_status st = step_args(c, rho, lam_next, lam_out, grad);
    if (st != SSLBM_OK)
        return st;
    const sslbm::AdjShape shape = sslbm::adjoint_shape(c->nx, c->ny);
    if (shape.slots() > NOALLOC_SLOTS)
        return SSLBM_E_LIMIT;
    double *partials = nullptr;
    st = scratch_address(c, &partials);
    if (st != SSLBM_OK)
        return st;
    return step_into(c, rho, lam_next, lam_out, grad, shape, partials,
                     (hipStream_t)hip_stream);
}

sslbm_status sslbm_adjoint_step(sslbm_ctx *c, const void *rho, const void *lam_next, void *lam_out,
                                double *grad, void *hip_stream) {
    sslbm_status st = step_args(c, rho, lam_next, lam_out, grad);
    if (st != SSLBM_OK)
        return st;
    const sslbm::AdjShape shape = sslbm::adjoint_shape(c->nx, c->ny);
    int dev = 0;
    st = hip_status(c, hipGetDevice(&dev));
    if (st != SSLBM_OK)
        return st;
    if (!c->adj_partials || c->adj_slots < shape.slots() || c->adj_device != dev) {
        if (c->adj_partials)
            (void)hipFree(c->adj_partials);
        c->adj_partials = nullptr;
        st = hip_status(c, hipMalloc((void **)&c->adj_partials, partials_bytes(shape)));
        if (st != SSLBM_OK)
            return st;
        c->adj_slots = shape.slots();
        c->adj_device = dev;
    }
    return step_into(c, rho, lam_next, lam_out, grad, shape, c->adj_partials,
                     (hipStream_t)hip_stream);
}

long long sslbm_checkpoint_count(long long nsteps, int every) {
    if (nsteps < 0 || every < 1)
        return -1;
    return (nsteps + every - 1) / every;
}

sslbm_status sslbm_run_checkpointed(sslbm_ctx *c, void *rho, void *scratch, long long nsteps,
                                    int every, void *checkpoints, void *hip_stream) {
    if (!c || !rho || !scratch || !checkpoints || nsteps < 0 || every < 1)
        return SSLBM_E_ARG;
    const size_t bytes = state_bytes(c);
    const long long count = sslbm_checkpoint_count(nsteps, every);
    const size_t cp_bytes = (size_t)count * bytes;
    if (overlap(checkpoints, cp_bytes, rho, bytes) || overlap(checkpoints, cp_bytes, scratch, bytes) ||
        overlap(rho, bytes, scratch, bytes))
        return SSLBM_E_ALIAS;
    const hipStream_t s = (hipStream_t)hip_stream;
    if (count == 0)
        return SSLBM_OK;
    if (every <= sslbm::march_max_depth(c->dtype, 1)) {
        // One pass per segment, written straight into the next checkpoint
        // (the last one into rho): one copy in all, no ping-pong through
        // scratch; checkpoints every 2 steps take two segments per pass. The
        // pass kernel gives the same bits at every depth.
        char *cp = static_cast<char *>(checkpoints);
        sslbm_status st = hip_status(c, hipMemcpyAsync(cp, rho, bytes, hipMemcpyDeviceToDevice, s));
        if (st != SSLBM_OK)
            return st;
        auto slot = [&](long long k) -> void * {
            return k < count ? static_cast<void *>(cp + (size_t)k * bytes) : rho;
        };
        for (long long k = 0; k < count;) {
            const long long n = nsteps - k * every < every ? nsteps - k * every : every;
            if (every == 2 && n == 2 && k + 1 < count && nsteps - (k + 1) * every >= 2) {
                // two segments in one pass of 4 steps, the state after 2
                // steps written on the way
                st = sslbm::run_pass_mid2(c, slot(k), slot(k + 1), slot(k + 2), s);
                k += 2;
            } else {
                st = sslbm::run_pass(c, slot(k), slot(k + 1), (int)n, s);
                k += 1;
            }
            if (st != SSLBM_OK)
                return st;
        }
        return SSLBM_OK;
    }
    for (long long k = 0; k < count; ++k) {
        char *slot = static_cast<char *>(checkpoints) + (size_t)k * bytes;
        sslbm_status st =
            hip_status(c, hipMemcpyAsync(slot, rho, bytes, hipMemcpyDeviceToDevice, s));
        if (st != SSLBM_OK)
            return st;
        const long long n = nsteps - k * every < every ? nsteps - k * every : every;
        st = sslbm_run(c, rho, scratch, n, hip_stream);
        if (st != SSLBM_OK)
            return st;
    }
    return SSLBM_OK;
}

size_t sslbm_adjoint_workspace_bytes(const sslbm_ctx *c, int every) {
    if (!c || every < 1)
        return 0;
    // the states at even offsets 2, 4, .. of a segment, one adjoint field,
    // the gradient slots of the single-step and the two-step kernels
    const sslbm::AdjShape s1 = sslbm::adjoint_shape(c->nx, c->ny);
    const sslbm::AdjShape s2 = sslbm::adjoint2_shape(c->nx, c->ny);
    const size_t states = (size_t)((every - 1) / 2) + 1;
    return align256(states * state_bytes(c)) + align256(partials_bytes(s1) + partials_bytes(s2));
}

// Reverse sweep of one segment of `len` steps from its checkpoint: the
// states at even offsets are recomputed with two-step passes; the adjoint
// then runs two steps per pass (the odd state recomputed in registers),
// with one single step first when len is odd.
sslbm_status sslbm_adjoint_run(sslbm_ctx *c, const void *checkpoints, long long nsteps, int every,
                               void *lam, double *grad, void *workspace, void *hip_stream) {
    if (!c || !checkpoints || !lam || !grad || !workspace || nsteps < 0 || every < 1)
        return SSLBM_E_ARG;
    const size_t bytes = state_bytes(c);
    const long long count = sslbm_checkpoint_count(nsteps, every);
    const size_t cp_bytes = (size_t)count * bytes;
    const size_t ws_bytes = sslbm_adjoint_workspace_bytes(c, every);
    if (overlap(lam, bytes, checkpoints, cp_bytes) || overlap(lam, bytes, workspace, ws_bytes) ||
        overlap(checkpoints, cp_bytes, workspace, ws_bytes) ||
        overlap(grad, 9 * sizeof(double), lam, bytes) ||
        overlap(grad, 9 * sizeof(double), workspace, ws_bytes))
        return SSLBM_E_ALIAS;
    if (nsteps == 0)
        return SSLBM_OK;

    char *ws = static_cast<char *>(workspace);
    const size_t nstates = (size_t)((every - 1) / 2);  // offsets 2, 4, ..
    char *lam_alt = ws + nstates * bytes;
    const sslbm::AdjShape s1 = sslbm::adjoint_shape(c->nx, c->ny);
    const sslbm::AdjShape s2 = sslbm::adjoint2_shape(c->nx, c->ny);
    double *part1 = reinterpret_cast<double *>(ws + align256((nstates + 1) * bytes));
    double *part2 = part1 + s1.slots() * sslbm::ADJ_SLOT;
    const sslbm::GridDesc g = grid_of(c);
    const hipStream_t s = (hipStream_t)hip_stream;
    sslbm_status st = hip_status(
        c, sslbm::launch_zero(part1, (s1.slots() + s2.slots()) * sslbm::ADJ_SLOT, s));
    if (st != SSLBM_OK)
        return st;

    void *cur = lam, *nxt = lam_alt;
    for (long long k = count - 1; k >= 0; --k) {
        const char *cp = static_cast<const char *>(checkpoints) + (size_t)k * bytes;
        const long long len = nsteps - k * every < every ? nsteps - k * every : every;
        // state at even offset i: the checkpoint, or workspace slot i / 2 - 1
        auto state = [&](long long i) -> const void * {
            return i == 0 ? (const void *)cp : (const void *)(ws + (size_t)(i / 2 - 1) * bytes);
        };
        // every second state of the segment from its checkpoint: four-step
        // passes that also write the state after two steps (the bits of two
        // two-step passes), one two-step pass for an odd count
        long long i = 2;
        for (; i + 2 < len; i += 4) {
            st = sslbm::run_pass_mid2(c, state(i - 2), ws + (size_t)(i / 2 - 1) * bytes,
                                      ws + (size_t)(i / 2) * bytes, s);
            if (st != SSLBM_OK)
                return st;
        }
        for (; i < len; i += 2) {
            st = sslbm::run_pass(c, state(i - 2), ws + (size_t)(i / 2 - 1) * bytes, 2, s);
            if (st != SSLBM_OK)
                return st;
        }
        long long top = len;
        if (len % 2) {
            st = hip_status(c, sslbm::launch_adjoint(c->dtype, state(len - 1), cur, nxt, g, c->coef,
                                                     s1, part1, false, s));
            if (st != SSLBM_OK)
                return st;
            std::swap(cur, nxt);
            top = len - 1;
        }
        for (long long i = top - 2; i >= 0; i -= 2) {
            st = hip_status(c, sslbm::launch_adjoint2(c->dtype, state(i), cur, nxt, g, c->coef,
                                                      s2, part2, s));
            if (st != SSLBM_OK)
                return st;
            std::swap(cur, nxt);
        }
    }
    if (cur != lam) {
        st = hip_status(c, hipMemcpyAsync(lam, cur, bytes, hipMemcpyDeviceToDevice, s));
        if (st != SSLBM_OK)
            return st;
    }
    return hip_status(c, sslbm::launch_adjoint_finish(part1, (int)(s1.slots() + s2.slots()),
                                                      factors_of(c), grad, s));
}

}  // extern "C"
