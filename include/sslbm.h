/*
 * sslbm.h -- C ABI of libsslbm.so: the single-step simplified lattice
 * Boltzmann method (SSLBM) for the spatial SEIRD epidemic model, and the BGK
 * lattice Boltzmann step it is compared with, on AMD MI355X (gfx950).
 *
 * Paper: A. De Rosis, "A distribution-free lattice Boltzmann method for
 * compartmental reaction-diffusion systems with application to epidemic
 * modelling", arXiv 2603.19789.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every entry point returns an sslbm_status (an int-sized enum; SSLBM_OK
 *   is 0), except the few that return a count, a depth or a HIP error
 *   code, which say so and return int.
 * - Arguments are validated on the host before any HIP call: a rejected call
 *   enqueues nothing, touches no device memory and works without a GPU.
 * - Device buffers are plain device pointers allocated and owned by the
 *   caller (hipMalloc, or torch tensors on the GPU). The library never frees
 *   them and never keeps them after the call returns.
 * - Work is enqueued on `hip_stream`, a hipStream_t passed as void* (NULL is
 *   the default stream). Only sslbm_total waits for the stream.
 * - A context holds host-side constants only (lattice diffusivities, rates
 *   times dt, launch shape). It is not thread-safe; distinct contexts are
 *   independent.
 *
 * Data layouts (x fastest, row-major, no padding; element type from dtype)
 * ------------------------------------------------------------------------
 * - rho  : [5][ny][nx], compartments in the order S, E, I, R, D.
 * - f    : [4][5][ny][nx], BGK populations of the mobile compartments
 *          C = S, E, I, R (outer index), directions i = 0..4 of the D2Q5
 *          lattice with c_i = (0,0), (1,0), (0,1), (-1,0), (0,-1) (Sec. II.B).
 * - rhoD : [ny][nx], the deceased density carried next to the BGK populations
 *          (Sec. II.B storage count).
 * x + 1 is the next element of a row and y + 1 the next row.
 */
#ifndef SSLBM_H
#define SSLBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SSLBM_OK = 0,
    SSLBM_E_ARG = -1,         /* null pointer, bad size, negative rate/diffusivity, dx or dt <= 0 */
    SSLBM_E_UNSTABLE = -2,    /* parameters outside the linear stability region (see sslbm_init) */
    SSLBM_E_UNSUPPORTED = -3, /* valid request this build does not serve (e.g. BGK with d[4] != 0) */
    SSLBM_E_ALIAS = -4,       /* input and output buffers overlap */
    SSLBM_E_HIP = -5,         /* a HIP call or kernel launch failed; see sslbm_last_hip_error */
    SSLBM_E_NOMEM = -6,       /* host allocation of the context failed */
    SSLBM_E_LIMIT = -7        /* the request needs more than a fixed-size buffer of the library holds */
} sslbm_status;

typedef enum { SSLBM_F32 = 0, SSLBM_F64 = 1 } sslbm_dtype;     /* storage and arithmetic type */
typedef enum { SSLBM_PERIODIC = 0, SSLBM_NOFLUX = 1 } sslbm_bc;

/*
 * Model parameters, in the paper's notation (Sec. II.A, Table "Table_params"):
 *   beta  contact rate, alpha inverse incubation period, gamma removal rate,
 *   phi   infection fatality ratio (0 <= phi <= 1), all rates per unit time;
 *   d[C]  diffusivity of S, E, I, R, D in length^2 / time (the paper keeps
 *         D at rest, d[4] = 0; a nonzero d[4] makes D a fifth mobile
 *         compartment under the same update);
 *   dx    lattice spacing, dt time step.
 * The lattice diffusivity is d_lu = d dt / dx^2 and the relaxation time
 * tau = 1/2 + 3 d_lu, Eq. (diffusivity) with c_s^2 = 1/3.
 * Workloads stated with (beta, sigma, gamma, mu) map to alpha = sigma,
 * gamma_paper = gamma + mu, phi = mu / (gamma + mu).
 */
typedef struct {
    double beta, alpha, gamma, phi;
    double d[5];
    double dx, dt;
} sslbm_params;

typedef struct sslbm_ctx sslbm_ctx;

/*
 * Create a context for an nx-by-ny grid.
 * dtype: SSLBM_F32 or SSLBM_F64 (element type of every buffer, and the
 *        arithmetic precision). bc: SSLBM_PERIODIC or SSLBM_NOFLUX. Both
 *        are passed as int so that any other value is rejected (an enum
 *        parameter could not hold one in C++).
 * Validation (no GPU needed):
 *   SSLBM_E_ARG      out or p null; nx, ny < 1 or above 1<<20; unknown dtype or
 *                    bc; any rate or d negative or not finite; phi > 1;
 *                    dx or dt not > 0.
 *   SSLBM_E_UNSTABLE some d_lu > 1/4 (the diffusion amplification factor
 *                    G(k) = 1 - 2 d_lu (2 - cos kx - cos ky) leaves [-1, 1];
 *                    Sec. II.C.2, stability of the purely diffusive case), or
 *                    dt |lambda_2| + 8 max(d_lu^E, d_lu^I) > 2, where
 *                    lambda_2 is the negative eigenvalue of the E-I block at
 *                    the disease-free equilibrium, Eq. (eigenvalues): the
 *                    decaying mode of the linearised update would oscillate
 *                    with growing amplitude.
 * On success *out owns host memory released by sslbm_destroy.
 */
sslbm_status sslbm_init(sslbm_ctx **out, int nx, int ny, int dtype, int bc,
                        const sslbm_params *p);

/* Replace the parameters (same validation as sslbm_init); grid, dtype and bc stay. */
sslbm_status sslbm_set_params(sslbm_ctx *c, const sslbm_params *p);

/*
 * The parameter struct from rates stated as (beta, sigma, gamma, mu): beta
 * contact rate, sigma = 1 / incubation period, gamma recovery rate, mu
 * death rate. The paper's Eq. (sources) has alpha = sigma, a removal rate
 * gamma_paper = gamma + mu and a fatality ratio phi = mu / (gamma + mu).
 * d, dx, dt are copied as given. Host only. SSLBM_E_ARG: out or d null, a
 * rate negative or not finite, or gamma + mu not > 0. The result still goes
 * through sslbm_init's validation.
 */
sslbm_status sslbm_params_from_rates(double beta, double sigma, double gamma, double mu,
                                     const double d[5], double dx, double dt, sslbm_params *out);

/*
 * Gradients with respect to (beta, sigma, gamma, mu) from those with
 * respect to (beta, alpha, gamma_paper, phi), the first four of the nine
 * that sslbm_adjoint_run returns, by the chain rule of the mapping above at
 * the given gamma and mu:
 *   dL/dsigma = dL/dalpha,
 *   dL/dgamma = dL/dgamma_paper - dL/dphi mu / (gamma + mu)^2,
 *   dL/dmu    = dL/dgamma_paper + dL/dphi gamma / (gamma + mu)^2.
 * grad_rates may alias grad_params. Host only. SSLBM_E_ARG: a null pointer,
 * gamma or mu negative or not finite, or gamma + mu not > 0.
 */
sslbm_status sslbm_rate_gradients(const double grad_params[4], double gamma, double mu,
                                  double grad_rates[4]);

/*
 * Blocking depth: the number of time steps sslbm_run advances per pass over
 * HBM (each pass reads and writes the five fields once). 0 restores the
 * automatic choice. Allowed range 0..SSLBM_MAX_BLOCKING; results are bit for
 * bit the same for every depth. Shorthand for the steps_per_pass field of
 * sslbm_set_launch below.
 */
#define SSLBM_MAX_BLOCKING 8
sslbm_status sslbm_set_blocking(sslbm_ctx *c, int steps_per_pass);
int sslbm_get_blocking(const sslbm_ctx *c);

/*
 * Launch shape of the pass kernel used by sslbm_run (sslbm_step always takes
 * one step per pass). Each wavefront owns a strip of 64 * cols_per_lane
 * columns, of which 64 * cols_per_lane - 2 * steps_per_pass (the halo rounded
 * up to a multiple of cols_per_lane) are output, and marches down
 * rows_per_wave output rows. Zero in a field selects the automatic value.
 * Shapes change speed only, never results (bit for bit). Valid:
 * steps_per_pass 0..SSLBM_MAX_BLOCKING, rows_per_wave 0..65536,
 * cols_per_lane 0..2. A combination whose register footprint does not fit one
 * wavefront (FP32 above 6 steps with two columns per lane; FP64 above 5 with
 * one, above 2 with two) returns SSLBM_E_UNSUPPORTED.
 * sslbm_get_launch reports the shape sslbm_run uses (automatic fields resolved).
 */
typedef struct {
    int steps_per_pass;
    int rows_per_wave;
    int cols_per_lane;
} sslbm_launch;
sslbm_status sslbm_set_launch(sslbm_ctx *c, const sslbm_launch *shape);
sslbm_status sslbm_get_launch(const sslbm_ctx *c, sslbm_launch *shape);

/*
 * Autotuner: times candidate launch shapes of sslbm_run on the caller's
 * state and keeps the fastest (it becomes the context's shape; *best, if not
 * NULL, receives it). Candidates: one and (for an even row length and
 * pair-aligned buffers) two columns per lane; every depth from 1 to the
 * register limit; rows_per_wave automatic (one round of resident
 * wavefronts) and 8, 16, 32, 64, 128 where at least twice the depth. Each
 * candidate runs one untimed and three timed passes rho -> scratch (device
 * buffers of 5 * nx * ny elements, not overlapping): rho is only read,
 * scratch is overwritten. Timed with HIP events on hip_stream after
 * synchronizing it; the call returns when tuning is done. Useful where the
 * automatic shape is far from the best, chiefly grids too small to give
 * every resident wavefront a tall chunk.
 */
sslbm_status sslbm_tune(sslbm_ctx *c, const void *rho, void *scratch, void *hip_stream,
                        sslbm_launch *best);

/*
 * One SSLBM time step for all five compartments, Eq. (sslbm_final_clean)
 * with rho_f, rho_b, rho_c of Eqs. (rhof), (rhob), (rhoc) for the mobile
 * compartments, the sources of Eq. (sources) and forward Euler for D,
 * Eq. (rhoD); every source term uses the densities at time t of the same node.
 * On the D2Q5 lattice rho_f and rho_b hold the same five values with the
 * same weights, so the update is computed as
 *   rho(t+dt) = rho + d_lu ((rho_N + rho_S) + (rho_E + rho_W) - 4 rho) + Psi dt.
 * Boundaries: periodic wrap, or no-flux (a neighbour outside the domain takes
 * the centre value, so nothing crosses the wall; Sec. II.C.2, mass
 * conservation).
 * rho_in, rho_out: device, layout rho, must not overlap (SSLBM_E_ALIAS).
 * The force of infection is zero where S + E + I + R <= 0, and in FP32 also
 * where that sum is a positive subnormal number (below 2^-126): the quotient
 * dropped there is below 2^-126 beta dt for non-negative densities.
 */
sslbm_status sslbm_step(sslbm_ctx *c, const void *rho_in, void *rho_out, void *hip_stream);

/*
 * nsteps SSLBM steps, several per HBM pass (see sslbm_set_blocking). The
 * result is left in rho; scratch is a device buffer of the same size whose
 * contents are undefined afterwards. Bit for bit equal to nsteps calls of
 * sslbm_step. nsteps = 0 leaves rho unchanged. rho and scratch must not overlap.
 */
sslbm_status sslbm_run(sslbm_ctx *c, void *rho, void *scratch, long long nsteps, void *hip_stream);

/*
 * How sslbm_run splits nsteps into passes with the context's current pass
 * shape: the fewest passes of at most steps_per_pass steps, one more if that
 * makes their count even and leaves every pass a step (the ping-pong then
 * ends in rho, with no copy), and the steps spread evenly over them: the
 * first passes take *longest steps, the rest *shortest (equal when the split
 * is exact). Host only, no device call. *passes = 0 for nsteps = 0.
 * longest and shortest may be NULL.
 */
sslbm_status sslbm_plan_run(const sslbm_ctx *c, long long nsteps, long long *passes, int *longest,
                            int *shortest);

/*
 * BGK comparison scheme, Eq. (pdf) with f^eq = w_i rho, the source w_i Psi dt
 * and tau from Eq. (diffusivity); collide then stream to x + c_i (periodic
 * wrap, or half-way bounce-back at no-flux walls). rho^D follows Eq. (rhoD)
 * by forward Euler. The paper's BGK carries D as a density, so every bgk_*
 * call returns SSLBM_E_UNSUPPORTED when d[4] != 0.
 *   bgk_init:    f_i = w_i rho (equilibrium start), rhoD = rho[D].
 *   bgk_step:    one step, f_in/rhoD_in -> f_out/rhoD_out (no overlap).
 *   bgk_run:     nsteps steps in place in f/rhoD, using same-size scratch
 *                (the steps alternate between the two; an odd nsteps ends
 *                with a copy of the state from the scratch into f/rhoD).
 *   bgk_density: rho[C] = sum_i f_i for S, E, I, R and rho[D] = rhoD.
 */
sslbm_status bgk_init(sslbm_ctx *c, const void *rho, void *f, void *rhoD, void *hip_stream);
sslbm_status bgk_step(sslbm_ctx *c, const void *f_in, const void *rhoD_in, void *f_out,
                      void *rhoD_out, void *hip_stream);
sslbm_status bgk_run(sslbm_ctx *c, void *f, void *rhoD, void *f_scratch, void *rhoD_scratch,
                     long long nsteps, void *hip_stream);
sslbm_status bgk_density(sslbm_ctx *c, const void *f, const void *rhoD, void *rho,
                         void *hip_stream);

/*
 * The finite-difference reference solver of Sec. III, used to validate the
 * SSLBM and to time the comparison the paper makes: the PDEs of
 * Eqs. (EqSEIRD_S)-(EqSEIRD_D) with the Laplacian by fourth-order centred
 * differences, (-u(-2) + 16 u(-1) - 30 u + 16 u(+1) - u(+2)) / (12 dx^2) per
 * axis, the classic fourth-order Runge-Kutta method in time, and the
 * reactions evaluated at every stage. The context's parameters, grid,
 * arithmetic type and walls apply; a no-flux wall takes ghost values by
 * even reflection about the boundary face (u(-1) = u(0), u(-2) = u(1)), a
 * periodic wall wraps. Every context sslbm_init accepts is stable here too
 * (d_lu <= 1/4 keeps dt d (32/3) / dx^2 inside the RK4 stability interval,
 * whose real extent is 2.78).
 *
 *   sslbm_fd4_workspace_bytes: bytes of the workspace sslbm_fd4_run needs
 *       (three states), 0 for a null context.
 *   sslbm_fd4_run: nsteps steps in place in rho (device, layout as
 *       sslbm_step), work a device buffer of work_bytes >= the workspace
 *       size, caller-owned and clobbered. SSLBM_E_ARG for null pointers,
 *       negative nsteps, a short or misaligned buffer; SSLBM_E_ALIAS if rho
 *       and work overlap. Four launches per step, queued on hip_stream.
 */
size_t sslbm_fd4_workspace_bytes(const sslbm_ctx *c);
sslbm_status sslbm_fd4_run(sslbm_ctx *c, void *rho, void *work, size_t work_bytes, long long nsteps,
                           void *hip_stream);

/*
 * Total population per compartment, out_totals[C] = sum_x rho[C](x) in FP64,
 * the quantity conserved by Eq. (mass_conservation) when summed over C.
 * Deterministic (fixed reduction order). Waits for the stream. The first
 * call allocates a small device buffer (5 doubles per block) kept by the
 * context until sslbm_destroy.
 */
sslbm_status sslbm_total(sslbm_ctx *c, const void *rho, double out_totals[5], void *hip_stream);

/* Release a context (NULL is allowed). */
void sslbm_destroy(sslbm_ctx *c);

/*
 * Reverse mode (adjoint). For a loss J of the state at the end of a run,
 * lam(t) = dJ/d rho(t) satisfies lam(t) = A(rho(t))^T lam(t + dt), A the
 * Jacobian of one step of Eq. (sslbm_final_clean) with the sources of
 * Eq. (sources) and Eq. (rhoD) (the deceased at rest follow forward Euler).
 * The gradient of J with respect to the parameters is the sum over steps of
 * each step's partial derivatives contracted with lam(t + dt). Gradients are
 * packed as grad[9] = dJ/d(beta, alpha, gamma, phi, d[0], ..., d[4]) with the
 * physical diffusivities of sslbm_params; dJ/d d[4] at d[4] = 0 is the
 * one-sided derivative for d[4] >= 0. All sums are deterministic.
 *
 *   sslbm_adjoint_step: lam_out = A(rho)^T lam_next for the state rho at time
 *       t and lam_next = dJ/d rho(t + dt) (device buffers, layout of rho);
 *       the step's parameter gradient is ADDED to grad, a device array of 9
 *       doubles. lam_out may not overlap rho, lam_next or grad. The first
 *       call allocates a small device buffer kept by the context.
 *   sslbm_checkpoint_count: ceil(nsteps / every), the number of states
 *       sslbm_run_checkpointed stores; -1 for nsteps < 0 or every < 1.
 *   sslbm_run_checkpointed: as sslbm_run (result in rho, scratch clobbered),
 *       and stores the state at steps 0, every, 2 every, ... into
 *       checkpoints, a device buffer of sslbm_checkpoint_count states. For
 *       every up to the deepest single pass of the dtype (5 in FP64, 8 in
 *       FP32) each segment is one pass written straight into the next
 *       checkpoint (scratch unused), two segments per pass when every
 *       = 2; the reverse sweep then recomputes nothing, at the cost of
 *       nsteps / 2 stored states (1024^2 FP64 x 2000 steps: 42 GB).
 *   sslbm_adjoint_workspace_bytes: bytes of device workspace the reverse
 *       sweep needs for this context and checkpoint interval (about
 *       every / 2 + 1 states plus 128 bytes per wavefront of the adjoint
 *       kernels); 0 for a bad argument.
 *   sslbm_adjoint_run: the reverse sweep of a run of nsteps steps recorded
 *       by sslbm_run_checkpointed with the same every and parameters. On
 *       entry lam holds dJ/d rho(T); on return dJ/d rho(0). The run's
 *       parameter gradient is ADDED to grad (device, 9 doubles). Each segment
 *       of `every` steps is recomputed from its checkpoint, every second state
 *       into the workspace (never read before it is written; clobbered); the
 *       reverse steps then go two per pass, the state in between recomputed
 *       on chip. Buffers may not overlap.
 * Errors: SSLBM_E_ARG (NULL pointer, nsteps < 0, every < 1), SSLBM_E_ALIAS,
 * SSLBM_E_HIP.
 */
#define SSLBM_GRAD_COUNT 9
sslbm_status sslbm_adjoint_step(sslbm_ctx *c, const void *rho, const void *lam_next, void *lam_out,
                                double *grad, void *hip_stream);

/*
 * sslbm_adjoint_step_noalloc: sslbm_adjoint_step for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc). Same arguments, results and
 * errors, bit for bit; it calls no hipMalloc, hipFree or other allocating
 * routine. The step's per-wavefront partial sums go to a fixed device
 * array of the library (SSLBM_ADJ_NOALLOC_SLOTS slots of 128 bytes,
 * 512 KiB, held on every GPU the library runs on until the process ends)
 * instead of a buffer of the context. Every slot the step reads is written
 * earlier in the same call, so nothing is carried over between calls; but
 * all calls on one GPU share that array, so calls that overlap in time on
 * one GPU (two streams, two threads) race and give wrong gradients.
 * Grids needing more slots than the array holds (one slot per wavefront:
 * about ceil(nx / 62) x max(1, 1024 / ceil(nx / 62)) wavefronts, so rows of
 * more than about 250000 cells) return SSLBM_E_LIMIT before any device call.
 */
#define SSLBM_ADJ_NOALLOC_SLOTS 4096
sslbm_status sslbm_adjoint_step_noalloc(sslbm_ctx *c, const void *rho, const void *lam_next,
                                        void *lam_out, double *grad, void *hip_stream);
long long sslbm_checkpoint_count(long long nsteps, int every);
sslbm_status sslbm_run_checkpointed(sslbm_ctx *c, void *rho, void *scratch, long long nsteps,
                                    int every, void *checkpoints, void *hip_stream);
size_t sslbm_adjoint_workspace_bytes(const sslbm_ctx *c, int every);
sslbm_status sslbm_adjoint_run(sslbm_ctx *c, const void *checkpoints, long long nsteps, int every,
                               void *lam, double *grad, void *workspace, void *hip_stream);

/*
 * Ensembles: many independent SSLBM grids of different sizes and parameters
 * advanced together (each instance gets exactly the bits sslbm_run would
 * give it alone).
 *
 * State layout: one device buffer holds all instances; instance i is a
 * [5][ny_i][nx_i] block at element offset sslbm_ensemble_offset(e, i)
 * (offsets are multiples of 4 elements; gaps between blocks hold no data and
 * their contents after a run are unspecified).
 * sslbm_ensemble_elements(e) is the buffer length in elements.
 *
 * Size classes. Instances whose five fields fit in 80 KiB (64 x 64 in
 * FP32) form the on-chip class: one launch holds each of them in the LDS
 * of one workgroup for every step of a run, reading and writing its fields
 * once. The others are grouped by the power-of-two bucket of their longest
 * side (up to 128, 256, 512, ...); each such march class takes passes of
 * several steps (as sslbm_run) with a pass shape of its own. During a run the
 * classes advance side by side, each on its own stream or graph branch.
 *
 *   sslbm_ensemble_create: count >= 1 instances; nx, ny: host arrays of
 *       count grid sizes (1 .. 65536 each); params: host array of count
 *       parameter sets (each validated as in sslbm_init); dtype and bc as in
 *       sslbm_init, shared by all instances. Host memory only; device tables
 *       are built on first use. Errors: SSLBM_E_ARG, SSLBM_E_UNSTABLE (with
 *       the failing instance index in *bad_instance if not NULL).
 *   sslbm_ensemble_class_count: number of size classes (>= 1).
 *   sslbm_ensemble_instance_class: the class of an instance.
 *   sslbm_ensemble_class_info: what a class holds and, for a march class,
 *       its resolved pass shape (zeros for the on-chip class). Host only.
 *   sslbm_ensemble_set_class_launch: pass shape of one march class, as
 *       sslbm_set_launch (zero fields automatic; SSLBM_E_UNSUPPORTED for the
 *       on-chip class). sslbm_ensemble_set_launch sets it for every march
 *       class; sslbm_ensemble_get_launch reports the shape of the march
 *       class with the most cells (zeros if there is none).
 *   sslbm_ensemble_tune: times rounds of one pass of every march class side
 *       by side on the current state (reads rho, writes only scratch) and
 *       keeps the shapes with the highest joint rate (cell-updates per
 *       second): first one shape for all march classes, then each class in
 *       turn, largest first, tries its own candidates while the others keep
 *       theirs. Candidates: every depth and column count within the register
 *       budget, rows per wavefront automatic or 8, 16, 32, 64, 128. Reports
 *       the largest class's shape in *best if not NULL. Waits for the stream.
 *   sslbm_ensemble_run: nsteps steps of every instance, result in rho,
 *       scratch clobbered. With SSLBM_RUN_GRAPH in flags the work of all
 *       classes is captured once into one HIP graph (one branch per class;
 *       cached for the same nsteps and buffers until a shape changes) and
 *       replayed as one launch; the graph runs on a stream of the ensemble
 *       that is ordered after, and before, hip_stream. Without the flag the
 *       classes fork from and join back to hip_stream. The first call with a
 *       new shape uploads tables (synchronous).
 *   sslbm_ensemble_run_class: nsteps steps of the instances of one class
 *       only, on hip_stream (the other instances are left as they are).
 */
#define SSLBM_RUN_GRAPH 1
typedef struct sslbm_ensemble sslbm_ensemble;
typedef struct {
    int on_chip;          /* 1: the instances stay in LDS for a whole run */
    int instances;        /* instances in the class */
    long long cells;      /* sum of nx * ny over them */
    int max_side;         /* their longest side */
    sslbm_launch launch;  /* pass shape of a march class, resolved; zeros on chip */
} sslbm_ensemble_class;
sslbm_status sslbm_ensemble_create(sslbm_ensemble **out, int count, const int *nx, const int *ny,
                                   int dtype, int bc, const sslbm_params *params,
                                   int *bad_instance);
long long sslbm_ensemble_offset(const sslbm_ensemble *e, int instance);
long long sslbm_ensemble_elements(const sslbm_ensemble *e);
int sslbm_ensemble_class_count(const sslbm_ensemble *e);
int sslbm_ensemble_instance_class(const sslbm_ensemble *e, int instance);
sslbm_status sslbm_ensemble_class_info(const sslbm_ensemble *e, int cls,
                                       sslbm_ensemble_class *info);
sslbm_status sslbm_ensemble_set_class_launch(sslbm_ensemble *e, int cls, const sslbm_launch *shape);
sslbm_status sslbm_ensemble_set_launch(sslbm_ensemble *e, const sslbm_launch *shape);
sslbm_status sslbm_ensemble_get_launch(const sslbm_ensemble *e, sslbm_launch *shape);
sslbm_status sslbm_ensemble_tune(sslbm_ensemble *e, const void *rho, void *scratch,
                                 void *hip_stream, sslbm_launch *best);
sslbm_status sslbm_ensemble_run(sslbm_ensemble *e, void *rho, void *scratch, long long nsteps,
                                int flags, void *hip_stream);
sslbm_status sslbm_ensemble_run_class(sslbm_ensemble *e, int cls, void *rho, void *scratch,
                                      long long nsteps, void *hip_stream);
int sslbm_ensemble_last_hip_error(const sslbm_ensemble *e);
void sslbm_ensemble_destroy(sslbm_ensemble *e);

/*
 * Generic compartmental models, Eq. (generic_pde): d_t C = Psi^C + d^C lap C
 * for 1..SSLBM_MAX_COMPARTMENTS compartments, SSLBM steps
 * (Eq. (sslbm_final_clean)) on the D2Q5 lattice (lattice = 5) or the D2Q9
 * lattice (lattice = 9: rest weight 4/9, axes 1/9, diagonals 1/36; its
 * symbol is 4/9 + (2/9)(cos kx + cos ky) + (1/9) cos kx cos ky, isotropic
 * to fourth order as the anisotropy analysis of Sec. II.C.2 states).
 * Layout: rho[compartments][ny][nx]. No-flux walls are mirror images (the
 * centre value on D2Q5, as sslbm_step); periodic walls wrap.
 *
 * Sources: transition r moves
 *     rate * C[src] * (catalyst >= 0 ? C[catalyst] : 1) / (frequency ? N : 1)
 * per unit time out of src into dst (dst = -1: out of the system), N being
 * the sum of the compartments with counted[c] != 0 (the flow is 0 where a
 * frequency-dependent transition sees N <= 0). The SEIRD model of Eq. (sources)
 * and Eq. (rhoD) is S->E (beta, catalyst I, frequency), E->I (alpha),
 * I->R ((1 - phi) gamma), I->D (phi gamma) with N = S + E + I + R.
 *
 *   sslbm_model_create: d (physical diffusivities, >= 0) and counted are host
 *       arrays of `compartments` entries; transitions: host array. Rejects
 *       (SSLBM_E_ARG) bad sizes, indices (src == dst, out of range), negative
 *       or non-finite rates; (SSLBM_E_UNSTABLE) any compartment with
 *       s * d_lu + dt * outflow > 2, s = 8 (D2Q5) or 16/3 (D2Q9), outflow the
 *       sum of its transitions' rates (density-dependent catalysis, whose
 *       flow has no bound, is left out). Host memory only.
 *   sslbm_model_step / sslbm_model_run: as sslbm_step / sslbm_run. The
 *       first call uploads a small transition table to the current device
 *       (synchronous); the model then stays on that device
 *       (SSLBM_E_UNSUPPORTED elsewhere). sslbm_model_step takes one step;
 *       sslbm_model_run takes up to the model's blocking depth of steps per
 *       pass over device memory.
 *   sslbm_model_set_blocking: steps per pass of sslbm_model_run, 1 ..
 *       SSLBM_MODEL_MAX_BLOCKING, or 0 for the automatic choice (else
 *       SSLBM_E_ARG). Results are bit for bit the same for every depth.
 *   sslbm_model_get_blocking: the depth sslbm_model_run uses (automatic
 *       choice resolved) into *steps_per_pass.
 */
#define SSLBM_MAX_COMPARTMENTS 8
#define SSLBM_MAX_TRANSITIONS 16
#define SSLBM_MODEL_MAX_BLOCKING 4
typedef struct {
    int src, dst, catalyst, frequency;
    double rate;
} sslbm_transition;
typedef struct sslbm_model sslbm_model;
sslbm_status sslbm_model_create(sslbm_model **out, int nx, int ny, int dtype, int bc,
                                int lattice, int compartments, const double *d, const int *counted,
                                double dx, double dt, int ntransitions,
                                const sslbm_transition *transitions);
sslbm_status sslbm_model_step(sslbm_model *m, const void *rho_in, void *rho_out, void *hip_stream);
sslbm_status sslbm_model_run(sslbm_model *m, void *rho, void *scratch, long long nsteps,
                             void *hip_stream);
sslbm_status sslbm_model_set_blocking(sslbm_model *m, int steps_per_pass);
sslbm_status sslbm_model_get_blocking(const sslbm_model *m, int *steps_per_pass);
int sslbm_model_last_hip_error(const sslbm_model *m);
void sslbm_model_destroy(sslbm_model *m);

/* Static description of a status code. */
const char *sslbm_strerror(int status);

/* hipError_t of the last failed HIP call made for this context (0 if none). */
int sslbm_last_hip_error(const sslbm_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* SSLBM_H */
