/*
 * oracle.c -- plain FP64 CPU oracle for the SSLBM SEIRD time step and for the
 * BGK lattice Boltzmann step it is compared with.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The product path (the
 * HIP library and its Python binding) never calls it, and this file shares no
 * code, header, table or constant with that path.
 *
 * Source: De Rosis, "A distribution-free lattice Boltzmann method for
 * compartmental reaction-diffusion systems with application to epidemic
 * modelling" (arXiv 2603.19789).
 *
 * Everything here is written for a reader checking it against the paper by
 * eye: literal formulas, one cell at a time, no blocking, no fusion, no
 * algebraic simplification. The only liberty is an OpenMP loop over rows,
 * which does not change any arithmetic (every output cell is computed by
 * exactly the same expression whatever the thread count).
 *
 * Notation (paper, Sec. II.A and Table "Table_params"):
 *   compartments C = S, E, I, R, D stored as rho[C][y][x], x fastest;
 *   rates beta (contact), alpha (1/incubation), gamma (removal), phi (fatality
 *   ratio); diffusivities d[C] in length^2/time; lattice spacing dx, step dt.
 *
 * Readings of points the paper leaves open (each one also listed in the
 * design notes of the repository):
 *   - the relaxation time follows Eq. (diffusivity) written in lattice units:
 *     d_lu = d*dt/dx^2 and tau = 1/2 + d_lu/c_s^2;
 *   - the force of infection is taken as zero where the contact-eligible
 *     population N_c <= 0 (the paper never divides by an empty cell);
 *   - no-flux boundary: a neighbour outside the domain takes the value of the
 *     centre cell (homogeneous Neumann, so the stencil difference across the
 *     wall is zero); BGK uses half-way bounce-back;
 *   - the deceased compartment does not diffuse in the paper (Sec. II.A) and
 *     follows the ODE of Eq. (rhoD), advanced by forward Euler with I at time
 *     t; if a caller gives D a nonzero diffusivity it is treated as a fifth
 *     mobile compartment with the SSLBM update;
 *   - BGK starts from equilibrium populations f_i = w_i rho.
 *
 * Parity: pinned by tests (closed forms, invariants, the paper's fourth-order
 * finite-difference reference, special cases, and planted-mistake tests).
 * The adjoint (reverse) step at the end of this file is pinned to the forward
 * step: the transpose identity <lam, A rho> = <A^T lam, rho> of the linear
 * case, self-adjointness of pure diffusion, and central finite differences.
 */
#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_E_ARG (-1)

#define BC_PERIODIC 0
#define BC_NOFLUX 1

enum { CS = 0, CE = 1, CI = 2, CR = 3, CD = 4 };

/* D2Q5 lattice, Sec. II.B: link vectors c_i = (c_ix, c_iy) and weights. */
static const int CX[5] = {0, 1, 0, -1, 0};
static const int CY[5] = {0, 0, 1, 0, -1};
static const double W[5] = {1.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0, 1.0 / 6.0};
/* direction opposite to i: c_opp(i) = -c_i (used by bounce-back only) */
static const int OPP[5] = {0, 3, 4, 1, 2};
/* lattice speed of sound squared, c_s = 1/sqrt(3) (Sec. II.B) */
static const double CS2 = 1.0 / 3.0;

/* rates[] layout: beta, alpha, gamma, phi */
typedef struct {
    double beta, alpha, gamma, phi;
} seird_rates;

static seird_rates unpack_rates(const double *r)
{
    seird_rates k;
    k.beta = r[0];
    k.alpha = r[1];
    k.gamma = r[2];
    k.phi = r[3];
    return k;
}

/* Relaxation time of compartment C from its diffusivity, Eq. (diffusivity):
 * d = c_s^2 (tau - 1/2) in lattice units, lattice diffusivity d*dt/dx^2. */
static double relaxation_time(double d, double dx, double dt)
{
    double d_lattice = d * dt / (dx * dx);
    return 0.5 + d_lattice / CS2;
}

/* Value of one field at lattice node (x, y); (xc, yc) is the centre node of
 * the stencil being evaluated, used by the no-flux rule. */
static double node_value(const double *field, int nx, int ny, int bc, int x, int y,
                         int xc, int yc)
{
    if (x < 0 || x >= nx || y < 0 || y >= ny) {
        if (bc == BC_PERIODIC) {
            x = ((x % nx) + nx) % nx;
            y = ((y % ny) + ny) % ny;
        } else {
            return field[(size_t)yc * nx + xc];
        }
    }
    return field[(size_t)y * nx + x];
}

/* SEIRD reaction sources, Eq. (sources) for S, E, I, R and Eq. (rhoD) for D,
 * all evaluated from the densities of one node at time t. */
static void seird_sources(const double rho[5], seird_rates k, double psi[5])
{
    double S = rho[CS], E = rho[CE], I = rho[CI], R = rho[CR];
    double Nc = S + E + I + R; /* contact-eligible population (excludes D) */
    double force = 0.0;
    if (Nc > 0.0)
        force = k.beta * S * I / Nc;
    psi[CS] = -force;
    psi[CE] = force - k.alpha * E;
    psi[CI] = k.alpha * E - k.gamma * I;
    psi[CR] = (1.0 - k.phi) * k.gamma * I;
    psi[CD] = k.phi * k.gamma * I;
}

static int valid_grid(int nx, int ny, int bc)
{
    return nx >= 1 && ny >= 1 && (bc == BC_PERIODIC || bc == BC_NOFLUX);
}

/*
 * One SSLBM step for all five compartments, out of place.
 * Eq. (sslbm_final_clean) with rho_f, rho_b, rho_c from Eqs. (rhof), (rhob),
 * (rhoc), for the mobile compartments; Eq. (rhoD) by forward Euler for D when
 * it does not diffuse.
 */
int oracle_sslbm_step(int nx, int ny, int bc, const double *rates, const double *d,
                      double dx, double dt, const double *in, double *out, int nthreads)
{
    if (!valid_grid(nx, ny, bc) || !rates || !d || !in || !out || in == out)
        return ORACLE_E_ARG;
    seird_rates k = unpack_rates(rates);
    double tau[5];
    for (int c = 0; c < 5; ++c)
        tau[c] = relaxation_time(d[c], dx, dt);
    size_t plane = (size_t)nx * ny;
    if (nthreads <= 0)
        nthreads = 1;

#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t cell = (size_t)y * nx + x;
            double centre[5], psi[5];
            for (int c = 0; c < 5; ++c)
                centre[c] = in[c * plane + cell];
            seird_sources(centre, k, psi);

            for (int c = 0; c < 5; ++c) {
                const double *field = in + c * plane;
                if (c == CD && d[CD] == 0.0) {
                    /* deceased: d rho^D / dt = phi gamma rho^I, Eq. (rhoD) */
                    out[c * plane + cell] = centre[CD] + psi[CD] * dt;
                    continue;
                }
                double rho_f = 0.0, rho_b = 0.0;
                for (int i = 0; i < 5; ++i) {
                    rho_f += W[i] * node_value(field, nx, ny, bc, x + CX[i], y + CY[i], x, y);
                    rho_b += W[i] * node_value(field, nx, ny, bc, x - CX[i], y - CY[i], x, y);
                }
                double rho_c = centre[c];
                out[c * plane + cell] =
                    rho_b + (tau[c] - 1.0) * (rho_f - 2.0 * rho_c + rho_b) + psi[c] * dt;
            }
        }
    }
    return ORACLE_OK;
}

/* nsteps SSLBM steps; result left in rho, work is a buffer of the same size. */
int oracle_sslbm_run(int nx, int ny, int bc, const double *rates, const double *d,
                     double dx, double dt, double *rho, double *work, long long nsteps,
                     int nthreads)
{
    if (!valid_grid(nx, ny, bc) || !rho || !work || rho == work || nsteps < 0)
        return ORACLE_E_ARG;
    double *a = rho, *b = work;
    for (long long n = 0; n < nsteps; ++n) {
        int rc = oracle_sslbm_step(nx, ny, bc, rates, d, dx, dt, a, b, nthreads);
        if (rc)
            return rc;
        double *t = a;
        a = b;
        b = t;
    }
    if (a != rho)
        memcpy(rho, a, sizeof(double) * 5 * (size_t)nx * ny);
    return ORACLE_OK;
}

/* ---------------------------------------------------------------- BGK --- */
/* Populations f[C][i][y][x] for the four mobile compartments C = S, E, I, R,
 * directions i = 0..4; the deceased are carried as a density (Sec. II.B: the
 * BGK storage holds five populations for four mobile groups plus rho^D). */

static size_t fidx(int c, int i, size_t plane) { return ((size_t)c * 5 + i) * plane; }

/* Equilibrium start, f_i = w_i rho (reading: the paper does not state it). */
int oracle_bgk_init(int nx, int ny, const double *rho, double *f, double *rhoD)
{
    if (nx < 1 || ny < 1 || !rho || !f || !rhoD)
        return ORACLE_E_ARG;
    size_t plane = (size_t)nx * ny;
    for (int c = 0; c < 4; ++c)
        for (int i = 0; i < 5; ++i)
            for (size_t p = 0; p < plane; ++p)
                f[fidx(c, i, plane) + p] = W[i] * rho[c * plane + p];
    for (size_t p = 0; p < plane; ++p)
        rhoD[p] = rho[CD * plane + p];
    return ORACLE_OK;
}

/* Macroscopic densities rho^C = sum_i f_i^C (Sec. II.B), plus rho^D. */
int oracle_bgk_density(int nx, int ny, const double *f, const double *rhoD, double *rho)
{
    if (nx < 1 || ny < 1 || !rho || !f || !rhoD)
        return ORACLE_E_ARG;
    size_t plane = (size_t)nx * ny;
    for (int c = 0; c < 4; ++c)
        for (size_t p = 0; p < plane; ++p) {
            double s = 0.0;
            for (int i = 0; i < 5; ++i)
                s += f[fidx(c, i, plane) + p];
            rho[c * plane + p] = s;
        }
    for (size_t p = 0; p < plane; ++p)
        rho[CD * plane + p] = rhoD[p];
    return ORACLE_OK;
}

/*
 * One BGK step, Eq. (pdf): collide with f^eq = w_i rho and the source w_i Psi dt,
 * then stream to x + c_i. Periodic wrap or half-way bounce-back. rho^D follows
 * Eq. (rhoD) by forward Euler. The deceased must not diffuse here.
 */
int oracle_bgk_step(int nx, int ny, int bc, const double *rates, const double *d,
                    double dx, double dt, const double *f_in, const double *rhoD_in,
                    double *f_out, double *rhoD_out, int nthreads)
{
    if (!valid_grid(nx, ny, bc) || !rates || !d || !f_in || !rhoD_in || !f_out ||
        !rhoD_out || f_in == f_out || rhoD_in == rhoD_out || d[CD] != 0.0)
        return ORACLE_E_ARG;
    seird_rates k = unpack_rates(rates);
    double tau[4];
    for (int c = 0; c < 4; ++c)
        tau[c] = relaxation_time(d[c], dx, dt);
    size_t plane = (size_t)nx * ny;
    if (nthreads <= 0)
        nthreads = 1;

#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t cell = (size_t)y * nx + x;
            double rho[5], psi[5];
            for (int c = 0; c < 4; ++c) {
                double s = 0.0;
                for (int i = 0; i < 5; ++i)
                    s += f_in[fidx(c, i, plane) + cell];
                rho[c] = s;
            }
            rho[CD] = rhoD_in[cell];
            seird_sources(rho, k, psi);

            for (int c = 0; c < 4; ++c) {
                for (int i = 0; i < 5; ++i) {
                    double f = f_in[fidx(c, i, plane) + cell];
                    double feq = W[i] * rho[c];
                    double fstar = f + (feq - f) / tau[c] + W[i] * psi[c] * dt;
                    int xd = x + CX[i], yd = y + CY[i];
                    if (xd < 0 || xd >= nx || yd < 0 || yd >= ny) {
                        if (bc == BC_PERIODIC) {
                            xd = (xd + nx) % nx;
                            yd = (yd + ny) % ny;
                        } else {
                            /* half-way bounce-back: returns reversed to this node */
                            f_out[fidx(c, OPP[i], plane) + cell] = fstar;
                            continue;
                        }
                    }
                    f_out[fidx(c, i, plane) + (size_t)yd * nx + xd] = fstar;
                }
            }
            rhoD_out[cell] = rho[CD] + psi[CD] * dt;
        }
    }
    return ORACLE_OK;
}

/* nsteps BGK steps; results in f, rhoD; f_work, rhoD_work have the same sizes. */
int oracle_bgk_run(int nx, int ny, int bc, const double *rates, const double *d, double dx,
                   double dt, double *f, double *rhoD, double *f_work, double *rhoD_work,
                   long long nsteps, int nthreads)
{
    if (!f || !rhoD || !f_work || !rhoD_work || nsteps < 0)
        return ORACLE_E_ARG;
    double *fa = f, *fb = f_work, *da = rhoD, *db = rhoD_work;
    for (long long n = 0; n < nsteps; ++n) {
        int rc = oracle_bgk_step(nx, ny, bc, rates, d, dx, dt, fa, da, fb, db, nthreads);
        if (rc)
            return rc;
        double *t = fa;
        fa = fb;
        fb = t;
        t = da;
        da = db;
        db = t;
    }
    size_t plane = (size_t)nx * ny;
    if (fa != f) {
        memcpy(f, fa, sizeof(double) * 20 * plane);
        memcpy(rhoD, da, sizeof(double) * plane);
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------ adjoint --- */
/*
 * Reverse step of oracle_sslbm_step: given lam_next = dJ/d rho(t+dt), return
 * lam_out = dJ/d rho(t) and add dJ/d(beta, alpha, gamma, phi, d[0..4]) of
 * this step to grad[9]. Written as the exact transpose of the literal update
 * above: every term w_i rho(x -/+ c_i) of rho_b / rho_f hands its weight back
 * to the node it read (the centre itself for a no-flux ghost), and every
 * source term hands back its partial derivatives at (x, t).
 */
int oracle_sslbm_adjoint_step(int nx, int ny, int bc, const double *rates, const double *d,
                              double dx, double dt, const double *rho, const double *lam_next,
                              double *lam_out, double *grad)
{
    if (!valid_grid(nx, ny, bc) || !rates || !d || !rho || !lam_next || !lam_out || !grad ||
        lam_out == lam_next)
        return ORACLE_E_ARG;
    seird_rates k = unpack_rates(rates);
    double tau[5];
    for (int c = 0; c < 5; ++c)
        tau[c] = relaxation_time(d[c], dx, dt);
    size_t plane = (size_t)nx * ny;
    memset(lam_out, 0, sizeof(double) * 5 * plane);

    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t cell = (size_t)y * nx + x;
            double centre[5], lam[5];
            for (int c = 0; c < 5; ++c) {
                centre[c] = rho[c * plane + cell];
                lam[c] = lam_next[c * plane + cell];
            }
            /* transport part, compartment by compartment */
            for (int c = 0; c < 5; ++c) {
                const double *field = rho + c * plane;
                double *back = lam_out + c * plane;
                /* A deceased compartment at rest moves by forward Euler only:
                 * D(t+dt) = D(t) + phi gamma I dt, so its transport is the
                 * identity. Its d-gradient is still the one-sided derivative of
                 * the SSLBM update at d = 0, which coincides with that update. */
                int at_rest = (c == CD && d[CD] == 0.0);
                double rho_f = 0.0, rho_b = 0.0;
                for (int i = 0; i < 5; ++i) {
                    /* rho_b reads x - c_i with weight w_i (1 + (tau - 1)) = w_i tau */
                    int xb = x - CX[i], yb = y - CY[i];
                    /* rho_f reads x + c_i with weight w_i (tau - 1) */
                    int xf = x + CX[i], yf = y + CY[i];
                    size_t nb_b = cell, nb_f = cell;
                    if (xb >= 0 && xb < nx && yb >= 0 && yb < ny)
                        nb_b = (size_t)yb * nx + xb;
                    else if (bc == BC_PERIODIC)
                        nb_b = (size_t)(((yb % ny) + ny) % ny) * nx + ((xb % nx) + nx) % nx;
                    if (xf >= 0 && xf < nx && yf >= 0 && yf < ny)
                        nb_f = (size_t)yf * nx + xf;
                    else if (bc == BC_PERIODIC)
                        nb_f = (size_t)(((yf % ny) + ny) % ny) * nx + ((xf % nx) + nx) % nx;
                    if (!at_rest) {
                        back[nb_b] += lam[c] * W[i] * tau[c];
                        back[nb_f] += lam[c] * W[i] * (tau[c] - 1.0);
                    }
                    rho_b += W[i] * field[nb_b];
                    rho_f += W[i] * field[nb_f];
                }
                if (at_rest)
                    back[cell] += lam[c];
                else
                    back[cell] += lam[c] * (-2.0) * (tau[c] - 1.0);
                /* d out / d tau = rho_f - 2 rho_c + rho_b; tau = 1/2 + 3 d dt / dx^2 */
                grad[4 + c] += lam[c] * (rho_f - 2.0 * centre[c] + rho_b) * 3.0 * dt / (dx * dx);
            }
            /* source part: out += Psi(rho(x, t)) dt */
            double S = centre[CS], E = centre[CE], I = centre[CI], R = centre[CR];
            double Nc = centre[CS] + centre[CE] + centre[CI] + centre[CR];
            double lS = lam[CS], lE = lam[CE], lI = lam[CI], lR = lam[CR], lD = lam[CD];
            if (Nc > 0.0) {
                double F = k.beta * S * I / Nc; /* force of infection */
                /* dF/dS, dF/dE, dF/dI, dF/dR */
                double fS = k.beta * I / Nc - F / Nc;
                double fE = -F / Nc;
                double fI = k.beta * S / Nc - F / Nc;
                double fR = -F / Nc;
                double g = (lE - lS) * dt; /* F enters S with -1 and E with +1 */
                lam_out[CS * plane + cell] += g * fS;
                lam_out[CE * plane + cell] += g * fE;
                lam_out[CI * plane + cell] += g * fI;
                lam_out[CR * plane + cell] += g * fR;
                grad[0] += (lE - lS) * dt * S * I / Nc;
            }
            /* alpha E moves E -> I; gamma I leaves I, (1 - phi) to R, phi to D */
            lam_out[CE * plane + cell] += (lI - lE) * k.alpha * dt;
            lam_out[CI * plane + cell] +=
                (-lI + (1.0 - k.phi) * lR + k.phi * lD) * k.gamma * dt;
            grad[1] += (lI - lE) * E * dt;
            grad[2] += (-lI + (1.0 - k.phi) * lR + k.phi * lD) * I * dt;
            grad[3] += (lD - lR) * k.gamma * I * dt;
        }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------ generic models --- */
/*
 * Generic compartmental model, Eq. (generic_pde): d_t C = Psi^C + d^C lap C
 * for M compartments, advanced by Eq. (sslbm_final_clean) on the D2Q5 or the
 * D2Q9 lattice (Sec. II.C.2, anisotropy paragraph: D2Q9 with rest weight
 * 4/9, axis weights 1/9 and diagonal weights 1/36). The source is a list of
 * transitions; transition r moves the flow
 *     f_r = rate_r * C[src_r] * (cat_r >= 0 ? C[cat_r] : 1) / (freq_r ? N : 1)
 * out of compartment src_r and into dst_r (dst_r < 0: out of the system),
 * with N the sum of the compartments flagged in `counted` (f_r = 0 where a
 * frequency-dependent transition sees N <= 0). The SEIRD sources of
 * Eq. (sources) and Eq. (rhoD) are the transitions S->E (rate beta, catalyst
 * I, frequency-dependent, N = S+E+I+R), E->I (alpha), I->R ((1-phi) gamma)
 * and I->D (phi gamma).
 * A compartment with d = 0 uses the same update (tau = 1/2), which leaves
 * only the source term: forward Euler, as Eq. (rhoD) for the deceased.
 * No-flux walls: the centre value on D2Q5 (as oracle_sslbm_step), the mirror
 * image on D2Q9 (node_value_mirror).
 */
static const int CX9[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY9[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double W9[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

#define GENERIC_MAX_COMPARTMENTS 8

/* No-flux wall on D2Q9: the field is extended by its mirror image about the
 * wall (homogeneous Neumann), coordinate by coordinate, so a diagonal ghost
 * across a wall takes the value of the node it mirrors. On D2Q5 this is the
 * same as taking the centre value (node_value). */
static double node_value_mirror(const double *field, int nx, int ny, int bc, int x, int y)
{
    if (bc == BC_PERIODIC) {
        x = (x + nx) % nx; /* |offset| <= 1 */
        y = (y + ny) % ny;
    } else {
        if (x < 0)
            x = -1 - x;
        if (x >= nx)
            x = 2 * nx - 1 - x;
        if (y < 0)
            y = -1 - y;
        if (y >= ny)
            y = 2 * ny - 1 - y;
    }
    return field[(size_t)y * nx + x];
}

int oracle_generic_step(int nx, int ny, int bc, int lattice, int m, const double *d, double dx,
                        double dt, int ntrans, const int *src, const int *dst, const int *cat,
                        const int *freq, const double *rate, const int *counted,
                        const double *in, double *out)
{
    if (!valid_grid(nx, ny, bc) || (lattice != 5 && lattice != 9) || m < 1 ||
        m > GENERIC_MAX_COMPARTMENTS || !d || ntrans < 0 || (ntrans && (!src || !dst || !cat ||
        !freq || !rate)) || !counted || !in || !out || in == out)
        return ORACLE_E_ARG;
    for (int r = 0; r < ntrans; ++r)
        if (src[r] < 0 || src[r] >= m || dst[r] >= m || cat[r] >= m)
            return ORACLE_E_ARG;
    const int *cx = lattice == 5 ? CX : CX9;
    const int *cy = lattice == 5 ? CY : CY9;
    const double *w = lattice == 5 ? W : W9;
    double tau[GENERIC_MAX_COMPARTMENTS];
    for (int c = 0; c < m; ++c)
        tau[c] = relaxation_time(d[c], dx, dt);
    size_t plane = (size_t)nx * ny;

    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t cell = (size_t)y * nx + x;
            double centre[GENERIC_MAX_COMPARTMENTS], psi[GENERIC_MAX_COMPARTMENTS];
            double total = 0.0;
            for (int c = 0; c < m; ++c) {
                centre[c] = in[c * plane + cell];
                psi[c] = 0.0;
                if (counted[c])
                    total += centre[c];
            }
            for (int r = 0; r < ntrans; ++r) {
                double flow = rate[r] * centre[src[r]];
                if (cat[r] >= 0)
                    flow *= centre[cat[r]];
                if (freq[r])
                    flow = total > 0.0 ? flow / total : 0.0;
                psi[src[r]] -= flow;
                if (dst[r] >= 0)
                    psi[dst[r]] += flow;
            }
            for (int c = 0; c < m; ++c) {
                const double *field = in + c * plane;
                double rho_f = 0.0, rho_b = 0.0;
                for (int i = 0; i < lattice; ++i) {
                    if (lattice == 5) {
                        rho_f += w[i] * node_value(field, nx, ny, bc, x + cx[i], y + cy[i], x, y);
                        rho_b += w[i] * node_value(field, nx, ny, bc, x - cx[i], y - cy[i], x, y);
                    } else {
                        rho_f += w[i] * node_value_mirror(field, nx, ny, bc, x + cx[i], y + cy[i]);
                        rho_b += w[i] * node_value_mirror(field, nx, ny, bc, x - cx[i], y - cy[i]);
                    }
                }
                double bracket = rho_f - 2.0 * centre[c] + rho_b;
                out[c * plane + cell] = (tau[c] - 1.0) * bracket + rho_b + dt * psi[c];
            }
        }
    }
    return ORACLE_OK;
}

/* ------------------------------------------------- FD4 / RK4 reference --- */
/*
 * The finite-difference reference solver of Sec. III (Results): the PDEs
 * Eqs. (EqSEIRD_S)-(EqSEIRD_D) written as
 *     d rho^C / dt = d^C lap(rho^C) + Psi^C(rho),
 * the Laplacian by fourth-order centred differences, time by the classic
 * fourth-order Runge-Kutta method, and the reactions evaluated explicitly at
 * every stage.
 * Readings (the paper names the orders but prints no stencil):
 *   - lap u = sum over the two axes of
 *       (-u(-2) + 16 u(-1) - 30 u(0) + 16 u(+1) - u(+2)) / (12 dx^2),
 *     the standard centred fourth-order second difference;
 *   - a no-flux wall takes ghost values by even reflection about the
 *     boundary face, u(-1) = u(0), u(-2) = u(1) (zero normal derivative, the
 *     mirror image used for the SSLBM); a periodic wall wraps;
 *   - the deceased diffuse only if d^D > 0 (otherwise their Laplacian term
 *     is multiplied by zero).
 * Parity: pinned by tests against the exact Runge-Kutta amplification of
 * every Fourier mode of pure diffusion, the textbook RK4 of the local ODE
 * without diffusion, the mirror extension, conservation of the total, and
 * the fourth-order convergence of the stencil.
 */

/* Index of lattice coordinate i along an axis of n nodes, ghosts included. */
static int fd4_fold(int i, int n, int bc)
{
    if (bc == BC_PERIODIC)
        return ((i % n) + n) % n;
    int period = 2 * n; /* the field and its mirror image */
    int m = ((i % period) + period) % period;
    return m < n ? m : period - 1 - m;
}

/* Right-hand side F(rho) of the semi-discrete system at every node. */
static void fd4_rhs(int nx, int ny, int bc, seird_rates k, const double *d, double dx,
                    const double *rho, double *F)
{
    size_t plane = (size_t)nx * ny;
    double h2 = 12.0 * dx * dx;
    for (int y = 0; y < ny; ++y) {
        for (int x = 0; x < nx; ++x) {
            size_t cell = (size_t)y * nx + x;
            double here[5], psi[5];
            for (int c = 0; c < 5; ++c)
                here[c] = rho[c * plane + cell];
            seird_sources(here, k, psi);
            for (int c = 0; c < 5; ++c) {
                const double *u = rho + c * plane;
                double along_x = -u[(size_t)y * nx + fd4_fold(x - 2, nx, bc)]
                                 + 16.0 * u[(size_t)y * nx + fd4_fold(x - 1, nx, bc)]
                                 - 30.0 * here[c]
                                 + 16.0 * u[(size_t)y * nx + fd4_fold(x + 1, nx, bc)]
                                 - u[(size_t)y * nx + fd4_fold(x + 2, nx, bc)];
                double along_y = -u[(size_t)fd4_fold(y - 2, ny, bc) * nx + x]
                                 + 16.0 * u[(size_t)fd4_fold(y - 1, ny, bc) * nx + x]
                                 - 30.0 * here[c]
                                 + 16.0 * u[(size_t)fd4_fold(y + 1, ny, bc) * nx + x]
                                 - u[(size_t)fd4_fold(y + 2, ny, bc) * nx + x];
                F[c * plane + cell] = d[c] * (along_x + along_y) / h2 + psi[c];
            }
        }
    }
}

/* nsteps steps of RK4 on the FD4 semi-discrete system, in place in rho. */
int oracle_fd4_rk4_run(int nx, int ny, int bc, const double *rates, const double *d,
                       double dx, double dt, double *rho, long long nsteps)
{
    if (!valid_grid(nx, ny, bc) || !rates || !d || !rho || nsteps < 0)
        return ORACLE_E_ARG;
    seird_rates k = unpack_rates(rates);
    size_t n = 5 * (size_t)nx * ny;
    double *k1 = malloc(sizeof(double) * n), *k2 = malloc(sizeof(double) * n);
    double *k3 = malloc(sizeof(double) * n), *k4 = malloc(sizeof(double) * n);
    double *stage = malloc(sizeof(double) * n);
    int rc = (k1 && k2 && k3 && k4 && stage) ? ORACLE_OK : ORACLE_E_ARG;
    for (long long step = 0; rc == ORACLE_OK && step < nsteps; ++step) {
        fd4_rhs(nx, ny, bc, k, d, dx, rho, k1);
        for (size_t i = 0; i < n; ++i)
            stage[i] = rho[i] + 0.5 * dt * k1[i];
        fd4_rhs(nx, ny, bc, k, d, dx, stage, k2);
        for (size_t i = 0; i < n; ++i)
            stage[i] = rho[i] + 0.5 * dt * k2[i];
        fd4_rhs(nx, ny, bc, k, d, dx, stage, k3);
        for (size_t i = 0; i < n; ++i)
            stage[i] = rho[i] + dt * k3[i];
        fd4_rhs(nx, ny, bc, k, d, dx, stage, k4);
        for (size_t i = 0; i < n; ++i)
            rho[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
    }
    free(k1);
    free(k2);
    free(k3);
    free(k4);
    free(stage);
    return rc;
}
