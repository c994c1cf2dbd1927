"""Checks that pin the oracle to what the paper and the mathematics fix.

Every function takes an ``oracle.Oracle`` (so the planted-mistake tests can run
the same checks against deliberately broken builds of the oracle) and raises
AssertionError when the oracle disagrees.
"""
from __future__ import annotations

import numpy as np

import references as ref
from paper_2603_19789_amd.inputs import Params, random_state

PURE_DIFFUSION = dict(beta=0.0, alpha=0.0, gamma=0.0, phi=0.0)


def _pure(d_lattice, dx=1.0, dt=1.0) -> Params:
    d = tuple(v * dx * dx / dt for v in d_lattice)
    return Params(d=d, dx=dx, dt=dt, **PURE_DIFFUSION)


def _tau(p, c):
    return 0.5 + 3.0 * ref.lattice_diffusivity(p, c)


# ------------------------------------------------------------ diffusion ----

def check_exact_discrete_diffusion(orc, nx=24, ny=20, nsteps=25, seed=11, tol=1e-13):
    """Psi = 0, periodic: the oracle equals G(k)^n mode by mode (Fourier
    analysis of Sec. II.C.2, G from the first line of Eq. G_exact)."""
    p = _pure((0.02, 0.11, 0.0, 0.2, 0.05))
    rho0 = random_state(nx, ny, seed)
    out = orc.sslbm_run(rho0, p, nsteps)
    for c in range(5):
        want = ref.exact_discrete_diffusion(rho0[c], _tau(p, c), nsteps)
        err = ref.rel_l2(out[c], want)
        assert err < tol, f"compartment {c}: exact-discrete error {err:.3e}"


def check_manufactured_eigenmode(orc, n=32, nsteps=40, d_lattice=0.05, tol=1e-13):
    """sin(2 pi x) sin(2 pi y) (Sec. III.B) is an exact eigenmode of the
    discrete scheme: after n steps it is G^n times the start."""
    x = np.arange(n) / n
    mode = np.outer(np.sin(2 * np.pi * x), np.sin(2 * np.pi * x))
    p = _pure((d_lattice,) * 5)
    rho0 = np.broadcast_to(mode, (5, n, n)).copy()
    out = orc.sslbm_run(rho0, p, nsteps)
    g = ref.sslbm_amplification(_tau(p, 0), 2 * np.pi / n, 2 * np.pi / n)
    err = ref.rel_l2(out[0], g ** nsteps * mode)
    assert err < tol, f"eigenmode error {err:.3e}"


def check_uniform_stays_uniform(orc, nx=9, ny=7, nsteps=30):
    """A spatially uniform state has zero stencil difference: every cell keeps
    the same value bit for bit (periodic and no-flux)."""
    p = Params(beta=0.7, alpha=0.3, gamma=0.2, phi=0.25,
               d=(0.5, 0.3, 0.2, 0.1, 0.0), dx=1.0, dt=0.05)
    rho0 = np.empty((5, ny, nx))
    for c, v in enumerate((0.9, 0.03, 0.05, 0.02, 0.0)):
        rho0[c] = v
    for bc in ("periodic", "noflux"):
        out = orc.sslbm_run(rho0, p, nsteps, bc=bc)
        for c in range(5):
            assert np.all(out[c] == out[c, 0, 0]), f"{bc}: compartment {c} not uniform"


# ----------------------------------------------------------- reactions -----

def check_zero_diffusion_is_euler(orc, nx=7, ny=5, nsteps=50, seed=3):
    """All d = 0 (tau = 1/2): the step reduces to forward Euler of the local
    SEIRD ODE, cell by cell (right-hand side taken from the PDE)."""
    p = Params(beta=0.9, alpha=0.25, gamma=0.15, phi=0.3, d=(0.0,) * 5, dx=1.0, dt=0.05)
    rho0 = random_state(nx, ny, seed)
    out = orc.sslbm_run(rho0, p, nsteps)
    want = ref.euler_ode(rho0, p, p.dt, nsteps)
    err = np.max(np.abs(out - want) / np.maximum(np.abs(want), 1e-300))
    assert err < 1e-13, f"zero-diffusion vs Euler: {err:.3e}"


def check_zero_diffusion_first_order(orc, seed=4):
    """Against RK4 at a step 250x below the finest one tried, the zero-diffusion
    scheme converges with order 1 in dt (the reaction is explicit Euler)."""
    p0 = Params(beta=0.9, alpha=0.25, gamma=0.15, phi=0.3, d=(0.0,) * 5, dx=1.0, dt=0.1)
    rho0 = random_state(3, 3, seed)
    T = 2.0
    truth = ref.rk4_ode(rho0, p0, T / 20000, 20000)
    errs = []
    for dt in (0.1, 0.05, 0.025):
        out = orc.sslbm_run(rho0, p0.with_(dt=dt), int(round(T / dt)))
        errs.append(np.linalg.norm(out - truth))
    slopes = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    for s in slopes:
        assert abs(s - 1.0) < 0.1, f"order in dt: {slopes}"


def check_dfe_growth_rate(orc):
    """Near the disease-free equilibrium the E-I perturbation grows per step by
    1 + dt lambda_1, lambda_1 from Eq. (eigenvalues); R0 = beta/gamma < 1 decays,
    R0 > 1 grows (Eq. R0_condition)."""
    for beta in (0.08, 0.5):
        p = Params(beta=beta, alpha=0.2, gamma=0.11, phi=0.1, d=(0.0,) * 5, dx=1.0, dt=0.01)
        rho0 = np.zeros((5, 3, 3))
        rho0[0], rho0[1], rho0[2] = 1.0, 1e-9, 1e-9
        n = 6000
        a = orc.sslbm_run(rho0, p, n)
        b = orc.sslbm_step(a, p)
        rate = b[2, 1, 1] / a[2, 1, 1]
        lam1, _ = ref.dfe_eigenvalues(p)
        want = 1.0 + p.dt * lam1
        assert abs(rate - want) < 1e-6 * abs(want), f"beta={beta}: {rate} vs {want}"
        assert (rate < 1.0) == (beta / p.gamma < 1.0)


def check_jacobi_superposition(orc, nx=11, ny=9, seed=5):
    """Every term of Eq. (sslbm_final_clean) is evaluated at time t, so one step
    equals (diffusion-only step) + (reaction-only step) - rho, to rounding."""
    full = Params(beta=0.8, alpha=0.3, gamma=0.2, phi=0.2,
                  d=(0.9, 0.6, 0.3, 0.45, 0.0), dx=1.0, dt=0.1)
    diff_only = full.with_(beta=0.0, alpha=0.0, gamma=0.0, phi=0.0)
    react_only = full.with_(d=(0.0,) * 5)
    rho0 = random_state(nx, ny, seed)
    for bc in ("periodic", "noflux"):
        a = orc.sslbm_step(rho0, full, bc=bc)
        b = orc.sslbm_step(rho0, diff_only, bc=bc) + orc.sslbm_step(rho0, react_only, bc=bc) - rho0
        err = np.max(np.abs(a - b))
        assert err < 1e-15, f"{bc}: superposition error {err:.3e}"


# --------------------------------------------------------- conservation ----

def check_conservation(orc, nx=13, ny=10, nsteps=60, seed=6, tol=1e-14):
    """Eq. (mass_conservation): total population is constant, periodic and
    no-flux; with Psi = 0 every compartment is conserved on its own."""
    p = Params(beta=1.2, alpha=0.3, gamma=0.25, phi=0.3,
               d=(1.0, 0.5, 0.2, 0.8, 0.0), dx=1.0, dt=0.1)
    rho0 = random_state(nx, ny, seed)
    total0 = rho0.sum()
    for bc in ("periodic", "noflux"):
        out = orc.sslbm_run(rho0, p, nsteps, bc=bc)
        drift = abs(out.sum() - total0) / total0
        assert drift < tol, f"{bc}: total drift {drift:.3e}"
        outp = orc.sslbm_run(rho0, p.with_(beta=0.0, alpha=0.0, gamma=0.0, phi=0.0),
                             nsteps, bc=bc)
        for c in range(5):
            dc = abs(outp[c].sum() - rho0[c].sum()) / rho0[c].sum()
            assert dc < tol, f"{bc}: compartment {c} drift {dc:.3e}"


def check_recovered_deceased_proportional(orc, nx=12, ny=10, seed=7):
    """With R and D diffusing alike and starting at zero, Eqs. (EqSEIRD_R),
    (EqSEIRD_D) give phi R = (1 - phi) D at every step and node."""
    rho0 = random_state(nx, ny, seed)
    rho0[3] = 0.0
    rho0[4] = 0.0
    for dRD in (0.0, 0.4):
        p = Params(beta=0.9, alpha=0.3, gamma=0.2, phi=0.3,
                   d=(0.5, 0.4, 0.1, dRD, dRD), dx=1.0, dt=0.1)
        for bc in ("periodic", "noflux"):
            out = orc.sslbm_run(rho0, p, 40, bc=bc)
            x = p.phi * out[3] - (1 - p.phi) * out[4]
            scale = np.max(np.abs(out[4]))
            assert scale > 0 and np.max(np.abs(x)) < 1e-14 * max(scale, 1.0), (
                f"d={dRD} {bc}: max |phi R - (1-phi) D| = {np.max(np.abs(x)):.3e}")


def check_noflux_is_reflection(orc, nx=10, ny=7, nsteps=15, seed=8):
    """No-flux (zero difference across the wall) equals the periodic scheme on
    the domain mirrored about both walls: the mirrored field stays mirrored."""
    p = Params(beta=0.8, alpha=0.3, gamma=0.2, phi=0.2,
               d=(0.9, 0.6, 0.3, 0.45, 0.0), dx=1.0, dt=0.1)
    rho0 = random_state(nx, ny, seed)
    mirrored = np.concatenate([rho0, rho0[:, :, ::-1]], axis=2)
    mirrored = np.concatenate([mirrored, mirrored[:, ::-1, :]], axis=1)
    a = orc.sslbm_run(rho0, p, nsteps, bc="noflux")
    b = orc.sslbm_run(mirrored, p, nsteps, bc="periodic")[:, :ny, :nx]
    assert np.max(np.abs(a - b)) < 1e-15


def check_empty_cells(orc, nx=14, ny=11, nsteps=60, seed=13):
    """Cells with no contact-eligible population (S = E = I = R = 0; N_c of
    Eq. (sources) leaves out D) have no force of infection (reading: F = 0
    where N_c <= 0) and, with E = I = 0, no source at all. So
    (1) a state of such cells with resting D stays fixed bit for bit;
    (2) one step of a state with a block of them is, on the block, one step of
        pure diffusion (the FFT solution of Eq. G_exact, periodic);
    (3) a long run from it, periodic and no-flux, stays finite and conserves
        the total (Eq. mass_conservation)."""
    p = Params(beta=0.9, alpha=0.3, gamma=0.2, phi=0.3,
               d=(0.9, 0.6, 0.3, 0.45, 0.0), dx=1.0, dt=0.1)
    rng = np.random.default_rng(seed)
    empty = np.zeros((5, ny, nx))
    empty[4] = rng.uniform(0.1, 1.0, size=(ny, nx))
    for bc in ("periodic", "noflux"):
        out = orc.sslbm_run(empty, p, 5, bc=bc)
        assert np.array_equal(out, empty), f"{bc}: an empty state moved"
    rho0 = random_state(nx, ny, seed)
    block = (slice(3, 8), slice(4, 10))
    rho0[(slice(0, 4),) + block] = 0.0
    one = orc.sslbm_step(rho0, p)
    assert np.all(np.isfinite(one)), "non-finite values next to empty cells"
    for c in range(5):
        want = ref.exact_discrete_diffusion(rho0[c], _tau(p, c), 1)
        err = np.max(np.abs(one[c][block] - want[block]))
        assert err < 1e-15, f"compartment {c}: empty-block step {err:.3e} from pure diffusion"
    total0 = rho0.sum()
    for bc in ("periodic", "noflux"):
        out = orc.sslbm_run(rho0, p, nsteps, bc=bc)
        assert np.all(np.isfinite(out)), f"{bc}: non-finite values after {nsteps} steps"
        drift = abs(out.sum() - total0) / total0
        assert drift < 1e-14, f"{bc}: total drift {drift:.3e} with empty cells"


# ------------------------------------------------------------------ BGK ----

def check_bgk_exact_discrete(orc, nx=16, ny=12, nsteps=20, seed=9, tol=1e-12):
    """Psi = 0, periodic, equilibrium start: oracle BGK equals the mode-by-mode
    solution of Eq. (pdf)."""
    p = _pure((0.02, 0.11, 0.3, 0.2, 0.0))
    rho0 = random_state(nx, ny, seed)
    out = orc.bgk_run_density(rho0, p, nsteps)
    for c in range(4):
        want = ref.bgk_exact_discrete(rho0[c], _tau(p, c), nsteps)
        err = ref.rel_l2(out[c], want)
        assert err < tol, f"compartment {c}: BGK exact-discrete error {err:.3e}"
    assert np.array_equal(out[4], rho0[4])


def check_bgk_conservation(orc, nx=11, ny=9, nsteps=40, seed=10, tol=1e-14):
    p = Params(beta=1.2, alpha=0.3, gamma=0.25, phi=0.3,
               d=(1.0, 0.5, 0.2, 0.8, 0.0), dx=1.0, dt=0.1)
    rho0 = random_state(nx, ny, seed)
    for bc in ("periodic", "noflux"):
        out = orc.bgk_run_density(rho0, p, nsteps, bc=bc)
        drift = abs(out.sum() - rho0.sum()) / rho0.sum()
        assert drift < tol, f"BGK {bc}: drift {drift:.3e}"
        outp = orc.bgk_run_density(rho0, p.with_(beta=0.0, alpha=0.0, gamma=0.0, phi=0.0),
                                   nsteps, bc=bc)
        for c in range(4):
            dc = abs(outp[c].sum() - rho0[c].sum()) / rho0[c].sum()
            assert dc < tol, f"BGK {bc}: compartment {c} drift {dc:.3e}"


def check_bgk_uniform_is_euler(orc, nsteps=40):
    """Uniform state, equilibrium start: collision leaves f = w_i (rho + Psi dt)
    and streaming moves nothing, so BGK is forward Euler of the local ODE."""
    p = Params(beta=0.9, alpha=0.25, gamma=0.15, phi=0.3,
               d=(0.7, 0.4, 0.2, 0.3, 0.0), dx=1.0, dt=0.05)
    rho0 = np.empty((5, 4, 5))
    for c, v in enumerate((0.8, 0.05, 0.1, 0.03, 0.02)):
        rho0[c] = v
    want = ref.euler_ode(rho0[:, 0, 0], p, p.dt, nsteps)
    for bc in ("periodic", "noflux"):
        out = orc.bgk_run_density(rho0, p, nsteps, bc=bc)
        err = np.max(np.abs(out - want[:, None, None]) / np.abs(want)[:, None, None])
        assert err < 1e-13, f"BGK {bc} uniform vs Euler: {err:.3e}"


def check_bgk_tau_one_matches_sslbm(orc, nx=10, ny=8, nsteps=12, seed=12):
    """At tau = 1 the BGK collision returns f to equilibrium, so pure-diffusion
    BGK is rho(t+1) = sum_i w_i rho(x - c_i), which is the SSLBM at tau = 1."""
    p = _pure((1 / 6,) * 4 + (0.0,))
    rho0 = random_state(nx, ny, seed)
    for bc in ("periodic", "noflux"):
        a = orc.bgk_run_density(rho0, p, nsteps, bc=bc)
        b = orc.sslbm_run(rho0, p, nsteps, bc=bc)
        assert np.max(np.abs(a - b)) < 1e-14, bc


def check_bgk_empty_cells(orc, nx=12, ny=9, nsteps=40, seed=14):
    """BGK with a block of cells without contact-eligible population: the
    shared source has F = 0 there, so the run stays finite and conserves the
    total (both walls), and a state made only of such cells stays fixed."""
    p = Params(beta=0.9, alpha=0.3, gamma=0.2, phi=0.3,
               d=(0.9, 0.6, 0.3, 0.45, 0.0), dx=1.0, dt=0.1)
    rho0 = random_state(nx, ny, seed)
    rho0[:4, 2:7, 3:9] = 0.0
    for bc in ("periodic", "noflux"):
        out = orc.bgk_run_density(rho0, p, nsteps, bc=bc)
        assert np.all(np.isfinite(out)), f"BGK {bc}: non-finite values"
        drift = abs(out.sum() - rho0.sum()) / rho0.sum()
        assert drift < 1e-14, f"BGK {bc}: drift {drift:.3e} with empty cells"
    empty = np.zeros((5, ny, nx))
    empty[4] = 0.5
    out = orc.bgk_run_density(empty, p, 5)
    assert np.array_equal(out, empty), "BGK: an empty state moved"


FAST_SSLBM_CHECKS = (
    check_exact_discrete_diffusion, check_manufactured_eigenmode, check_uniform_stays_uniform,
    check_zero_diffusion_is_euler, check_dfe_growth_rate, check_jacobi_superposition,
    check_conservation, check_recovered_deceased_proportional, check_noflux_is_reflection,
    check_empty_cells,
)
FAST_BGK_CHECKS = (
    check_bgk_exact_discrete, check_bgk_conservation, check_bgk_uniform_is_euler,
    check_bgk_tau_one_matches_sslbm, check_bgk_empty_cells,
)
