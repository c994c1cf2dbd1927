"""Checks that pin the oracle's finite-difference reference solver (Sec. III:
fourth-order centred differences in space, classic RK4 in time, reactions
explicit at every stage) to what the mathematics fixes. Each function takes
an ``oracle.Oracle`` and raises AssertionError on a mismatch."""
from __future__ import annotations

import numpy as np

import references as ref
from paper_2603_19789_amd.inputs import Params, random_state

NO_REACTIONS = dict(beta=0.0, alpha=0.0, gamma=0.0, phi=0.0)


def rk4_amplification(z):
    """The classic RK4 step applied to u' = lambda u multiplies u by
    R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24, z = dt lambda (its stability
    polynomial, textbook)."""
    return 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24


def check_pure_diffusion_fourier(orc, nx=12, ny=10, nsteps=9, seed=41):
    """Pure diffusion on a periodic grid: every Fourier mode of every
    compartment evolves on its own, multiplied per step by the RK4 polynomial
    of dt d times the stencil's eigenvalue. The eigenvalue of the centred
    fourth-order second difference on exp(i k x) is
    (-2 cos 2k + 32 cos k - 30) / (12 dx^2) per axis. Checks the stage
    structure and weights of RK4 and the indexing of the stencil."""
    d = (0.9, 0.5, 0.3, 0.7, 0.2)
    p = Params(d=d, dx=1.3, dt=0.07, **NO_REACTIONS)
    rho = random_state(nx, ny, seed)
    got = orc.fd4_rk4_run(rho, p, nsteps)
    kx = 2 * np.pi * np.fft.fftfreq(nx)[None, :]
    ky = 2 * np.pi * np.fft.fftfreq(ny)[:, None]
    eig = ((-2 * np.cos(2 * kx) + 32 * np.cos(kx) - 30)
           + (-2 * np.cos(2 * ky) + 32 * np.cos(ky) - 30)) / (12 * p.dx ** 2)
    for c in range(5):
        want = np.fft.ifft2(np.fft.fft2(rho[c]) * rk4_amplification(p.dt * d[c] * eig) ** nsteps)
        assert np.max(np.abs(want.imag)) < 1e-12
        err = np.max(np.abs(got[c] - want.real))
        assert err < 1e-12, (c, err)


def check_reaction_limit_is_rk4_ode(orc, nx=6, ny=5, nsteps=15, seed=43):
    """Without diffusion every node follows the textbook RK4 of the local
    SEIRD ODE, Eqs. (EqSEIRD_S)-(EqSEIRD_D), on both walls."""
    p = Params(beta=0.9, alpha=0.35, gamma=0.25, phi=0.2, d=(0.0,) * 5, dx=1.0, dt=0.2)
    rho = random_state(nx, ny, seed, infected_scale=0.4)
    want = ref.rk4_ode(rho, p, p.dt, nsteps)
    for bc in ("periodic", "noflux"):
        got = orc.fd4_rk4_run(rho, p, nsteps, bc=bc)
        err = np.max(np.abs(got - want))
        assert err < 1e-14, (bc, err)


def _mirror_extension(rho):
    """The field and its mirror images about the right and top faces: a
    periodic field of twice the size whose symmetry makes the normal
    derivative vanish on the original walls."""
    wide = np.concatenate([rho, rho[:, :, ::-1]], axis=2)
    return np.concatenate([wide, wide[:, ::-1, :]], axis=1)


def check_noflux_is_mirror_extension(orc, seed=47):
    """No-flux walls by even reflection: the run equals a periodic run on the
    field extended by its mirror images, restricted to the original grid
    (odd, tiny and one-row grids included)."""
    p = Params(beta=0.6, alpha=0.3, gamma=0.2, phi=0.1, d=(1.2, 0.7, 0.4, 0.9, 0.3), dx=1.0,
               dt=0.05)
    for nx, ny in ((7, 5), (2, 3), (1, 4), (9, 1)):
        rho = random_state(nx, ny, seed + nx)
        got = orc.fd4_rk4_run(rho, p, 6, bc="noflux")
        want = orc.fd4_rk4_run(_mirror_extension(rho), p, 6, bc="periodic")[:, :ny, :nx]
        err = np.max(np.abs(got - want))
        assert err < 1e-15, ((nx, ny), err)


def check_total_population_conserved(orc, nx=9, ny=8, nsteps=40, seed=53):
    """The sources only move people between compartments and the centred
    stencil sums to zero over a periodic grid or a grid with even-reflection
    walls, so the total population stays constant (Eq. (mass_conservation))."""
    p = Params(beta=0.8, alpha=0.3, gamma=0.25, phi=0.3, d=(1.1, 0.6, 0.2, 0.8, 0.0), dx=1.0,
               dt=0.05)
    rho = random_state(nx, ny, seed)
    total = rho.sum()
    for bc in ("periodic", "noflux"):
        got = orc.fd4_rk4_run(rho, p, nsteps, bc=bc)
        drift = abs(got.sum() - total) / total
        assert drift < 1e-14, (bc, drift)


def check_fourth_order_in_space(orc):
    """Pure diffusion of u = 1 + sin(2 pi x) cos(2 pi y) / 2 on the periodic
    unit square, to t = 0.01 with d = 1: against the continuum solution
    1 + exp(-8 pi^2 t) sin cos / 2, the error falls 16-fold per halving of dx
    (time steps of 0.02 dx^2 keep the RK4 error far below it)."""
    errs = []
    for n in (8, 16, 32):
        dx = 1.0 / n
        steps = int(np.ceil(0.01 / (0.02 * dx * dx)))
        dt = 0.01 / steps
        p = Params(d=(1.0, 0.0, 0.0, 0.0, 0.0), dx=dx, dt=dt, **NO_REACTIONS)
        x = np.arange(n) * dx
        shape = np.sin(2 * np.pi * x)[None, :] * np.cos(2 * np.pi * x)[:, None]
        rho = np.zeros((5, n, n))
        rho[0] = 1.0 + 0.5 * shape
        got = orc.fd4_rk4_run(rho, p, steps)[0]
        want = 1.0 + 0.5 * np.exp(-8 * np.pi ** 2 * 0.01) * shape
        errs.append(np.max(np.abs(got - want)))
    ratios = [errs[i] / errs[i + 1] for i in range(2)]
    assert all(14.0 < r < 18.0 for r in ratios), (errs, ratios)


def check_matches_numpy_reference(orc, seed=59):
    """The independent NumPy solver of the test references (array padding
    instead of index folding, whole-array RK4 stages) gives the same states
    on both walls."""
    p = Params(beta=0.7, alpha=0.3, gamma=0.2, phi=0.15, d=(0.8, 0.5, 0.1, 0.6, 0.0), dx=1.0,
               dt=0.05)
    rho = random_state(10, 7, seed)
    for bc in ("periodic", "noflux"):
        got = orc.fd4_rk4_run(rho, p, 12, bc=bc)
        want = ref.fd4_rk4_run(rho, p, 12, bc=bc)
        err = np.max(np.abs(got - want))
        assert err < 1e-13, (bc, err)


FAST_FD4_CHECKS = (
    check_pure_diffusion_fourier, check_reaction_limit_is_rk4_ode,
    check_noflux_is_mirror_extension, check_total_population_conserved,
    check_fourth_order_in_space, check_matches_numpy_reference,
)
