"""Checks that pin the oracle's adjoint (reverse) step to the forward step.

The adjoint of one step is the transpose of the step's Jacobian applied to
dJ/d rho(t+dt), plus the step's partial derivatives with respect to the rates
and diffusivities. Each check ties it to something the oracle's adjoint does
not compute itself: the forward oracle (already pinned to the paper) through
exact linear identities or central finite differences.

Every function takes an ``oracle.Oracle`` and raises AssertionError on a
mismatch, so the planted-mistake tests can reuse them.
"""
from __future__ import annotations

import numpy as np

from paper_2603_19789_amd.inputs import Params, random_state

PARAM_NAMES = ("beta", "alpha", "gamma", "phi", "d_S", "d_E", "d_I", "d_R", "d_D")


def _params(seed: int, beta: float = 0.9, d_dead: float = 0.07, dt: float = 0.1) -> Params:
    """Rates of order one and lattice diffusivities in (0.03, 0.2), so every
    term of the step is visible in a few steps on a small grid."""
    rng = np.random.default_rng(seed)
    d_lattice = list(rng.uniform(0.03, 0.2, size=4)) + [d_dead]
    dx = 0.5
    d = tuple(v * dx * dx / dt for v in d_lattice)
    return Params(beta=beta, alpha=float(rng.uniform(0.3, 1.2)), gamma=float(rng.uniform(0.3, 1.2)),
                  phi=float(rng.uniform(0.1, 0.6)), d=d, dx=dx, dt=dt)


def _vector(p: Params) -> np.ndarray:
    return np.array([p.beta, p.alpha, p.gamma, p.phi, *p.d])


def _from_vector(p: Params, v: np.ndarray) -> Params:
    return p.with_(beta=float(v[0]), alpha=float(v[1]), gamma=float(v[2]), phi=float(v[3]),
                   d=tuple(float(x) for x in v[4:]))


def _objective(orc, rho0, p, nsteps, weight, bc):
    return float(np.sum(weight * orc.sslbm_run(rho0, p, nsteps, bc=bc)))


def check_adjoint_is_transpose_when_linear(orc, nx=9, ny=7, seed=21):
    """With beta = 0 the force of infection vanishes and one step is a linear
    map A (transport plus the linear E, I, R, D sources), so the adjoint must
    satisfy <lam, A rho> = <A^T lam, rho> for every pair; this fixes every
    transport weight, boundary rule and linear source term."""
    for bc in ("periodic", "noflux"):
        for d_dead in (0.07, 0.0):
            p = _params(seed, beta=0.0, d_dead=d_dead)
            rng = np.random.default_rng(seed + (bc == "noflux") + 10 * (d_dead == 0.0))
            for _ in range(3):
                rho = rng.normal(size=(5, ny, nx))
                lam = rng.normal(size=(5, ny, nx))
                left = float(np.sum(lam * orc.sslbm_step(rho, p, bc=bc)))
                back, _ = orc.sslbm_adjoint_step(rho, lam, p, bc=bc)
                right = float(np.sum(back * rho))
                scale = float(np.sum(np.abs(lam)) * np.max(np.abs(rho)))
                assert abs(left - right) <= 1e-13 * scale, (bc, d_dead, left, right)


def check_adjoint_of_pure_diffusion_is_the_step(orc, nx=10, ny=8, seed=22):
    """With every rate zero the step is the five-point diffusion update, a
    symmetric operator on periodic and no-flux (mirror) grids, so the adjoint
    step applied to lam equals the forward step applied to lam."""
    for bc in ("periodic", "noflux"):
        p = _params(seed).with_(beta=0.0, alpha=0.0, gamma=0.0, phi=0.0)
        lam = np.random.default_rng(seed).normal(size=(5, ny, nx))
        back, grad = orc.sslbm_adjoint_step(np.ones((5, ny, nx)), lam, p, bc=bc)
        want = orc.sslbm_step(lam, p, bc=bc)
        assert np.max(np.abs(back - want)) < 1e-14, bc
        # a uniform state has no Laplacian: no diffusivity gradient
        assert np.max(np.abs(grad[4:])) < 1e-13, (bc, grad)


def _directional_fd(orc, rho0, p, nsteps, weight, bc, direction, h):
    plus = _objective(orc, rho0 + h * direction, p, nsteps, weight, bc)
    minus = _objective(orc, rho0 - h * direction, p, nsteps, weight, bc)
    return (plus - minus) / (2.0 * h)


def check_adjoint_state_gradient_fd(orc, nx=8, ny=6, nsteps=4, seed=23):
    """Nonlinear run: dJ/d rho(0) from the reverse sweep against central
    differences of the forward oracle along random directions, for
    J = <w, rho(n)>."""
    for bc in ("periodic", "noflux"):
        p = _params(seed)
        rng = np.random.default_rng(seed + 5 * (bc == "noflux"))
        rho0 = random_state(nx, ny, seed, infected_scale=0.4)
        weight = rng.normal(size=rho0.shape)
        lam0, _ = orc.sslbm_adjoint_run(rho0, p, nsteps, weight, bc=bc)
        for _ in range(4):
            v = rng.normal(size=rho0.shape)
            fd = _directional_fd(orc, rho0, p, nsteps, weight, bc, v, 1e-6)
            got = float(np.sum(lam0 * v))
            assert abs(got - fd) <= 1e-7 * max(1.0, abs(fd)), (bc, got, fd)


def check_adjoint_parameter_gradient_fd(orc, nx=8, ny=6, nsteps=5, seed=24):
    """dJ/d(beta, alpha, gamma, phi, d^S..d^D) from the reverse sweep against
    central differences of the forward oracle (relative step 1e-6)."""
    for bc in ("periodic", "noflux"):
        p = _params(seed)
        rng = np.random.default_rng(seed + 7 * (bc == "noflux"))
        rho0 = random_state(nx, ny, seed, infected_scale=0.4)
        weight = rng.normal(size=rho0.shape)
        _, grad = orc.sslbm_adjoint_run(rho0, p, nsteps, weight, bc=bc)
        base = _vector(p)
        for j, name in enumerate(PARAM_NAMES):
            h = 1e-6 * abs(base[j])
            up, down = base.copy(), base.copy()
            up[j] += h
            down[j] -= h
            fd = (_objective(orc, rho0, _from_vector(p, up), nsteps, weight, bc)
                  - _objective(orc, rho0, _from_vector(p, down), nsteps, weight, bc)) / (2 * h)
            assert abs(grad[j] - fd) <= 1e-6 * max(1.0, abs(fd)), (bc, name, grad[j], fd)


def check_adjoint_resting_deceased_gradient(orc, nx=8, ny=6, nsteps=5, seed=25):
    """At d^D = 0 the deceased do not move, and the diffusivity gradient of D
    is the one-sided derivative: checked by the second-order one-sided
    difference (-3 J(0) + 4 J(h) - J(2h)) / (2h)."""
    for bc in ("periodic", "noflux"):
        p = _params(seed, d_dead=0.0)
        rng = np.random.default_rng(seed)
        rho0 = random_state(nx, ny, seed, infected_scale=0.4)
        rho0[4] = rng.uniform(0.0, 0.5, size=(ny, nx))  # a rough D field
        weight = rng.normal(size=rho0.shape)
        _, grad = orc.sslbm_adjoint_run(rho0, p, nsteps, weight, bc=bc)
        h = 1e-5
        j = [_objective(orc, rho0, p.with_(d=p.d[:4] + (s * h,)), nsteps, weight, bc)
             for s in (0, 1, 2)]
        fd = (-3 * j[0] + 4 * j[1] - j[2]) / (2 * h)
        assert abs(grad[8] - fd) <= 1e-6 * max(1.0, abs(fd)), (bc, grad[8], fd)


FAST_ADJOINT_CHECKS = (
    check_adjoint_is_transpose_when_linear, check_adjoint_of_pure_diffusion_is_the_step,
    check_adjoint_state_gradient_fd, check_adjoint_parameter_gradient_fd,
    check_adjoint_resting_deceased_gradient,
)
