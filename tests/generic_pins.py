"""Checks that pin the oracle's generic compartmental step (Eq. (generic_pde)
on D2Q5 and D2Q9) to what the paper and the mathematics fix. Each function
takes an ``oracle.Oracle`` and raises AssertionError on a mismatch."""
from __future__ import annotations

import numpy as np

import references as ref
from paper_2603_19789_amd.inputs import GenericModel, Params, random_state

D2Q9_LINKS = [(0, 0, 4 / 9)] + [(cx, cy, 1 / 9) for cx, cy in ((1, 0), (0, 1), (-1, 0), (0, -1))] \
    + [(cx, cy, 1 / 36) for cx, cy in ((1, 1), (-1, 1), (-1, -1), (1, -1))]


def d2q9_symbol(kx, ky):
    """Lambda(k) = sum_i w_i exp(i k.c_i) on D2Q9 (rest 4/9, axes 1/9,
    diagonals 1/36): 4/9 + (2/9)(cos kx + cos ky) + (1/9) cos kx cos ky."""
    return 4 / 9 + (2 / 9) * (np.cos(kx) + np.cos(ky)) + (1 / 9) * np.cos(kx) * np.cos(ky)


def seird_as_transitions(p: Params, lattice=5) -> GenericModel:
    """The SEIRD sources of Eq. (sources) and Eq. (rhoD) as transitions."""
    S, E, I, R, D = range(5)
    t = ((S, E, I, p.beta, 1), (E, I, -1, p.alpha, 0), (I, R, -1, (1 - p.phi) * p.gamma, 0),
         (I, D, -1, p.phi * p.gamma, 0))
    return GenericModel(("S", "E", "I", "R", "D"), p.d, t, (1, 1, 1, 1, 0), lattice, p.dx, p.dt)


def check_seird_special_case(orc, nx=11, ny=9, seed=31):
    """SEIRD written as transitions on D2Q5 reproduces the SEIRD oracle step
    (itself pinned to the paper) on random states, both walls, D at rest and
    diffusing."""
    for d4 in (0.0, 0.9):
        p = Params(beta=0.8, alpha=0.4, gamma=0.3, phi=0.25, d=(2.0, 1.1, 0.4, 1.6, d4), dx=1.0,
                   dt=0.05)
        rho = random_state(nx, ny, seed, infected_scale=0.4)
        for bc in ("periodic", "noflux"):
            a = orc.generic_step(rho, seird_as_transitions(p), bc=bc)
            b = orc.sslbm_step(rho, p, bc=bc)
            assert np.max(np.abs(a - b)) < 1e-15, (bc, d4, np.max(np.abs(a - b)))


def check_d2q9_exact_discrete(orc, nx=20, ny=16, nsteps=15, seed=32, tol=1e-13):
    """Psi = 0, periodic, D2Q9: mode by mode G(k)^n with
    G = 1 - (2 tau - 1)(1 - Lambda_9(k)), Lambda_9 from the link sum."""
    d_lu = (0.03, 0.11, 0.3, 0.0)
    m = GenericModel(("a", "b", "c", "d"), tuple(v * 1.0 / 1.0 for v in d_lu), (), (1, 1, 1, 1),
                     9, 1.0, 1.0)
    rho0 = random_state(nx, ny, seed)[:4]
    out = orc.generic_run(rho0, m, nsteps)
    kx, ky = ref.wavenumbers(nx, ny)
    for c in range(4):
        g = 1.0 - 6.0 * d_lu[c] * (1.0 - d2q9_symbol(kx, ky))
        want = np.real(np.fft.ifft2(np.fft.fft2(rho0[c]) * g ** nsteps))
        err = ref.rel_l2(out[c], want)
        assert err < tol, (c, err)


def check_d2q9_symbol_reading():
    """The D2Q9 symbol must equal 1 at k = 0 (mass) and expand as
    |k|^2/6 - |k|^4/72 with no k_x^2 k_y^2 term (isotropy to fourth order,
    the property the anisotropy paragraph states). The link sum has both; the
    printed formula (1/9 on the axes, 1/36 on the diagonal cosines, i.e. the
    weights without the factor 2 of the +/- pair) gives Lambda(0) = 13/18."""
    assert abs(d2q9_symbol(0.0, 0.0) - 1.0) < 1e-15
    link = lambda kx, ky: sum(w * np.cos(kx * cx + ky * cy) for cx, cy, w in D2Q9_LINKS)
    for kx, ky in ((0.3, -1.1), (2.0, 0.7), (np.pi, np.pi)):
        assert abs(link(kx, ky) - d2q9_symbol(kx, ky)) < 1e-15
    printed = lambda kx, ky: 4 / 9 + (np.cos(kx) + np.cos(ky)) / 9 + (np.cos(kx + ky) + np.cos(kx - ky)) / 36
    assert abs(printed(0.0, 0.0) - 13 / 18) < 1e-15
    for r in (1e-2, 2e-2):
        for th in np.linspace(0, np.pi / 2, 7):
            kx, ky = r * np.cos(th), r * np.sin(th)
            rem = 1 - d2q9_symbol(kx, ky) - r ** 2 / 6 + r ** 4 / 72
            assert abs(rem) < 1e-3 * r ** 4, (r, th, rem)  # only O(|k|^6) is left


def check_linear_transition_closed_form(orc, nsteps=40):
    """One transition A -> B at rate k, no diffusion: forward Euler gives
    A_n = A_0 (1 - k dt)^n exactly and B_n = A_0 + B_0 - A_n."""
    m = GenericModel(("A", "B"), (0.0, 0.0), ((0, 1, -1, 0.7, 0),), (1, 1), 9, 1.0, 0.05)
    rho0 = np.stack([np.full((3, 4), 2.0), np.full((3, 4), 0.5)])
    out = orc.generic_run(rho0, m, nsteps)
    a = 2.0 * (1 - 0.7 * 0.05) ** nsteps
    assert np.max(np.abs(out[0] - a)) < 1e-13 and np.max(np.abs(out[1] - (2.5 - a))) < 1e-13


def check_generic_conservation(orc, nx=12, ny=10, nsteps=30, seed=33):
    """Transitions that stay inside the system conserve the total on both
    lattices and walls; a sink removes exactly its flow."""
    from paper_2603_19789_amd.inputs import seirvd_model, seirvd_state
    rho0 = seirvd_state(nx, ny, seed, foci=3)
    for lattice in (5, 9):
        m = seirvd_model(lattice=lattice, dt=0.05)
        for bc in ("periodic", "noflux"):
            out = orc.generic_run(rho0, m, nsteps, bc=bc)
            assert abs(out.sum() - rho0.sum()) < 1e-12 * rho0.sum(), (lattice, bc)
    sink = GenericModel(("A",), (0.5,), ((0, -1, -1, 0.2, 0),), (1,), 9, 1.0, 0.1)
    a0 = random_state(nx, ny, seed)[:1]
    out = orc.generic_step(a0, sink)
    assert abs(out.sum() - a0.sum() * (1 - 0.02)) < 1e-12 * a0.sum()


def check_d2q9_noflux_is_reflection(orc, nx=9, ny=7, nsteps=6, seed=34):
    """No-flux D2Q9 equals the periodic run of the mirror-extended field
    (the reflection about both walls, a 2nx x 2ny periodic grid)."""
    from paper_2603_19789_amd.inputs import seirvd_model
    m = seirvd_model(lattice=9, dt=0.05)
    rho0 = random_state(nx, ny, seed)
    rho0 = np.concatenate([rho0, rho0[:1] * 0.1], axis=0)  # six compartments
    ext = np.concatenate([rho0, rho0[:, :, ::-1]], axis=2)
    ext = np.concatenate([ext, ext[:, ::-1, :]], axis=1)
    a = orc.generic_run(rho0, m, nsteps, bc="noflux")
    b = orc.generic_run(ext, m, nsteps, bc="periodic")[:, :ny, :nx]
    assert np.max(np.abs(a - b)) < 1e-14


FAST_GENERIC_CHECKS = (
    check_seird_special_case, check_d2q9_exact_discrete, check_linear_transition_closed_form,
    check_generic_conservation, check_d2q9_noflux_is_reflection,
)
