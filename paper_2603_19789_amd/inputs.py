"""Seeded synthetic inputs: parameter sets and initial states.

This module holds no arithmetic of the method: it only draws and lays out
inputs (densities, rates, diffusivities) that both the HIP path and the CPU
oracle consume. Densities are NumPy float64 arrays of shape (5, ny, nx) in the
compartment order S, E, I, R, D with x fastest.

Rates follow the paper's notation (Sec. II.A, Table "Table_params"): beta, alpha,
gamma, phi. Workloads are often quoted with the other common naming (beta,
sigma, gamma, mu) where E leaves at rate sigma, I recovers at rate gamma and
dies at rate mu. The two are the same model with alpha = sigma,
gamma_paper = gamma + mu and phi = mu / (gamma + mu); ``from_sigma_mu`` does the
conversion.

Diffusivities ``d`` are physical (length^2/time). Workloads are usually quoted
in lattice units d_lu = d dt / dx^2; ``lattice_to_physical`` converts.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

COMPARTMENTS = ("S", "E", "I", "R", "D")


@dataclass(frozen=True)
class Params:
    beta: float
    alpha: float
    gamma: float
    phi: float
    d: tuple = (0.0, 0.0, 0.0, 0.0, 0.0)
    dx: float = 1.0
    dt: float = 0.01

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)


def lattice_to_physical(d_lattice, dx: float, dt: float) -> tuple:
    """Physical diffusivities for lattice-unit values d_lu = d dt / dx^2."""
    return tuple(float(v) * dx * dx / dt for v in d_lattice)


def from_sigma_mu(beta, sigma, gamma, mu, d_lattice, dx=1.0, dt=0.01) -> Params:
    """Parameters from the (beta, sigma, gamma, mu) naming and lattice diffusivities."""
    return Params(beta=float(beta), alpha=float(sigma), gamma=float(gamma + mu),
                  phi=float(mu / (gamma + mu)), d=lattice_to_physical(d_lattice, dx, dt),
                  dx=float(dx), dt=float(dt))


# ----------------------------------------------------------------- states --

def _min_image_sq(n: int, centre: float) -> np.ndarray:
    """Squared periodic minimum-image distance of cells 0..n-1 to ``centre``."""
    delta = np.abs(np.arange(n, dtype=np.float64) - centre)
    delta = np.minimum(delta, n - delta)
    return delta * delta


def gaussian_foci_state(nx: int, ny: int, centres, amplitude: float, width: float) -> np.ndarray:
    """S = 1 - I, E = R = D = 0, I a sum of periodic Gaussian bumps (std ``width``)
    of height ``amplitude`` at the given (x, y) cells, clipped to at most 1."""
    infected = np.zeros((ny, nx))
    for cx, cy in centres:
        gx = np.exp(-_min_image_sq(nx, cx) / (2.0 * width * width))
        gy = np.exp(-_min_image_sq(ny, cy) / (2.0 * width * width))
        infected += amplitude * np.outer(gy, gx)
    infected = np.minimum(infected, 1.0)
    rho = np.zeros((5, ny, nx))
    rho[0] = 1.0 - infected
    rho[2] = infected
    return rho


def gaussian_foci_factors(nx: int, ny: int, centres, amplitude: float, width: float):
    """The separable factors of ``gaussian_foci_state``'s infected field before
    clipping: (gy, gx) of shapes (foci, ny) and (foci, nx), the amplitude
    folded into gy, so that the field is the sum over the foci of the outer
    products gy[f] gx[f] (for building many such states on a device)."""
    gx = np.stack([np.exp(-_min_image_sq(nx, cx) / (2.0 * width * width)) for cx, _ in centres])
    gy = np.stack([amplitude * np.exp(-_min_image_sq(ny, cy) / (2.0 * width * width))
                   for _, cy in centres])
    return gy, gx


def seeded_centres(nx: int, ny: int, count: int, seed: int):
    rng = np.random.default_rng(seed)
    xs = rng.integers(0, nx, size=count)
    ys = rng.integers(0, ny, size=count)
    return list(zip(xs.tolist(), ys.tolist()))


def random_state(nx: int, ny: int, seed: int, infected_scale: float = 0.2) -> np.ndarray:
    """Rough, strictly positive random densities: S in [0.3, 1], E, I, R, D up to
    ``infected_scale``; every cell different, so any wrong index shows up."""
    rng = np.random.default_rng(seed)
    rho = np.empty((5, ny, nx))
    rho[0] = rng.uniform(0.3, 1.0, size=(ny, nx))
    for c in range(1, 5):
        rho[c] = rng.uniform(0.0, infected_scale, size=(ny, nx))
    return rho


def empty_block_state(nx: int, ny: int, seed: int, rows: slice, cols: slice,
                      compartments: int = 5) -> np.ndarray:
    """``random_state`` (or, for more than five compartments, uniform random
    densities) with S = E = I = R = 0 on a block of cells (D > 0 there: the
    deceased are not contact-eligible) and one cell that is entirely empty:
    cells whose contact-eligible population is zero, next to populated ones,
    so that diffusion carries ever smaller (eventually subnormal) densities
    into the block."""
    if compartments == 5:
        rho = random_state(nx, ny, seed)
    else:
        rng = np.random.default_rng(seed)
        rho = rng.uniform(0.0, 0.3, size=(compartments, ny, nx))
        rho[0] += 0.5
    counted = [c for c in range(compartments) if c != 4]
    for c in counted:
        rho[c, rows, cols] = 0.0
    rho[:, min(3, ny - 1), min(5, nx - 1)] = 0.0
    return rho


# ---------------------------------------------------------------- configs --

@dataclass(frozen=True)
class Workload:
    name: str
    nx: int
    ny: int
    params: Params
    rho0: np.ndarray = field(repr=False)
    nsteps: int
    bc: str = "periodic"


def c1_params() -> Params:
    """SEIRD rates beta=0.5, sigma=0.2, gamma=0.1, mu=0.01 (R0 = beta/(gamma+mu) ~ 4.5),
    lattice diffusivity 1e-3 for S, E, I, R, none for D; dx = 1, dt = 0.01."""
    return from_sigma_mu(0.5, 0.2, 0.1, 0.01, (1e-3, 1e-3, 1e-3, 1e-3, 0.0))


def c1_workload(nx: int = 128, ny: int = 128, seed: int = 1, nsteps: int = 1000) -> Workload:
    """128x128 periodic grid, 1000 steps, one Gaussian bump of infected
    (amplitude 0.01, width 5 cells) at a seeded cell."""
    centre = seeded_centres(nx, ny, 1, seed)
    rho0 = gaussian_foci_state(nx, ny, centre, amplitude=0.01, width=5.0)
    return Workload("sslbm-seird-128x128-periodic", nx, ny, c1_params(), rho0, nsteps)


def c2_diffusivities(seed: int = 2) -> tuple:
    """Lattice diffusivities of S, E, I, R drawn log-uniform in [1e-4, 1e-2]; D = 0."""
    rng = np.random.default_rng(seed + 1000)
    lo, hi = np.log(1e-4), np.log(1e-2)
    return tuple(np.exp(rng.uniform(lo, hi, size=4)).tolist()) + (0.0,)


def c2_params(r0: float, seed: int = 2) -> Params:
    """Steep-gradient regime: sigma=0.2, gamma=0.1, mu=0.01, beta = R0 (gamma+mu)."""
    gamma, mu = 0.1, 0.01
    return from_sigma_mu(r0 * (gamma + mu), 0.2, gamma, mu, c2_diffusivities(seed))


C2_R0 = (1.5, 3.0, 5.0)


def c2_state(nx: int = 4096, ny: int = 4096, seed: int = 2, foci: int = 64) -> np.ndarray:
    """64 seeded infected foci of width 2 cells and amplitude 0.01."""
    return gaussian_foci_state(nx, ny, seeded_centres(nx, ny, foci, seed), 0.01, 2.0)


def c2_workload(r0: float = 3.0, nx: int = 4096, ny: int = 4096, seed: int = 2,
                nsteps: int = 10000) -> Workload:
    return Workload(f"sslbm-seird-{nx}x{ny}-64foci-R0={r0:g}", nx, ny, c2_params(r0, seed),
                    c2_state(nx, ny, seed), nsteps)


def paper_test_case(nx: int, ny: int, chi: float, r0: float, seed: int, eps: float = 1e-3):
    """The paper's accuracy test (Sec. III): total population N = 5e6 over a
    200 x 200 km^2 domain, a fraction chi exposed plus a small random field,
    gamma = 1/5, alpha = 1/7, phi = 0.3, beta = R0 gamma, d^{S,E,R} = 4.35e-2,
    d^I = 1e-4 km^2/day, dx = 1 km, dt = 0.01 day. The law of the random field is
    not given; it is read here as uniform in [-1, 1] times eps * chi * N / A."""
    gamma = 1.0 / 5.0
    p = Params(beta=r0 * gamma, alpha=1.0 / 7.0, gamma=gamma, phi=0.3,
               d=(4.35e-2, 4.35e-2, 1e-4, 4.35e-2, 0.0), dx=1.0, dt=0.01)
    density = 5e6 / (200.0 * 200.0)
    rng = np.random.default_rng(seed)
    rho = np.zeros((5, ny, nx))
    exposed = chi * density + eps * chi * density * rng.uniform(-1.0, 1.0, size=(ny, nx))
    rho[1] = exposed
    rho[0] = density - exposed
    return p, rho


# ------------------------------------------------------------- ensembles --

@dataclass(frozen=True)
class EnsembleWorkload:
    name: str
    sizes: list = field(repr=False)      # (nx, ny) per instance
    params: list = field(repr=False)     # Params per instance
    nsteps: int = 2000
    bc: str = "periodic"

    def states(self):
        """Initial state of every instance (generated on demand: 512 of them
        take ~0.9 GB in FP64)."""
        rng = np.random.default_rng(self._seed + 77)
        for nx, ny in self.sizes:
            foci = int(rng.integers(1, 9))
            centres = list(zip(rng.integers(0, nx, foci).tolist(), rng.integers(0, ny, foci).tolist()))
            yield gaussian_foci_state(nx, ny, centres, amplitude=0.01, width=4.0)

    _seed: int = 3


def ensemble_workload(count: int = 512, seed: int = 3, nsteps: int = 2000,
                      sides=(64, 128, 256, 512)) -> EnsembleWorkload:
    """Uneven ensemble: square grids with sides drawn uniformly from `sides`,
    R0 uniform in [1.5, 5] through beta = R0 (gamma + mu), lattice
    diffusivities of S, E, I, R log-uniform in [1e-4, 1e-2] (D at rest),
    sigma = 0.2, gamma = 0.1, mu = 0.01, and 1 to 8 Gaussian foci of width 4
    cells and amplitude 0.01 per instance."""
    rng = np.random.default_rng(seed)
    n = rng.choice(np.asarray(sides), size=count)
    r0 = rng.uniform(1.5, 5.0, size=count)
    dl = np.exp(rng.uniform(np.log(1e-4), np.log(1e-2), size=(count, 4)))
    gamma, mu = 0.1, 0.01
    params = [from_sigma_mu(r0[i] * (gamma + mu), 0.2, gamma, mu, tuple(dl[i]) + (0.0,))
              for i in range(count)]
    sizes = [(int(v), int(v)) for v in n]
    return EnsembleWorkload(f"sslbm-ensemble-{count}-uneven", sizes, params, nsteps,
                            _seed=seed)


# --------------------------------------------------------------- adjoint --

def c4_params() -> Params:
    """Rates beta=0.5, sigma=0.2, gamma=0.1, mu=0.01 and lattice diffusivity
    1e-3 for all five compartments (D included, so that central differences in
    every diffusivity stay inside d >= 0); dx = 1, dt = 0.01."""
    return from_sigma_mu(0.5, 0.2, 0.1, 0.01, (1e-3,) * 5)


C4_SIGMA_MU = (0.5, 0.2, 0.1, 0.01)


def c4_perturbed_sigma_mu(seed: int = 4) -> tuple:
    """(beta, sigma, gamma, mu) of the fitting target: each rate of C4
    multiplied by 1 + 0.05 N(0, 1)."""
    rng = np.random.default_rng(seed)
    return tuple(float(v * (1.0 + 0.05 * z)) for v, z in zip(C4_SIGMA_MU, rng.normal(size=4)))


def c4_target_params(seed: int = 4) -> Params:
    return from_sigma_mu(*c4_perturbed_sigma_mu(seed), (1e-3,) * 5)


def c4_state(nx: int = 1024, ny: int = 1024, seed: int = 4) -> np.ndarray:
    """16 seeded Gaussian foci of infected, amplitude 0.01, width 8 cells."""
    return gaussian_foci_state(nx, ny, seeded_centres(nx, ny, 16, seed), 0.01, 8.0)


def c4_workload(nx: int = 1024, ny: int = 1024, seed: int = 4, nsteps: int = 2000) -> Workload:
    return Workload(f"sslbm-adjoint-{nx}x{ny}-fp64", nx, ny, c4_params(), c4_state(nx, ny, seed),
                    nsteps)


# ------------------------------------------------------------- surrogate --

def c5_rollout_workload(n: int = 1024, seed: int = 5, nsteps: int = 5000) -> Workload:
    """Surrogate rollout: n x n periodic grid, R0 = 3 through beta, lattice
    diffusivities of S, E, I, R log-uniform in [1e-4, 1e-2] (seeded), D at
    rest, 16 seeded Gaussian foci of amplitude 0.01 and width 8, 5000 steps
    (100 surrogate jumps of 50 steps)."""
    return Workload(f"sslbm-surrogate-rollout-{n}x{n}", n, n, c2_params(3.0, seed),
                    gaussian_foci_state(n, n, seeded_centres(n, n, 16, seed), 0.01, 8.0), nsteps)


# --------------------------------------------------------- generic models --

@dataclass(frozen=True)
class GenericModel:
    """A compartmental model d_t C = Psi^C + d^C lap C (Eq. (generic_pde)).
    transitions: (src, dst, catalyst, rate, frequency) tuples; transition r
    moves rate * C[src] * C[catalyst] (1 when catalyst < 0), divided by the
    sum of the `counted` compartments when frequency is 1, from src to dst
    (dst < 0: out of the system). d: physical diffusivities; lattice 5 or 9."""
    names: tuple
    d: tuple
    transitions: tuple
    counted: tuple
    lattice: int = 5
    dx: float = 1.0
    dt: float = 0.01


def seirvd_model(lattice: int = 9, dt: float = 0.01) -> GenericModel:
    """A richer model than SEIRD: vaccinated V (rate nu from S, leaky
    protection: V infected at 30 % of the susceptible rate) and waning
    immunity (R -> S at rate omega). Compartments S, E, I, R, D, V; D at
    rest; lattice diffusivities 2e-3 (S, E, R, V) and 5e-4 (I)."""
    beta, sigma, gamma, mu, nu, omega, leak = 0.5, 0.2, 0.1, 0.01, 0.02, 0.005, 0.3
    d_lu = (2e-3, 2e-3, 5e-4, 2e-3, 0.0, 2e-3)
    S, E, I, R, D, V = range(6)
    transitions = ((S, E, I, beta, 1), (V, E, I, leak * beta, 1), (E, I, -1, sigma, 0),
                   (I, R, -1, gamma, 0), (I, D, -1, mu, 0), (S, V, -1, nu, 0),
                   (R, S, -1, omega, 0))
    return GenericModel(("S", "E", "I", "R", "D", "V"), lattice_to_physical(d_lu, 1.0, dt),
                        transitions, (1, 1, 1, 1, 0, 1), lattice, 1.0, dt)


def seirvd_state(nx: int, ny: int, seed: int = 6, foci: int = 8) -> np.ndarray:
    """S = 1 - I, 8 seeded infected foci (amplitude 0.02, width 4), others 0."""
    base = gaussian_foci_state(nx, ny, seeded_centres(nx, ny, foci, seed), 0.02, 4.0)
    rho = np.zeros((6, ny, nx))
    rho[:5] = base
    return rho
