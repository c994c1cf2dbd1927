"""Independent FP64 references used to pin the oracle (CPU, NumPy).

None of these re-types the oracle's update formula. Each is derived from a
different statement in the paper or from mathematics that fixes the answer:

* ``seird_rhs``            -- the PDE right-hand side, Eqs. (EqSEIRD_S)-(EqSEIRD_D)
* ``lattice_symbol``       -- Lambda(k) as the sum over links (Sec. II.C.2, stability)
* ``sslbm_amplification``  -- G(k) from the unsimplified first line of Eq. (G_exact)
* ``exact_discrete_diffusion`` -- G(k)^n applied mode by mode (FFT), Psi = 0
* ``bgk_exact_discrete``   -- the BGK LBE (Eq. pdf) solved mode by mode (5x5 per k)
* ``fd4_rk4_run``          -- the paper's fourth-order FD / RK4 reference (Sec. III)
* ``euler_ode`` / ``rk4_ode`` -- textbook integrators of the local SEIRD ODE
* ``dfe_eigenvalues``      -- Eq. (eigenvalues) for the E-I block at the DFE
* ``heat_kernel_gaussian`` -- continuum solution of pure diffusion from a Gaussian
* ``bgk_fp32_model``       -- the BGK scheme (Eq. pdf) evaluated in plain NumPy
                              float32, to measure what FP32 storage and
                              arithmetic alone cost (not a pin of the oracle)
"""
from __future__ import annotations

import numpy as np

# D2Q5 lattice as printed in Sec. II.B (kept here independently of the oracle)
CX = np.array([0, 1, 0, -1, 0])
CY = np.array([0, 0, 1, 0, -1])
WEIGHTS = np.array([1 / 3, 1 / 6, 1 / 6, 1 / 6, 1 / 6])


def lattice_diffusivity(p, c: int) -> float:
    return p.d[c] * p.dt / (p.dx * p.dx)


# ------------------------------------------------------------ the PDE RHS --

def seird_rhs(y: np.ndarray, p) -> np.ndarray:
    """Reaction part of Eqs. (EqSEIRD_S)-(EqSEIRD_D) with the contact-eligible
    population N_c = S + E + I + R; y has the compartments on axis 0."""
    S, E, I, R = y[0], y[1], y[2], y[3]
    Nc = S + E + I + R
    safe = np.where(Nc > 0, Nc, 1.0)
    infection = np.where(Nc > 0, p.beta * S * I / safe, 0.0)
    out = np.empty_like(y)
    out[0] = -infection
    out[1] = infection - p.alpha * E
    out[2] = p.alpha * E - p.gamma * I
    out[3] = (1 - p.phi) * p.gamma * I
    out[4] = p.phi * p.gamma * I
    return out


def euler_ode(y0: np.ndarray, p, dt: float, nsteps: int) -> np.ndarray:
    y = np.array(y0, dtype=np.float64)
    for _ in range(nsteps):
        y = y + dt * seird_rhs(y, p)
    return y


def rk4_ode(y0: np.ndarray, p, dt: float, nsteps: int) -> np.ndarray:
    y = np.array(y0, dtype=np.float64)
    for _ in range(nsteps):
        k1 = seird_rhs(y, p)
        k2 = seird_rhs(y + 0.5 * dt * k1, p)
        k3 = seird_rhs(y + 0.5 * dt * k2, p)
        k4 = seird_rhs(y + dt * k3, p)
        y = y + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


def dfe_eigenvalues(p):
    """lambda_{1,2} of the E-I block of the Jacobian at the disease-free
    equilibrium, Eq. (eigenvalues), with the paper's alpha and gamma."""
    a, g, b = p.alpha, p.gamma, p.beta
    root = np.sqrt((a - g) ** 2 + 4 * a * b)
    return (-(a + g) + root) / 2, (-(a + g) - root) / 2


# ------------------------------------------------------- Fourier analysis --

def lattice_symbol(kx, ky):
    """Lambda(k) = sum_i w_i exp(i k . c_i), evaluated as the complex sum."""
    kx = np.asarray(kx, dtype=np.float64)[..., None]
    ky = np.asarray(ky, dtype=np.float64)[..., None]
    return np.sum(WEIGHTS * np.exp(1j * (kx * CX + ky * CY)), axis=-1)


def sslbm_amplification(tau: float, kx, ky):
    """G(k) from the first line of Eq. (G_exact): substitute rho_f = rho_b =
    Lambda rho and rho_c = rho into the diffusion update Eq. (sslbm_clean)."""
    lam = lattice_symbol(kx, ky).real
    return lam + (tau - 1.0) * (lam - 2.0 + lam)


def wavenumbers(nx: int, ny: int):
    kx = 2 * np.pi * np.fft.fftfreq(nx)
    ky = 2 * np.pi * np.fft.fftfreq(ny)
    return np.meshgrid(kx, ky)  # arrays of shape (ny, nx)


def exact_discrete_diffusion(field: np.ndarray, tau: float, nsteps: int) -> np.ndarray:
    """Pure-diffusion SSLBM on a periodic grid, solved exactly mode by mode."""
    ny, nx = field.shape
    KX, KY = wavenumbers(nx, ny)
    g = sslbm_amplification(tau, KX, KY)
    return np.real(np.fft.ifft2(np.fft.fft2(field) * g ** nsteps))


def bgk_exact_discrete(field: np.ndarray, tau: float, nsteps: int) -> np.ndarray:
    """Pure-diffusion BGK (Eq. pdf with Psi = 0) from equilibrium start on a
    periodic grid, solved mode by mode: collision f* = f + (w rho - f)/tau is
    the 5x5 matrix (1 - 1/tau) Id + (1/tau) w 1^T, and streaming to x + c_i
    multiplies mode k of population i by exp(-i k . c_i)."""
    ny, nx = field.shape
    KX, KY = wavenumbers(nx, ny)
    collide = (1 - 1 / tau) * np.eye(5) + (1 / tau) * np.outer(WEIGHTS, np.ones(5))
    shift = np.exp(-1j * (KX[..., None] * CX + KY[..., None] * CY))  # (ny, nx, 5)
    step = shift[..., :, None] * collide[None, None, :, :]  # (ny, nx, 5, 5)
    fh = WEIGHTS[None, None, :] * np.fft.fft2(field)[..., None]
    for _ in range(nsteps):
        fh = np.einsum("yxij,yxj->yxi", step, fh)
    return np.real(np.fft.ifft2(fh.sum(axis=-1)))


def heat_kernel_gaussian(nx, ny, cx, cy, amplitude, s0, d, t):
    """Continuum solution of d_t u = d lap u on the plane from
    amplitude * exp(-r^2 / (2 s0^2)); distances are periodic minimum images."""
    x = np.arange(nx) - cx
    y = np.arange(ny) - cy
    x = np.minimum(np.abs(x), nx - np.abs(x))
    y = np.minimum(np.abs(y), ny - np.abs(y))
    r2 = y[:, None] ** 2 + x[None, :] ** 2
    s2 = s0 * s0 + 2 * d * t
    return amplitude * (s0 * s0 / s2) * np.exp(-r2 / (2 * s2))


# ------------------------------------------------ fourth-order FD + RK4 ----

def _laplacian4(u: np.ndarray, dx: float, bc: str) -> np.ndarray:
    """Fourth-order centred Laplacian, (-u[-2] + 16u[-1] - 30u + 16u[+1] - u[+2])/12
    per axis. Periodic wraps; no-flux uses an even reflection about the
    boundary face (zero normal derivative)."""
    pad = [(0, 0)] * (u.ndim - 2) + [(2, 2), (2, 2)]
    w = np.pad(u, pad, mode="wrap" if bc == "periodic" else "symmetric")
    c = w[..., 2:-2, 2:-2]
    acc = (-w[..., 2:-2, :-4] + 16 * w[..., 2:-2, 1:-3] - 30 * c + 16 * w[..., 2:-2, 3:-1]
           - w[..., 2:-2, 4:])
    acc += (-w[..., :-4, 2:-2] + 16 * w[..., 1:-3, 2:-2] - 30 * c + 16 * w[..., 3:-1, 2:-2]
            - w[..., 4:, 2:-2])
    return acc / (12 * dx * dx)


def fd4_rk4_rhs(rho: np.ndarray, p, bc: str) -> np.ndarray:
    out = seird_rhs(rho, p)
    dvec = np.asarray(p.d, dtype=np.float64)
    lap = _laplacian4(rho, p.dx, bc)
    return out + dvec[:, None, None] * lap


def fd4_rk4_run(rho0: np.ndarray, p, nsteps: int, bc: str = "periodic") -> np.ndarray:
    """Reference solver of Sec. III: classic RK4 in time, fourth-order centred
    differences in space, reactions explicit at every stage."""
    y = np.array(rho0, dtype=np.float64)
    dt = p.dt
    for _ in range(nsteps):
        k1 = fd4_rk4_rhs(y, p, bc)
        k2 = fd4_rk4_rhs(y + 0.5 * dt * k1, p, bc)
        k3 = fd4_rk4_rhs(y + 0.5 * dt * k2, p, bc)
        k4 = fd4_rk4_rhs(y + dt * k3, p, bc)
        y = y + dt / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


# ------------------------------------------------------------------ norms --

def rel_l2(a: np.ndarray, b: np.ndarray) -> float:
    """||a - b||_2 / ||b||_2 (absolute when ||b|| = 0)."""
    nb = np.linalg.norm(b)
    diff = np.linalg.norm(np.asarray(a, dtype=np.float64) - b)
    return float(diff / nb) if nb > 0 else float(diff)


def rel_l2_per_compartment(a: np.ndarray, b: np.ndarray):
    return [rel_l2(a[c], b[c]) for c in range(a.shape[0])]


# ------------------------------------------------------- FP32 rounding floor --

def bgk_fp32_model(rho0: np.ndarray, p, nsteps: int) -> np.ndarray:
    """The BGK scheme of Eq. (pdf) with f^eq = w_i rho and the source
    w_i Psi dt (Eq. sources, Eq. rhoD by forward Euler for D), equilibrium
    start, periodic push streaming, every value stored and every operation
    rounded in float32 by NumPy. Returns the densities in float64. It is not
    a reference for the scheme (the FP64 oracle is), only for how far FP32
    rounding alone moves it."""
    f32 = np.float32
    w = WEIGHTS.astype(f32)
    rho = np.asarray(rho0, dtype=f32)
    f = np.stack([w[i] * rho[:4] for i in range(5)], axis=1)
    dead = rho[4].copy()
    dl = np.array([lattice_diffusivity(p, c) for c in range(4)])
    omega = (1.0 / (0.5 + 3.0 * dl)).astype(f32)
    bdt, ke, ki = f32(p.beta * p.dt), f32(p.alpha * p.dt), f32(p.gamma * p.dt)
    kr, kd = f32((1 - p.phi) * p.gamma * p.dt), f32(p.phi * p.gamma * p.dt)
    for _ in range(nsteps):
        r = f.sum(axis=1, dtype=f32)
        S, E, I, R = r
        nc = (S + E) + (I + R)
        force = np.where(nc > 0, bdt * S * I / np.where(nc > 0, nc, f32(1)), f32(0))
        src = np.stack([-force, force - ke * E, ke * E - ki * I, kr * I])
        new = np.empty_like(f)
        for c in range(4):
            for i in range(5):
                post = f[c, i] + (w[i] * r[c] - f[c, i]) * omega[c] + w[i] * src[c]
                new[c, i] = np.roll(post, (CY[i], CX[i]), axis=(0, 1))
        dead = dead + kd * I
        f = new
    return np.concatenate([f.sum(axis=1, dtype=f32), dead[None]]).astype(np.float64)
