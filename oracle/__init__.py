"""FP64 CPU oracle for the SSLBM SEIRD step and the BGK comparison step.

TEST INFRASTRUCTURE. Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` may import this package. The product path (the
HIP library and its binding in ``paper_2603_19789_amd``) never imports it, and
the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, FP64, compiled with gcc without
FMA contraction). This module only marshals NumPy arrays through ctypes and
builds the library with gcc when it is missing.

Parameters are passed as any object with attributes ``beta, alpha, gamma, phi``
(the paper's rates, Sec. II.A), ``d`` (five diffusivities, length^2/time),
``dx`` and ``dt``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

HERE = Path(__file__).resolve().parent
SOURCE = HERE / "oracle.c"
LIBRARY = HERE / "liboracle.so"

PERIODIC = 0
NOFLUX = 1
_BC = {"periodic": PERIODIC, "noflux": NOFLUX, PERIODIC: PERIODIC, NOFLUX: NOFLUX}


def compile_library(source: Path = SOURCE, output: Path = LIBRARY, defines=()) -> Path:
    """Compile the oracle with gcc: -O2, IEEE FP64, no FMA contraction, OpenMP."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-o", str(output), str(source), "-lm"]
    cmd[1:1] = [f"-D{d}" for d in defines]
    subprocess.run(cmd, check=True)
    return output


_DP = ctypes.POINTER(ctypes.c_double)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_DP)


def _f64(a, shape=None) -> np.ndarray:
    out = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None and out.shape != tuple(shape):
        raise ValueError(f"expected shape {tuple(shape)}, got {out.shape}")
    return out


class Oracle:
    """ctypes view of one compiled copy of ``oracle.c``."""

    def __init__(self, path: Path | str = LIBRARY):
        self.path = Path(path)
        lib = ctypes.CDLL(str(self.path))
        i, d, ll = ctypes.c_int, ctypes.c_double, ctypes.c_longlong
        lib.oracle_sslbm_step.argtypes = [i, i, i, _DP, _DP, d, d, _DP, _DP, i]
        lib.oracle_sslbm_run.argtypes = [i, i, i, _DP, _DP, d, d, _DP, _DP, ll, i]
        lib.oracle_bgk_init.argtypes = [i, i, _DP, _DP, _DP]
        lib.oracle_bgk_density.argtypes = [i, i, _DP, _DP, _DP]
        lib.oracle_bgk_step.argtypes = [i, i, i, _DP, _DP, d, d, _DP, _DP, _DP, _DP, i]
        lib.oracle_bgk_run.argtypes = [i, i, i, _DP, _DP, d, d, _DP, _DP, _DP, _DP, ll, i]
        lib.oracle_sslbm_adjoint_step.argtypes = [i, i, i, _DP, _DP, d, d, _DP, _DP, _DP, _DP]
        _IP = ctypes.POINTER(ctypes.c_int)
        lib.oracle_generic_step.argtypes = [i, i, i, i, i, _DP, d, d, i, _IP, _IP, _IP, _IP, _DP,
                                            _IP, _DP, _DP]
        lib.oracle_fd4_rk4_run.argtypes = [i, i, i, _DP, _DP, d, d, _DP, ll]
        for f in ("oracle_sslbm_step", "oracle_sslbm_run", "oracle_bgk_init",
                  "oracle_bgk_density", "oracle_bgk_step", "oracle_bgk_run",
                  "oracle_sslbm_adjoint_step", "oracle_generic_step", "oracle_fd4_rk4_run"):
            getattr(lib, f).restype = ctypes.c_int
        self.lib = lib

    @staticmethod
    def _params(p):
        rates = np.array([p.beta, p.alpha, p.gamma, p.phi], dtype=np.float64)
        d = _f64(p.d, (5,)).copy()
        return rates, d, float(p.dx), float(p.dt)

    @staticmethod
    def _check(rc: int, what: str):
        if rc != 0:
            raise ValueError(f"{what}: oracle rejected the arguments (code {rc})")

    # ------------------------------------------------------------- SSLBM --
    def sslbm_step(self, rho, p, bc="periodic", threads: int = 1) -> np.ndarray:
        """One step, Eq. (sslbm_final_clean); rho has shape (5, ny, nx)."""
        rho = _f64(rho)
        _, ny, nx = rho.shape
        out = np.empty_like(rho)
        rates, d, dx, dt = self._params(p)
        rc = self.lib.oracle_sslbm_step(nx, ny, _BC[bc], _ptr(rates), _ptr(d), dx, dt,
                                        _ptr(rho), _ptr(out), threads)
        self._check(rc, "sslbm_step")
        return out

    def sslbm_run(self, rho, p, nsteps: int, bc="periodic", threads: int = 1) -> np.ndarray:
        rho = _f64(rho).copy()
        _, ny, nx = rho.shape
        work = np.empty_like(rho)
        rates, d, dx, dt = self._params(p)
        rc = self.lib.oracle_sslbm_run(nx, ny, _BC[bc], _ptr(rates), _ptr(d), dx, dt,
                                       _ptr(rho), _ptr(work), int(nsteps), threads)
        self._check(rc, "sslbm_run")
        return rho

    def fd4_rk4_run(self, rho, p, nsteps: int, bc="periodic") -> np.ndarray:
        """The finite-difference reference of Sec. III: fourth-order centred
        Laplacian, classic RK4, reactions explicit at every stage."""
        rho = _f64(rho).copy()
        _, ny, nx = rho.shape
        rates, d, dx, dt = self._params(p)
        rc = self.lib.oracle_fd4_rk4_run(nx, ny, _BC[bc], _ptr(rates), _ptr(d), dx, dt,
                                         _ptr(rho), int(nsteps))
        self._check(rc, "fd4_rk4_run")
        return rho

    # ------------------------------------------------------------ adjoint --
    def sslbm_adjoint_step(self, rho, lam_next, p, bc="periodic"):
        """Reverse of one step at state rho (time t): returns dJ/d rho(t) and the
        step's dJ/d(beta, alpha, gamma, phi, d[0..4]) given dJ/d rho(t+dt)."""
        rho = _f64(rho)
        lam_next = _f64(lam_next, rho.shape)
        _, ny, nx = rho.shape
        lam = np.empty_like(rho)
        grad = np.zeros(9)
        rates, d, dx, dt = self._params(p)
        rc = self.lib.oracle_sslbm_adjoint_step(nx, ny, _BC[bc], _ptr(rates), _ptr(d), dx, dt,
                                                _ptr(rho), _ptr(lam_next), _ptr(lam), _ptr(grad))
        self._check(rc, "sslbm_adjoint_step")
        return lam, grad

    def sslbm_adjoint_run(self, rho0, p, nsteps: int, lam_final, bc="periodic"):
        """Whole-run reverse sweep: forward storing every state, then the
        adjoint steps back to t = 0. Returns dJ/d rho0 and dJ/d params (9)."""
        states = [_f64(rho0).copy()]
        for _ in range(nsteps):
            states.append(self.sslbm_step(states[-1], p, bc=bc))
        lam = _f64(lam_final).copy()
        grad = np.zeros(9)
        for n in range(nsteps - 1, -1, -1):
            lam, g = self.sslbm_adjoint_step(states[n], lam, p, bc=bc)
            grad += g
        return lam, grad

    # ------------------------------------------------------ generic models --
    def generic_step(self, rho, model, bc="periodic"):
        """One step of a generic compartmental model (see GenericModel)."""
        rho = _f64(rho)
        m, ny, nx = rho.shape
        out = np.empty_like(rho)
        ip = lambda v: (ctypes.c_int * max(len(v), 1))(*[int(x) for x in v])
        dp = lambda v: (ctypes.c_double * max(len(v), 1))(*[float(x) for x in v])
        t = model.transitions
        rc = self.lib.oracle_generic_step(
            nx, ny, _BC[bc], model.lattice, m, dp(model.d), model.dx, model.dt, len(t),
            ip([x[0] for x in t]), ip([x[1] for x in t]), ip([x[2] for x in t]),
            ip([x[4] for x in t]), dp([x[3] for x in t]), ip(model.counted), _ptr(rho), _ptr(out))
        self._check(rc, "generic_step")
        return out

    def generic_run(self, rho, model, nsteps: int, bc="periodic"):
        rho = _f64(rho).copy()
        for _ in range(nsteps):
            rho = self.generic_step(rho, model, bc=bc)
        return rho

    # --------------------------------------------------------------- BGK --
    def bgk_init(self, rho):
        """Equilibrium populations: returns f (4, 5, ny, nx) and rhoD (ny, nx)."""
        rho = _f64(rho)
        _, ny, nx = rho.shape
        f = np.empty((4, 5, ny, nx))
        rd = np.empty((ny, nx))
        self._check(self.lib.oracle_bgk_init(nx, ny, _ptr(rho), _ptr(f), _ptr(rd)), "bgk_init")
        return f, rd

    def bgk_density(self, f, rhoD) -> np.ndarray:
        f = _f64(f)
        ny, nx = f.shape[2:]
        rhoD = _f64(rhoD, (ny, nx))
        rho = np.empty((5, ny, nx))
        self._check(self.lib.oracle_bgk_density(nx, ny, _ptr(f), _ptr(rhoD), _ptr(rho)),
                    "bgk_density")
        return rho

    def bgk_step(self, f, rhoD, p, bc="periodic", threads: int = 1):
        f = _f64(f)
        ny, nx = f.shape[2:]
        rhoD = _f64(rhoD, (ny, nx))
        fo, do = np.empty_like(f), np.empty_like(rhoD)
        rates, d, dx, dt = self._params(p)
        rc = self.lib.oracle_bgk_step(nx, ny, _BC[bc], _ptr(rates), _ptr(d), dx, dt, _ptr(f),
                                      _ptr(rhoD), _ptr(fo), _ptr(do), threads)
        self._check(rc, "bgk_step")
        return fo, do

    def bgk_run(self, f, rhoD, p, nsteps: int, bc="periodic", threads: int = 1):
        f = _f64(f).copy()
        ny, nx = f.shape[2:]
        rhoD = _f64(rhoD, (ny, nx)).copy()
        fw, dw = np.empty_like(f), np.empty_like(rhoD)
        rates, d, dx, dt = self._params(p)
        rc = self.lib.oracle_bgk_run(nx, ny, _BC[bc], _ptr(rates), _ptr(d), dx, dt, _ptr(f),
                                     _ptr(rhoD), _ptr(fw), _ptr(dw), int(nsteps), threads)
        self._check(rc, "bgk_run")
        return f, rhoD

    def bgk_run_density(self, rho0, p, nsteps: int, bc="periodic", threads: int = 1):
        """Equilibrium start from rho0, nsteps BGK steps, densities out."""
        f, rd = self.bgk_init(rho0)
        f, rd = self.bgk_run(f, rd, p, nsteps, bc, threads)
        return self.bgk_density(f, rd)


_DEFAULT: Oracle | None = None


def load() -> Oracle:
    """The oracle built from ``oracle.c`` (compiled with gcc only if no build exists)."""
    global _DEFAULT
    if _DEFAULT is None:
        if not LIBRARY.exists():
            compile_library()
        _DEFAULT = Oracle(LIBRARY)
    return _DEFAULT


def host_threads() -> int:
    """Threads the oracle may use on this host (OMP_NUM_THREADS if set)."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return os.cpu_count() or 1
