"""ctypes binding of libsslbm.so (argument marshalling only).

Every step of the solver runs in the HIP kernels of ``libsslbm.so``; this
module checks tensors, passes raw device pointers and the current HIP stream,
and turns status codes into ``SSLBMError``. There is no other code path: if
the library is missing, every call raises.

Tensors are torch tensors on the GPU, contiguous, float32 or float64:
  rho  (5, ny, nx)      densities S, E, I, R, D
  f    (4, 5, ny, nx)   BGK populations of S, E, I, R over the D2Q5 links
  rhoD (ny, nx)         deceased density of the BGK state
Parameters are any object with attributes beta, alpha, gamma, phi, d (5
values), dx, dt (see ``inputs.Params``).
"""
from __future__ import annotations

import ctypes
from pathlib import Path

LIBRARY = Path(__file__).resolve().parent / "libsslbm.so"
HEADER = Path(__file__).resolve().parent.parent / "include" / "sslbm.h"

OK, E_ARG, E_UNSTABLE, E_UNSUPPORTED, E_ALIAS, E_HIP, E_NOMEM, E_LIMIT = (
    0, -1, -2, -3, -4, -5, -6, -7)
F32, F64 = 0, 1
GRAD_COUNT = 9  # dJ/d(beta, alpha, gamma, phi, d[0..4])
PERIODIC, NOFLUX = 0, 1
MAX_BLOCKING = 8
MODEL_MAX_BLOCKING = 4
_BC = {"periodic": PERIODIC, "noflux": NOFLUX, PERIODIC: PERIODIC, NOFLUX: NOFLUX}


class SSLBMError(RuntimeError):
    def __init__(self, status: int, what: str, hip_error: int = 0):
        self.status = status
        self.hip_error = hip_error
        msg = f"{what}: {_strerror(status)} (status {status}"
        msg += f", hipError {hip_error})" if hip_error else ")"
        super().__init__(msg)


class Params(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_double), ("alpha", ctypes.c_double),
                ("gamma", ctypes.c_double), ("phi", ctypes.c_double),
                ("d", ctypes.c_double * 5), ("dx", ctypes.c_double), ("dt", ctypes.c_double)]

    @classmethod
    def of(cls, p) -> "Params":
        return cls(float(p.beta), float(p.alpha), float(p.gamma), float(p.phi),
                   (ctypes.c_double * 5)(*[float(v) for v in p.d]), float(p.dx), float(p.dt))


class Transition(ctypes.Structure):
    _fields_ = [("src", ctypes.c_int), ("dst", ctypes.c_int), ("catalyst", ctypes.c_int),
                ("frequency", ctypes.c_int), ("rate", ctypes.c_double)]


class Launch(ctypes.Structure):
    """Pass shape (zero = automatic): steps per HBM pass, output rows per
    wavefront, adjacent columns per lane."""
    _fields_ = [("steps_per_pass", ctypes.c_int), ("rows_per_wave", ctypes.c_int),
                ("cols_per_lane", ctypes.c_int)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class EnsembleClass(ctypes.Structure):
    """One size class of an ensemble (sslbm_ensemble_class)."""
    _fields_ = [("on_chip", ctypes.c_int), ("instances", ctypes.c_int),
                ("cells", ctypes.c_longlong), ("max_side", ctypes.c_int), ("launch", Launch)]

    def as_dict(self):
        return {"on_chip": bool(self.on_chip), "instances": self.instances, "cells": self.cells,
                "max_side": self.max_side, "launch": self.launch.as_dict()}


_LIB = None


def library() -> ctypes.CDLL:
    """The loaded libsslbm.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not LIBRARY.exists():
            raise RuntimeError(
                f"{LIBRARY} is missing: build it with `python -m paper_2603_19789_amd.build` "
                "(or __graft_entry__.build()); there is no fallback path")
        lib = ctypes.CDLL(str(LIBRARY))
        vp, i, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_longlong
        f, sz, fp = ctypes.c_float, ctypes.c_size_t, ctypes.POINTER(ctypes.c_float)
        pp = ctypes.POINTER(Params)
        sig = {
            "sslbm_init": [ctypes.POINTER(vp), i, i, i, i, pp],
            "sslbm_set_params": [vp, pp],
            "sslbm_set_blocking": [vp, i],
            "sslbm_get_blocking": [vp],
            "sslbm_set_launch": [vp, ctypes.POINTER(Launch)],
            "sslbm_get_launch": [vp, ctypes.POINTER(Launch)],
            "sslbm_tune": [vp, vp, vp, vp, ctypes.POINTER(Launch)],
            "sslbm_step": [vp, vp, vp, vp],
            "sslbm_run": [vp, vp, vp, ll, vp],
            "sslbm_plan_run": [vp, ll, ctypes.POINTER(ll), ctypes.POINTER(i), ctypes.POINTER(i)],
            "bgk_init": [vp, vp, vp, vp, vp],
            "bgk_step": [vp, vp, vp, vp, vp, vp],
            "bgk_run": [vp, vp, vp, vp, vp, ll, vp],
            "bgk_density": [vp, vp, vp, vp, vp],
            "sslbm_total": [vp, vp, ctypes.POINTER(ctypes.c_double), vp],
            "sslbm_fd4_run": [vp, vp, vp, sz, ll, vp],
            "sslbm_strerror": [i],
            "sslbm_last_hip_error": [vp],
            "sslbm_ensemble_create": [ctypes.POINTER(vp), i, ctypes.POINTER(i),
                                      ctypes.POINTER(i), i, i, pp, ctypes.POINTER(i)],
            "sslbm_ensemble_set_launch": [vp, ctypes.POINTER(Launch)],
            "sslbm_ensemble_get_launch": [vp, ctypes.POINTER(Launch)],
            "sslbm_ensemble_tune": [vp, vp, vp, vp, ctypes.POINTER(Launch)],
            "sslbm_ensemble_run": [vp, vp, vp, ll, i, vp],
            "sslbm_ensemble_run_class": [vp, i, vp, vp, ll, vp],
            "sslbm_ensemble_class_count": [vp],
            "sslbm_ensemble_instance_class": [vp, i],
            "sslbm_ensemble_class_info": [vp, i, ctypes.POINTER(EnsembleClass)],
            "sslbm_ensemble_set_class_launch": [vp, i, ctypes.POINTER(Launch)],
            "sslbm_ensemble_last_hip_error": [vp],
            "sslbm_adjoint_step": [vp, vp, vp, vp, vp, vp],
            "sslbm_adjoint_step_noalloc": [vp, vp, vp, vp, vp, vp],
            "sslbm_run_checkpointed": [vp, vp, vp, ll, i, vp, vp],
            "sslbm_adjoint_run": [vp, vp, ll, i, vp, vp, vp, vp],
            "sslbm_model_create": [ctypes.POINTER(vp), i, i, i, i, i, i,
                                   ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i),
                                   ctypes.c_double, ctypes.c_double, i,
                                   ctypes.POINTER(Transition)],
            "sslbm_model_step": [vp, vp, vp, vp],
            "sslbm_model_run": [vp, vp, vp, ll, vp],
            "sslbm_model_set_blocking": [vp, i],
            "sslbm_model_get_blocking": [vp, ctypes.POINTER(i)],
            "sslbm_model_last_hip_error": [vp],
            # surrogate.h
            "sur_conv3x3_forward": [vp, i, i, i, i, i, vp, vp, vp, i, i, i, f, vp],
            "sur_conv3x3_forward_pool": [vp, i, i, i, i, i, vp, vp, vp, i, i, i, f, vp, i, vp],
            "sur_conv3x3_forward_up": [vp, i, i, vp, i, i, i, i, i, vp, vp, vp, i, i, i, f, vp],
            "sur_conv3x3_backward_data": [vp, i, i, i, i, i, vp, i, vp, i, vp, vp],
            "sur_conv3x3_backward_weight": [vp, i, vp, i, i, i, i, i, i, vp, vp, vp, sz, vp],
            "sur_conv3x3_backward_weight_up": [vp, i, i, vp, i, vp, i, i, i, i, i, i, vp, vp, vp,
                                               sz, vp],
            "sur_conv3x3_backward_data_flipped": [vp, i, i, i, i, i, vp, i, vp, i, vp, i, f, vp],
            "sur_conv3x3_backward_data_up": [vp, i, i, i, i, i, vp, i, i, vp, i, vp, i, vp, i, f,
                                             vp],
            "sur_conv3x3_backward_weight_overlap": [vp, i, i, vp, i, vp, i, i, i, i, i, i, vp, vp,
                                                    vp, sz, vp, vp, vp],
            "sur_flip_weights": [i, ctypes.POINTER(vp), ctypes.POINTER(i), ctypes.POINTER(i),
                                 ctypes.POINTER(vp), vp],
            "sur_leaky_backward": [vp, i, vp, i, vp, i, ll, i, f, vp],
            "sur_pool2": [vp, i, i, i, i, i, vp, i, vp],
            "sur_pool2_backward": [vp, i, i, i, i, i, vp, i, i, vp],
            "sur_pool2_backward_act": [vp, i, i, i, i, i, vp, i, i, vp, i, f, vp],
            "sur_up2": [vp, i, i, i, i, i, vp, i, vp],
            "sur_up2_backward": [vp, i, i, i, i, i, vp, i, vp],
            "sur_up2_backward_act": [vp, i, i, i, i, i, vp, i, vp, i, f, vp],
            "sur_pack_input": [vp, i, i, i, vp, fp, vp, vp],
            "sur_apply_output": [vp, vp, i, i, i, fp, vp, vp],
            "sur_mse_loss": [vp, vp, vp, i, i, i, fp, vp, vp, vp, vp],
            "sur_adam": [vp, vp, vp, vp, vp, ll, i, f, f, f, f, vp],
            "sur_to_bf16": [vp, vp, ll, vp],
            "sur_crop_periodic": [vp, i, i, i, i, i, i, vp, vp],
        }
        for name, args in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_int
        dp = ctypes.POINTER(ctypes.c_double)
        lib.sslbm_params_from_rates.argtypes = [ctypes.c_double] * 4 + [dp, ctypes.c_double,
                                                                        ctypes.c_double, pp]
        lib.sslbm_params_from_rates.restype = ctypes.c_int
        lib.sslbm_rate_gradients.argtypes = [dp, ctypes.c_double, ctypes.c_double, dp]
        lib.sslbm_rate_gradients.restype = ctypes.c_int
        lib.sslbm_strerror.restype = ctypes.c_char_p
        lib.sslbm_destroy.argtypes = [vp]
        lib.sslbm_destroy.restype = None
        lib.sslbm_ensemble_destroy.argtypes = [vp]
        lib.sslbm_ensemble_destroy.restype = None
        lib.sslbm_model_destroy.argtypes = [vp]
        lib.sslbm_model_destroy.restype = None
        for name in ("sslbm_ensemble_offset", "sslbm_ensemble_elements"):
            getattr(lib, name).restype = ll
        lib.sslbm_ensemble_offset.argtypes = [vp, i]
        lib.sslbm_ensemble_elements.argtypes = [vp]
        lib.sslbm_checkpoint_count.argtypes = [ll, i]
        lib.sslbm_checkpoint_count.restype = ll
        lib.sslbm_adjoint_workspace_bytes.argtypes = [vp, i]
        lib.sslbm_adjoint_workspace_bytes.restype = ctypes.c_size_t
        lib.sslbm_fd4_workspace_bytes.argtypes = [vp]
        lib.sslbm_fd4_workspace_bytes.restype = ctypes.c_size_t
        lib.sur_conv3x3_backward_weight_workspace.argtypes = [i, i, i, i, i]
        lib.sur_conv3x3_backward_weight_workspace.restype = ctypes.c_size_t
        _LIB = lib
    return _LIB


def _strerror(status: int) -> str:
    try:
        return library().sslbm_strerror(status).decode()
    except Exception:  # library unavailable while formatting an error
        return "error"


# --------------------------------------------------------------- tensors --

def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class _Context:
    def __init__(self, nx: int, ny: int, params, dtype, bc):
        torch = _torch()
        if dtype in (torch.float32, "f32", "float32", F32):
            self.dtype, self.code = torch.float32, F32
        elif dtype in (torch.float64, "f64", "float64", F64):
            self.dtype, self.code = torch.float64, F64
        else:
            raise ValueError(f"unsupported dtype {dtype!r}")
        if bc not in _BC:
            raise ValueError(f"unknown boundary condition {bc!r}")
        self.nx, self.ny, self.bc = int(nx), int(ny), bc
        self.lib = library()
        h = ctypes.c_void_p()
        st = self.lib.sslbm_init(ctypes.byref(h), self.nx, self.ny, self.code, _BC[bc],
                                 ctypes.byref(Params.of(params)))
        if st != OK:
            raise SSLBMError(st, "sslbm_init")
        self.handle = h
        self.params = params

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.sslbm_destroy(h)
            self.handle = None

    def _check(self, st: int, what: str):
        if st != OK:
            raise SSLBMError(st, what, self.lib.sslbm_last_hip_error(self.handle))

    def _tensor(self, t, shape, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch tensor")
        if t.device.type != "cuda":
            raise ValueError(f"{name} must be on the GPU")
        if t.dtype != self.dtype:
            raise ValueError(f"{name} must be {self.dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return ctypes.c_void_p(t.data_ptr())

    def empty(self, *shape):
        return _torch().empty(shape, dtype=self.dtype, device="cuda")

    def set_params(self, params):
        self._check(self.lib.sslbm_set_params(self.handle, ctypes.byref(Params.of(params))),
                    "sslbm_set_params")
        self.params = params


class Solver(_Context):
    """SSLBM SEIRD solver on an nx-by-ny grid (HIP kernels, one GPU)."""

    def __init__(self, nx, ny, params, dtype="f64", bc="periodic", blocking: int = 0):
        super().__init__(nx, ny, params, dtype, bc)
        if blocking:
            self.set_blocking(blocking)

    @property
    def shape(self):
        return (5, self.ny, self.nx)

    def set_blocking(self, steps_per_pass: int):
        self._check(self.lib.sslbm_set_blocking(self.handle, int(steps_per_pass)),
                    "sslbm_set_blocking")

    @property
    def blocking(self) -> int:
        return self.lib.sslbm_get_blocking(self.handle)

    def set_launch(self, steps_per_pass=0, rows_per_wave=0, cols_per_lane=0):
        """Pass shape (0 = automatic); changes speed, never results."""
        shape = Launch(int(steps_per_pass), int(rows_per_wave), int(cols_per_lane))
        self._check(self.lib.sslbm_set_launch(self.handle, ctypes.byref(shape)),
                    "sslbm_set_launch")

    def launch(self) -> dict:
        """The pass shape sslbm_run uses, automatic fields resolved."""
        shape = Launch()
        self._check(self.lib.sslbm_get_launch(self.handle, ctypes.byref(shape)),
                    "sslbm_get_launch")
        return shape.as_dict()

    def tune(self, rho, scratch=None, stream=None) -> dict:
        """Time candidate pass shapes on `rho` (only read; `scratch` is
        overwritten) and keep the fastest; returns it."""
        if scratch is None:
            scratch = self.empty(*self.shape)
        a = self._tensor(rho, self.shape, "rho")
        b = self._tensor(scratch, self.shape, "scratch")
        best = Launch()
        self._check(self.lib.sslbm_tune(self.handle, a, b, _stream(stream), ctypes.byref(best)),
                    "sslbm_tune")
        return best.as_dict()

    def step(self, rho_in, rho_out=None, stream=None):
        """One time step rho_in -> rho_out (allocated when not given)."""
        if rho_out is None:
            rho_out = self.empty(*self.shape)
        a = self._tensor(rho_in, self.shape, "rho_in")
        b = self._tensor(rho_out, self.shape, "rho_out")
        self._check(self.lib.sslbm_step(self.handle, a, b, _stream(stream)), "sslbm_step")
        return rho_out

    def run(self, rho, nsteps: int, scratch=None, stream=None):
        """nsteps time steps in place in rho; scratch (same shape) is clobbered."""
        if scratch is None:
            scratch = self.empty(*self.shape)
        a = self._tensor(rho, self.shape, "rho")
        b = self._tensor(scratch, self.shape, "scratch")
        self._check(self.lib.sslbm_run(self.handle, a, b, int(nsteps), _stream(stream)),
                    "sslbm_run")
        return rho

    def plan(self, nsteps: int) -> dict:
        """How `run` splits nsteps into passes with the current pass shape:
        {"passes", "longest", "shortest"} (host only)."""
        n, hi, lo = ctypes.c_longlong(), ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.sslbm_plan_run(self.handle, int(nsteps), ctypes.byref(n),
                                            ctypes.byref(hi), ctypes.byref(lo)),
                    "sslbm_plan_run")
        return {"passes": n.value, "longest": hi.value, "shortest": lo.value}

    def total(self, rho, stream=None):
        """Per-compartment totals (5 floats, FP64 sums); waits for the stream."""
        out = (ctypes.c_double * 5)()
        a = self._tensor(rho, self.shape, "rho")
        self._check(self.lib.sslbm_total(self.handle, a, out, _stream(stream)), "sslbm_total")
        return [out[i] for i in range(5)]

    # ---------------------------------------------- finite-difference reference --
    def fd4_workspace_bytes(self) -> int:
        return int(self.lib.sslbm_fd4_workspace_bytes(self.handle))

    def fd4_run(self, rho, nsteps: int, work=None, stream=None):
        """nsteps steps of the fourth-order finite-difference / RK4 reference
        solver (Sec. III) in place in rho; work (uint8, at least
        fd4_workspace_bytes()) is clobbered."""
        torch = _torch()
        need = self.fd4_workspace_bytes()
        if work is None:
            work = torch.empty(need, dtype=torch.uint8, device="cuda")
        if (not isinstance(work, torch.Tensor) or work.device.type != "cuda"
                or not work.is_contiguous()):
            raise ValueError("work must be a contiguous GPU tensor")
        nbytes = work.numel() * work.element_size()
        a = self._tensor(rho, self.shape, "rho")
        self._check(self.lib.sslbm_fd4_run(self.handle, a, ctypes.c_void_p(work.data_ptr()),
                                           nbytes, int(nsteps), _stream(stream)),
                    "sslbm_fd4_run")
        return rho

    # ------------------------------------------------------------ adjoint --
    def _grad(self, grad):
        torch = _torch()
        if grad is None:
            grad = torch.zeros(GRAD_COUNT, dtype=torch.float64, device="cuda")
        if (not isinstance(grad, torch.Tensor) or grad.device.type != "cuda"
                or grad.dtype != torch.float64 or tuple(grad.shape) != (GRAD_COUNT,)
                or not grad.is_contiguous()):
            raise ValueError("grad must be a contiguous float64 GPU tensor of 9 elements")
        return grad

    def adjoint_step(self, rho, lam_next, lam_out=None, grad=None, stream=None):
        """One reverse step at state rho: returns (lam_out, grad) with
        lam_out = dJ/d rho(t) and the step's dJ/d(beta, alpha, gamma, phi,
        d[0..4]) added to grad (float64, 9, zeros when not given)."""
        if lam_out is None:
            lam_out = self.empty(*self.shape)
        grad = self._grad(grad)
        a = self._tensor(rho, self.shape, "rho")
        b = self._tensor(lam_next, self.shape, "lam_next")
        c = self._tensor(lam_out, self.shape, "lam_out")
        self._check(self.lib.sslbm_adjoint_step(self.handle, a, b, c,
                                                ctypes.c_void_p(grad.data_ptr()),
                                                _stream(stream)), "sslbm_adjoint_step")
        return lam_out, grad

    def checkpoint_count(self, nsteps: int, every: int) -> int:
        n = self.lib.sslbm_checkpoint_count(int(nsteps), int(every))
        if n < 0:
            raise ValueError("nsteps must be >= 0 and every >= 1")
        return n

    def run_checkpointed(self, rho, nsteps: int, every: int, checkpoints=None, scratch=None,
                         stream=None):
        """nsteps steps in place in rho, storing the state every `every` steps
        (steps 0, every, ...). Returns the checkpoints tensor."""
        count = self.checkpoint_count(nsteps, every)
        if checkpoints is None:
            checkpoints = self.empty(max(count, 1), *self.shape)
        if scratch is None:
            scratch = self.empty(*self.shape)
        a = self._tensor(rho, self.shape, "rho")
        b = self._tensor(scratch, self.shape, "scratch")
        if (tuple(checkpoints.shape[1:]) != self.shape or checkpoints.shape[0] < count
                or checkpoints.dtype != self.dtype or not checkpoints.is_contiguous()
                or checkpoints.device.type != "cuda"):
            raise ValueError(f"checkpoints must be a contiguous GPU tensor of >= {count} states")
        self._check(self.lib.sslbm_run_checkpointed(
            self.handle, a, b, int(nsteps), int(every), ctypes.c_void_p(checkpoints.data_ptr()),
            _stream(stream)), "sslbm_run_checkpointed")
        return checkpoints

    def adjoint_workspace_bytes(self, every: int) -> int:
        n = self.lib.sslbm_adjoint_workspace_bytes(self.handle, int(every))
        if n == 0:
            raise ValueError("every must be >= 1")
        return n

    def adjoint_run(self, checkpoints, nsteps: int, every: int, lam, grad=None, workspace=None,
                    stream=None):
        """Reverse sweep of a run recorded by run_checkpointed: lam holds
        dJ/d rho(T) on entry and dJ/d rho(0) on return; the parameter gradient
        is added to grad. Returns (lam, grad)."""
        torch = _torch()
        count = self.checkpoint_count(nsteps, every)
        if (checkpoints.shape[0] < count or tuple(checkpoints.shape[1:]) != self.shape
                or checkpoints.dtype != self.dtype or not checkpoints.is_contiguous()
                or checkpoints.device.type != "cuda"):
            raise ValueError(f"checkpoints must hold >= {count} states of shape {self.shape}")
        need = self.adjoint_workspace_bytes(every)
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
        if workspace.numel() * workspace.element_size() < need or workspace.device.type != "cuda":
            raise ValueError(f"workspace must be a GPU tensor of at least {need} bytes")
        grad = self._grad(grad)
        a = self._tensor(lam, self.shape, "lam")
        self._check(self.lib.sslbm_adjoint_run(
            self.handle, ctypes.c_void_p(checkpoints.data_ptr()), int(nsteps), int(every), a,
            ctypes.c_void_p(grad.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
            _stream(stream)), "sslbm_adjoint_run")
        return lam, grad


class BGK(_Context):
    """BGK lattice Boltzmann comparison scheme on the same grid (HIP kernels)."""

    def __init__(self, nx, ny, params, dtype="f64", bc="periodic"):
        super().__init__(nx, ny, params, dtype, bc)

    @property
    def f_shape(self):
        return (4, 5, self.ny, self.nx)

    def init(self, rho, stream=None):
        f = self.empty(*self.f_shape)
        rd = self.empty(self.ny, self.nx)
        self._check(self.lib.bgk_init(self.handle, self._tensor(rho, (5, self.ny, self.nx), "rho"),
                                      self._tensor(f, self.f_shape, "f"),
                                      self._tensor(rd, (self.ny, self.nx), "rhoD"),
                                      _stream(stream)), "bgk_init")
        return f, rd

    def step(self, f, rhoD, f_out=None, rhoD_out=None, stream=None):
        if f_out is None:
            f_out = self.empty(*self.f_shape)
        if rhoD_out is None:
            rhoD_out = self.empty(self.ny, self.nx)
        plane = (self.ny, self.nx)
        self._check(self.lib.bgk_step(self.handle, self._tensor(f, self.f_shape, "f"),
                                      self._tensor(rhoD, plane, "rhoD"),
                                      self._tensor(f_out, self.f_shape, "f_out"),
                                      self._tensor(rhoD_out, plane, "rhoD_out"),
                                      _stream(stream)), "bgk_step")
        return f_out, rhoD_out

    def run(self, f, rhoD, nsteps: int, f_scratch=None, rhoD_scratch=None, stream=None):
        if f_scratch is None:
            f_scratch = self.empty(*self.f_shape)
        if rhoD_scratch is None:
            rhoD_scratch = self.empty(self.ny, self.nx)
        plane = (self.ny, self.nx)
        self._check(self.lib.bgk_run(self.handle, self._tensor(f, self.f_shape, "f"),
                                     self._tensor(rhoD, plane, "rhoD"),
                                     self._tensor(f_scratch, self.f_shape, "f_scratch"),
                                     self._tensor(rhoD_scratch, plane, "rhoD_scratch"),
                                     int(nsteps), _stream(stream)), "bgk_run")
        return f, rhoD

    def density(self, f, rhoD, rho=None, stream=None):
        if rho is None:
            rho = self.empty(5, self.ny, self.nx)
        plane = (self.ny, self.nx)
        self._check(self.lib.bgk_density(self.handle, self._tensor(f, self.f_shape, "f"),
                                         self._tensor(rhoD, plane, "rhoD"),
                                         self._tensor(rho, (5, self.ny, self.nx), "rho"),
                                         _stream(stream)), "bgk_density")
        return rho


RUN_GRAPH = 1


class Ensemble:
    """Many independent SSLBM grids of different sizes and parameters,
    advanced together: size classes side by side (instances of at most 80 KiB
    held in LDS for the whole run, the others in passes with a shape per
    class), optionally captured as one HIP graph per run.

    The state is one flat tensor of ``elements`` values; ``views(state)``
    gives the (5, ny_i, nx_i) block of every instance."""

    def __init__(self, sizes, params, dtype="f32", bc="periodic"):
        torch = _torch()
        if dtype in (torch.float32, "f32", "float32", F32):
            self.dtype, self.code = torch.float32, F32
        elif dtype in (torch.float64, "f64", "float64", F64):
            self.dtype, self.code = torch.float64, F64
        else:
            raise ValueError(f"unsupported dtype {dtype!r}")
        if bc not in _BC:
            raise ValueError(f"unknown boundary condition {bc!r}")
        sizes = [(int(nx), int(ny)) for nx, ny in sizes]
        params = list(params)
        if len(sizes) != len(params) or not sizes:
            raise ValueError("need one parameter set per instance")
        n = len(sizes)
        self.lib = library()
        nx = (ctypes.c_int * n)(*[s[0] for s in sizes])
        ny = (ctypes.c_int * n)(*[s[1] for s in sizes])
        ps = (Params * n)(*[Params.of(p) for p in params])
        bad = ctypes.c_int(-1)
        h = ctypes.c_void_p()
        st = self.lib.sslbm_ensemble_create(ctypes.byref(h), n, nx, ny, self.code, _BC[bc], ps,
                                            ctypes.byref(bad))
        if st != OK:
            raise SSLBMError(st, f"sslbm_ensemble_create (instance {bad.value})")
        self.handle = h
        self.sizes = sizes
        self.params = params
        self.bc = bc
        self.offsets = [self.lib.sslbm_ensemble_offset(h, i) for i in range(n)]
        self.elements = self.lib.sslbm_ensemble_elements(h)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.sslbm_ensemble_destroy(h)
            self.handle = None

    def _check(self, st, what):
        if st != OK:
            raise SSLBMError(st, what, self.lib.sslbm_ensemble_last_hip_error(self.handle))

    def empty(self):
        return _torch().empty(self.elements, dtype=self.dtype, device="cuda")

    def views(self, state):
        return [state[o:o + 5 * ny * nx].view(5, ny, nx)
                for o, (nx, ny) in zip(self.offsets, self.sizes)]

    def _flat(self, t, name):
        torch = _torch()
        if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != self.dtype:
            raise ValueError(f"{name} must be a {self.dtype} tensor on the GPU")
        if t.numel() != self.elements or not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous with {self.elements} elements")
        return ctypes.c_void_p(t.data_ptr())

    def set_launch(self, steps_per_pass=0, rows_per_wave=0, cols_per_lane=0):
        shape = Launch(int(steps_per_pass), int(rows_per_wave), int(cols_per_lane))
        self._check(self.lib.sslbm_ensemble_set_launch(self.handle, ctypes.byref(shape)),
                    "sslbm_ensemble_set_launch")

    def launch(self) -> dict:
        shape = Launch()
        self._check(self.lib.sslbm_ensemble_get_launch(self.handle, ctypes.byref(shape)),
                    "sslbm_ensemble_get_launch")
        return shape.as_dict()

    def tune(self, state, scratch=None, stream=None) -> dict:
        """Time candidate pass shapes of every march class on `state`
        (unchanged), keep the fastest per class; returns the largest class's."""
        if scratch is None:
            scratch = self.empty()
        best = Launch()
        self._check(self.lib.sslbm_ensemble_tune(self.handle, self._flat(state, "state"),
                                                 self._flat(scratch, "scratch"), _stream(stream),
                                                 ctypes.byref(best)), "sslbm_ensemble_tune")
        return best.as_dict()

    def classes(self) -> list:
        """Every size class: on_chip, instances, cells, max_side, launch."""
        out = []
        for c in range(self.lib.sslbm_ensemble_class_count(self.handle)):
            info = EnsembleClass()
            self._check(self.lib.sslbm_ensemble_class_info(self.handle, c, ctypes.byref(info)),
                        "sslbm_ensemble_class_info")
            out.append(info.as_dict())
        return out

    def instance_class(self, instance: int) -> int:
        c = self.lib.sslbm_ensemble_instance_class(self.handle, int(instance))
        if c < 0:
            raise SSLBMError(c, "sslbm_ensemble_instance_class")
        return c

    def set_class_launch(self, cls, steps_per_pass=0, rows_per_wave=0, cols_per_lane=0):
        shape = Launch(int(steps_per_pass), int(rows_per_wave), int(cols_per_lane))
        self._check(self.lib.sslbm_ensemble_set_class_launch(self.handle, int(cls),
                                                             ctypes.byref(shape)),
                    "sslbm_ensemble_set_class_launch")

    def run_class(self, cls, state, nsteps: int, scratch=None, stream=None):
        """nsteps steps of the instances of class `cls` only."""
        if scratch is None:
            scratch = self.empty()
        self._check(self.lib.sslbm_ensemble_run_class(self.handle, int(cls),
                                                      self._flat(state, "state"),
                                                      self._flat(scratch, "scratch"),
                                                      int(nsteps), _stream(stream)),
                    "sslbm_ensemble_run_class")
        return state

    def run(self, state, nsteps: int, scratch=None, graph: bool = False, stream=None):
        if scratch is None:
            scratch = self.empty()
        flags = RUN_GRAPH if graph else 0
        self._check(self.lib.sslbm_ensemble_run(self.handle, self._flat(state, "state"),
                                                self._flat(scratch, "scratch"), int(nsteps),
                                                flags, _stream(stream)), "sslbm_ensemble_run")
        return state


class Model:
    """A generic compartmental model (inputs.GenericModel) on an nx-by-ny
    grid: D2Q5 or D2Q9, up to 8 compartments, transition-list sources."""

    def __init__(self, nx, ny, model, dtype="f64", bc="periodic"):
        torch = _torch()
        self.lib = library()
        if dtype in (torch.float32, "f32", "float32", F32):
            self.dtype, self.code = torch.float32, F32
        elif dtype in (torch.float64, "f64", "float64", F64):
            self.dtype, self.code = torch.float64, F64
        else:
            raise ValueError(f"unsupported dtype {dtype!r}")
        if bc not in _BC:
            raise ValueError(f"unknown boundary condition {bc!r}")
        self.nx, self.ny, self.model = int(nx), int(ny), model
        m = len(model.d)
        d = (ctypes.c_double * m)(*model.d)
        counted = (ctypes.c_int * m)(*[int(v) for v in model.counted])
        tr = (Transition * max(len(model.transitions), 1))(
            *[Transition(int(t[0]), int(t[1]), int(t[2]), int(t[4]), float(t[3]))
              for t in model.transitions])
        h = ctypes.c_void_p()
        st = self.lib.sslbm_model_create(ctypes.byref(h), self.nx, self.ny, self.code, _BC[bc],
                                         int(model.lattice), m, d, counted, float(model.dx),
                                         float(model.dt), len(model.transitions), tr)
        if st != OK:
            raise SSLBMError(st, "sslbm_model_create")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            self.lib.sslbm_model_destroy(h)
            self.handle = None

    @property
    def shape(self):
        return (len(self.model.d), self.ny, self.nx)

    def _check(self, st, what):
        if st != OK:
            raise SSLBMError(st, what, self.lib.sslbm_model_last_hip_error(self.handle))

    def _t(self, t, name):
        torch = _torch()
        if (not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != self.dtype
                or tuple(t.shape) != self.shape or not t.is_contiguous()):
            raise ValueError(f"{name} must be a contiguous {self.dtype} GPU tensor of shape "
                             f"{self.shape}")
        return ctypes.c_void_p(t.data_ptr())

    def set_blocking(self, steps_per_pass: int = 0):
        """Steps per pass of run() (0 = automatic); changes speed, never results."""
        self._check(self.lib.sslbm_model_set_blocking(self.handle, int(steps_per_pass)),
                    "sslbm_model_set_blocking")

    @property
    def blocking(self) -> int:
        """Steps per pass run() uses, automatic choice resolved."""
        k = ctypes.c_int()
        self._check(self.lib.sslbm_model_get_blocking(self.handle, ctypes.byref(k)),
                    "sslbm_model_get_blocking")
        return k.value

    def step(self, rho_in, rho_out=None, stream=None):
        torch = _torch()
        if rho_out is None:
            rho_out = torch.empty(self.shape, dtype=self.dtype, device="cuda")
        self._check(self.lib.sslbm_model_step(self.handle, self._t(rho_in, "rho_in"),
                                              self._t(rho_out, "rho_out"), _stream(stream)),
                    "sslbm_model_step")
        return rho_out

    def run(self, rho, nsteps: int, scratch=None, stream=None):
        torch = _torch()
        if scratch is None:
            scratch = torch.empty(self.shape, dtype=self.dtype, device="cuda")
        self._check(self.lib.sslbm_model_run(self.handle, self._t(rho, "rho"),
                                             self._t(scratch, "scratch"), int(nsteps),
                                             _stream(stream)), "sslbm_model_run")
        return rho
