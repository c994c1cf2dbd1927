"""The C-ABI library on the CPU: it loads, exports what include/sslbm.h
declares, and rejects bad arguments on the host before any HIP call."""
import ctypes
import math
import re
from pathlib import Path

import numpy as np
import pytest

from paper_2603_19789_amd import binding
from paper_2603_19789_amd.binding import Params
from paper_2603_19789_amd.inputs import c1_params

SIG_RE = re.compile(r"^\s*(?:sslbm_status|int|void|long\s+long|size_t|const\s+char\s*\*)\s*\**\s*(\w+)\s*\(",
                    re.M)


@pytest.fixture(scope="module")
def lib():
    return binding.library()


def declared_functions():
    text = binding.HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(SIG_RE.findall(text)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for required in ("sslbm_init", "sslbm_step", "sslbm_run", "bgk_step", "bgk_init",
                     "bgk_run", "bgk_density", "sslbm_total", "sslbm_destroy",
                     "sslbm_set_params", "sslbm_set_blocking", "sslbm_get_blocking",
                     "sslbm_set_launch", "sslbm_get_launch",
                     "sslbm_strerror", "sslbm_last_hip_error", "sslbm_adjoint_step",
                     "sslbm_run_checkpointed", "sslbm_adjoint_run", "sslbm_checkpoint_count",
                     "sslbm_adjoint_workspace_bytes", "sslbm_ensemble_run"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def _init(lib, nx=8, ny=8, dtype=binding.F64, bc=binding.PERIODIC, p=None):
    h = ctypes.c_void_p()
    params = Params.of(p if p is not None else c1_params())
    st = lib.sslbm_init(ctypes.byref(h), nx, ny, dtype, bc, ctypes.byref(params))
    return st, h


def test_valid_init_and_destroy(lib):
    st, h = _init(lib)
    assert st == binding.OK and h.value
    assert lib.sslbm_get_blocking(h) >= 1
    assert lib.sslbm_last_hip_error(h) == 0
    lib.sslbm_destroy(h)
    lib.sslbm_destroy(None)


@pytest.mark.parametrize("nx,ny,dtype,bc", [
    (0, 8, binding.F64, binding.PERIODIC), (8, -1, binding.F64, binding.PERIODIC),
    ((1 << 20) + 1, 8, binding.F64, binding.PERIODIC), (8, 8, 2, binding.PERIODIC),
    (8, 8, binding.F32, 7),
])
def test_init_rejects_bad_grid(lib, nx, ny, dtype, bc):
    st, h = _init(lib, nx, ny, dtype, bc)
    assert st == binding.E_ARG and not h.value


def test_init_rejects_null(lib):
    h = ctypes.c_void_p()
    assert lib.sslbm_init(ctypes.byref(h), 8, 8, 0, 0, None) == binding.E_ARG
    assert lib.sslbm_init(None, 8, 8, 0, 0, ctypes.byref(Params.of(c1_params()))) == binding.E_ARG


@pytest.mark.parametrize("change", [
    dict(beta=-0.1), dict(alpha=math.nan), dict(gamma=math.inf), dict(phi=1.5), dict(phi=-0.1),
    dict(dx=0.0), dict(dt=-0.01), dict(dt=math.nan), dict(d=(0.1, -1e-3, 0.1, 0.1, 0.0)),
    dict(d=(0.1, 0.1, math.nan, 0.1, 0.0)),
])
def test_init_rejects_bad_parameters(lib, change):
    st, _ = _init(lib, p=c1_params().with_(**change))
    assert st == binding.E_ARG


def test_diffusion_stability_limit(lib):
    """d_lu = d dt / dx^2 must stay in [0, 1/4]."""
    p = c1_params()
    ok = p.with_(d=(25.0, 0.0, 0.0, 0.0, 0.0))          # d_lu = 0.25
    bad = p.with_(d=(25.01, 0.0, 0.0, 0.0, 0.0))        # d_lu > 0.25
    assert _init(lib, p=ok)[0] == binding.OK
    assert _init(lib, p=bad)[0] == binding.E_UNSTABLE


def test_reaction_stability_limit(lib):
    """dt |lambda_2| + 8 max(d_lu^E, d_lu^I) <= 2, lambda_2 from Eq. (eigenvalues)."""
    p = c1_params().with_(d=(0.0,) * 5)
    a, g, b = p.alpha, p.gamma, p.beta
    lam2 = abs(0.5 * (-(a + g) - math.sqrt((a - g) ** 2 + 4 * a * b)))
    assert _init(lib, p=p.with_(dt=1.99 / lam2))[0] == binding.OK
    assert _init(lib, p=p.with_(dt=2.01 / lam2))[0] == binding.E_UNSTABLE
    # with diffusion of E the margin shrinks by 8 d_lu
    dt = 1.0 / lam2
    d_e = 0.13 / dt  # d_lu^E = 0.13 -> 1 + 1.04 > 2
    assert _init(lib, p=p.with_(dt=dt, d=(0.0, d_e, 0.0, 0.0, 0.0)))[0] == binding.E_UNSTABLE


def test_aliasing_and_argument_errors_before_any_gpu_call(lib):
    st, h = _init(lib, 16, 8)
    assert st == binding.OK
    nbytes = 5 * 16 * 8 * 8
    a = ctypes.c_void_p(0x100000)
    b = ctypes.c_void_p(0x100000 + nbytes - 8)       # overlaps a
    c = ctypes.c_void_p(0x100000 + nbytes)           # adjacent, no overlap
    assert lib.sslbm_step(h, a, b, None) == binding.E_ALIAS
    assert lib.sslbm_step(h, a, None, None) == binding.E_ARG
    assert lib.sslbm_run(h, a, b, 5, None) == binding.E_ALIAS
    assert lib.sslbm_run(h, a, c, -1, None) == binding.E_ARG
    assert lib.sslbm_run(h, a, c, 0, None) == binding.OK   # nothing to do, no HIP call
    assert lib.sslbm_tune(h, a, b, None, None) == binding.E_ALIAS
    assert lib.sslbm_tune(h, a, None, None, None) == binding.E_ARG
    assert lib.sslbm_tune(None, a, c, None, None) == binding.E_ARG
    out = (ctypes.c_double * 5)()
    assert lib.sslbm_total(h, None, out, None) == binding.E_ARG
    assert lib.sslbm_set_blocking(h, -1) == binding.E_ARG
    assert lib.sslbm_set_blocking(h, binding.MAX_BLOCKING + 1) == binding.E_ARG
    assert lib.sslbm_set_blocking(h, 3) == binding.OK
    assert lib.sslbm_get_blocking(h) == 3
    assert lib.sslbm_set_blocking(h, 0) == binding.OK
    L = binding.Launch
    for bad in (L(0, -1, 0), L(0, 65537, 0), L(-1, 0, 0), L(9, 0, 0), L(0, 0, 3), L(0, 0, -1)):
        assert lib.sslbm_set_launch(h, ctypes.byref(bad)) == binding.E_ARG
    assert lib.sslbm_set_launch(h, ctypes.byref(L(2, 40, 2))) == binding.OK
    got = L()
    assert lib.sslbm_get_launch(h, ctypes.byref(got)) == binding.OK
    assert got.as_dict() == L(2, 40, 2).as_dict()
    # FP64 beyond the register budget of one wavefront
    assert lib.sslbm_set_launch(h, ctypes.byref(L(6, 0, 1))) == binding.E_UNSUPPORTED
    assert lib.sslbm_set_launch(h, ctypes.byref(L(3, 0, 2))) == binding.E_UNSUPPORTED
    assert lib.sslbm_set_launch(h, ctypes.byref(L(5, 0, 1))) == binding.OK
    assert lib.sslbm_set_launch(h, ctypes.byref(L(0, 0, 0))) == binding.OK
    assert lib.sslbm_get_launch(h, ctypes.byref(got)) == binding.OK
    assert got.steps_per_pass >= 1 and got.rows_per_wave >= 1 and got.cols_per_lane in (1, 2)
    lib.sslbm_destroy(h)


def test_bgk_rejects_diffusing_deceased(lib):
    p = c1_params().with_(d=(0.1, 0.1, 0.1, 0.1, 0.1))
    st, h = _init(lib, p=p)
    assert st == binding.OK  # the SSLBM supports a diffusing D
    a, b = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x900000)
    assert lib.bgk_step(h, a, b, a, b, None) == binding.E_UNSUPPORTED
    assert lib.bgk_init(h, a, b, a, None) == binding.E_UNSUPPORTED
    lib.sslbm_destroy(h)


def test_bgk_aliasing(lib):
    st, h = _init(lib, 8, 8)
    pb = 8 * 8 * 8
    f_in, d_in = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x100000 + 20 * pb)
    f_out = ctypes.c_void_p(0x100000 + 10 * pb)  # overlaps f_in
    d_out = ctypes.c_void_p(0x900000)
    assert lib.bgk_step(h, f_in, d_in, f_out, d_out, None) == binding.E_ALIAS
    assert lib.bgk_run(h, f_in, d_in, f_out, d_out, 3, None) == binding.E_ALIAS
    lib.sslbm_destroy(h)


def test_set_params_revalidates(lib):
    st, h = _init(lib)
    assert lib.sslbm_set_params(h, ctypes.byref(Params.of(c1_params().with_(beta=-1.0)))) \
        == binding.E_ARG
    assert lib.sslbm_set_params(h, ctypes.byref(Params.of(c1_params()))) == binding.OK
    lib.sslbm_destroy(h)


def test_strerror(lib):
    for code in (0, -1, -2, -3, -4, -5, -6, 42):
        assert lib.sslbm_strerror(code)


def test_python_solver_raises_on_bad_parameters():
    with pytest.raises(binding.SSLBMError) as exc:
        binding.Solver(8, 8, c1_params().with_(d=(100.0,) * 5))
    assert exc.value.status == binding.E_UNSTABLE


def test_adjoint_host_checks(lib):
    """Reverse-mode entry points: counts, workspace size and argument errors,
    all decided on the host."""
    assert lib.sslbm_checkpoint_count(0, 100) == 0
    assert lib.sslbm_checkpoint_count(2000, 100) == 20
    assert lib.sslbm_checkpoint_count(2001, 100) == 21
    assert lib.sslbm_checkpoint_count(5, 0) == -1
    assert lib.sslbm_checkpoint_count(-1, 3) == -1
    st, h = _init(lib, 130, 45, binding.F64)
    assert st == binding.OK
    state = 5 * 130 * 45 * 8
    ws = lib.sslbm_adjoint_workspace_bytes(h, 10)
    assert ws >= (9 // 2 + 1) * state and ws % 256 == 0  # every second state, and one field
    assert lib.sslbm_adjoint_workspace_bytes(h, 0) == 0
    assert lib.sslbm_adjoint_workspace_bytes(None, 10) == 0
    vp = ctypes.c_void_p
    a, b, c, g, w = (vp(0x100000000 * k) for k in (1, 2, 3, 4, 5))
    assert lib.sslbm_adjoint_step(h, None, b, c, g, None) == binding.E_ARG
    assert lib.sslbm_adjoint_step(h, a, b, c, None, None) == binding.E_ARG
    assert lib.sslbm_adjoint_step(h, a, b, b, g, None) == binding.E_ALIAS
    assert lib.sslbm_adjoint_step(h, a, b, a, g, None) == binding.E_ALIAS
    assert lib.sslbm_adjoint_step(h, a, b, c, vp(c.value + 8), None) == binding.E_ALIAS
    assert lib.sslbm_run_checkpointed(h, a, b, 10, 0, c, None) == binding.E_ARG
    assert lib.sslbm_run_checkpointed(h, a, b, -1, 5, c, None) == binding.E_ARG
    assert lib.sslbm_run_checkpointed(h, a, b, 30, 10, vp(a.value - state), None) == binding.E_ALIAS
    assert lib.sslbm_adjoint_run(h, a, 10, 0, b, g, w, None) == binding.E_ARG
    assert lib.sslbm_adjoint_run(h, a, 10, 5, b, g, None, None) == binding.E_ARG
    assert lib.sslbm_adjoint_run(h, a, 10, 5, vp(w.value + 64), g, w, None) == binding.E_ALIAS
    assert lib.sslbm_adjoint_run(h, a, 10, 5, b, vp(w.value + 8), w, None) == binding.E_ALIAS
    # nothing to do for a run of zero steps: no GPU call is made
    assert lib.sslbm_adjoint_run(h, a, 0, 5, b, g, w, None) == binding.OK
    lib.sslbm_destroy(h)


S_OUT_F32 = 2  # surrogate.h: SUR_OUT_F32


def test_surrogate_header_exports_and_host_checks(lib):
    """surrogate.h: every declared function is exported, and bad arguments
    are rejected on the host (no GPU call is made for them)."""
    text = re.sub(r"/\*.*?\*/", "", (binding.HEADER.parent / "surrogate.h").read_text(), flags=re.S)
    names = sorted(set(SIG_RE.findall(text)))
    assert "sur_conv3x3_forward" in names and "sur_adam" in names
    for name in names:
        assert hasattr(lib, name), name
    vp = ctypes.c_void_p
    a, b, c = vp(0x100000000), vp(0x200000000), vp(0x300000000)
    fwd = lib.sur_conv3x3_forward
    assert fwd(a, 16, 1, 8, 8, 16, b, None, c, 16, 32, 0, 0.1, None) == binding.E_ARG  # pitch < cout
    assert fwd(vp(a.value + 2), 16, 1, 8, 8, 16, b, None, c, 32, 32, 0, 0.1, None) == binding.E_ARG
    assert fwd(a, 16, 1, 8, 8, 12, b, None, c, 32, 32, 0, 0.1, None) == binding.E_ARG  # cin % 8
    assert fwd(a, 16, 0, 8, 8, 16, b, None, c, 32, 32, 0, 0.1, None) == binding.E_ARG
    assert fwd(a, 16, 1, 8, 8, 16, b, None, c, 32, 32, 4, 0.1, None) == binding.E_ARG  # flags
    # the input view must span less than 2 GiB (32-bit byte offsets):
    # (1 x 8192 x 8192 pixels - 1) x pitch 16 + 16 channels = 2^31 bytes
    assert fwd(a, 16, 1, 8192, 8192, 16, b, None, c, 32, 32, 0, 0.1, None) == binding.E_ARG
    assert lib.sur_conv3x3_backward_data(a, 16, 1, 8192, 8192, 16, b, 8, c, 8, vp(0x400000000),
                                         None) == binding.E_ARG
    # fused pooling: BF16 output only, even sizes, an aligned pooled view
    d = vp(0x400000000)
    fp = lib.sur_conv3x3_forward_pool
    assert fp(a, 16, 1, 8, 8, 16, b, None, c, 32, 32, S_OUT_F32, 0.1, d, 32, None) == binding.E_ARG
    assert fp(a, 16, 1, 7, 8, 16, b, None, c, 32, 32, 0, 0.1, d, 32, None) == binding.E_ARG
    assert fp(a, 16, 1, 8, 8, 16, b, None, c, 32, 32, 0, 0.1, None, 32, None) == binding.E_ARG
    assert fp(a, 16, 1, 8, 8, 16, b, None, c, 32, 32, 0, 0.1, vp(d.value + 2), 32,
              None) == binding.E_ARG
    assert fp(a, 16, 1, 8, 8, 16, b, None, c, 32, 32, 0, 0.1, d, 24, None) == binding.E_ARG
    # upsampled input: cu a multiple of 32 below cin, even sizes, BF16 output;
    # images under 8 x 32 pixels are left to the caller
    fu = lib.sur_conv3x3_forward_up
    assert fu(a, 16, 16, d, 32, 1, 8, 32, 48, b, None, c, 32, 32, 0, 0.1, None) == binding.E_ARG
    assert fu(a, 32, 32, d, 16, 1, 8, 32, 32, b, None, c, 32, 32, 0, 0.1, None) == binding.E_ARG
    assert fu(a, 32, 32, d, 16, 1, 9, 32, 48, b, None, c, 32, 32, 0, 0.1, None) == binding.E_ARG
    assert fu(a, 32, 32, d, 16, 1, 8, 32, 48, b, None, c, 32, 32, S_OUT_F32, 0.1,
              None) == binding.E_ARG
    assert fu(a, 32, 32, d, 16, 1, 6, 32, 48, b, None, c, 32, 32, 0, 0.1,
              None) == binding.E_UNSUPPORTED
    assert fu(a, 32, 32, d, 16, 1, 8, 16, 48, b, None, c, 32, 32, 0, 0.1,
              None) == binding.E_UNSUPPORTED
    assert lib.sur_conv3x3_backward_weight_workspace(1, 8, 12, 16, 16) == 0  # w % 8
    assert lib.sur_conv3x3_backward_weight_workspace(1, 8, 16, 16, 16) > 0
    ws = lib.sur_conv3x3_backward_weight_workspace(2, 8, 16, 32, 64)
    assert lib.sur_conv3x3_backward_weight(a, 32, b, 64, 2, 8, 16, 32, 64, c, None, vp(0x400000000),
                                           ws - 1, None) == binding.E_ARG
    assert lib.sur_pool2(a, 16, 1, 7, 8, 16, b, 16, None) == binding.E_ARG  # odd height
    bad = (ctypes.c_float * 5)(1, 1, 0, 1, 1)
    assert lib.sur_pack_input(a, 1, 8, 8, b, bad, c, None) == binding.E_ARG
    assert lib.sur_adam(a, None, b, c, vp(0x500000000), 10, 0, 1e-3, 0.9, 0.999, 1e-8,
                        None) == binding.E_ARG  # step 0
    assert lib.sur_adam(a, None, b, c, vp(0x500000000), 10, 1, 1e-3, 1.0, 0.999, 1e-8,
                        None) == binding.E_ARG  # beta1 = 1
    # several layers' backward-data weights: 1..32 layers, valid shapes,
    # 16-byte aligned outputs
    ptrs = (vp * 33)(*([b] * 33))
    outs = (vp * 33)(*([c] * 33))
    ints = (ctypes.c_int * 33)(*([16] * 33))
    flip = lib.sur_flip_weights
    assert flip(0, ptrs, ints, ints, outs, None) == binding.E_ARG
    assert flip(33, ptrs, ints, ints, outs, None) == binding.E_ARG
    assert flip(2, ptrs, ints, ints, None, None) == binding.E_ARG
    assert flip(1, ptrs, (ctypes.c_int * 1)(0), ints, outs, None) == binding.E_ARG
    assert flip(1, ptrs, ints, ints, (vp * 1)(vp(c.value + 2)), None) == binding.E_ARG
    # backward data on pre-flipped weights through an activation: the
    # activation view's channels and alignment, a finite slope
    bdf = lib.sur_conv3x3_backward_data_flipped
    assert bdf(a, 16, 1, 8, 8, 16, b, 8, c, 8, d, 4, 0.1, None) == binding.E_ARG  # pitch < cin
    assert bdf(a, 16, 1, 8, 8, 16, b, 8, c, 8, vp(d.value + 2), 8, 0.1, None) == binding.E_ARG
    assert bdf(a, 16, 1, 8, 8, 16, b, 8, c, 8, d, 8, float("nan"), None) == binding.E_ARG
    assert bdf(a, 16, 1, 8, 8, 16, vp(b.value + 2), 8, c, 8, None, 0, 0.1, None) == binding.E_ARG
    assert bdf(a, 16, 1, 8192, 8192, 16, b, 8, c, 8, None, 0, 0.1, None) == binding.E_ARG
    # backward data with the upsampling adjoint: cu a multiple of 16 up to
    # cin, even sizes, aligned half-resolution views, a finite slope
    bdu = lib.sur_conv3x3_backward_data_up
    e = vp(0x500000000)
    assert bdu(a, 16, 1, 8, 32, 16, b, 48, 0, c, 48, d, 32, e, 32, 0.1, None) == binding.E_ARG
    assert bdu(a, 16, 1, 8, 32, 16, b, 48, 24, c, 48, d, 24, e, 24, 0.1, None) == binding.E_ARG
    assert bdu(a, 16, 1, 8, 32, 16, b, 48, 64, c, 48, d, 64, e, 64, 0.1, None) == binding.E_ARG
    assert bdu(a, 16, 1, 8, 32, 16, b, 48, 48, c, 48, d, 48, e, 48, 0.1, None) == binding.E_ARG
    assert bdu(a, 16, 1, 8, 32, 16, b, 48, 32, c, 8, d, 32, e, 32, 0.1, None) == binding.E_ARG
    assert bdu(a, 16, 1, 9, 32, 16, b, 48, 32, c, 48, d, 32, e, 32, 0.1, None) == binding.E_ARG
    assert bdu(a, 16, 1, 8, 31, 16, b, 48, 32, c, 48, d, 32, e, 32, 0.1, None) == binding.E_ARG
    assert bdu(a, 16, 1, 8, 32, 16, b, 48, 32, c, 48, None, 32, e, 32, 0.1, None) == binding.E_ARG
    assert bdu(a, 16, 1, 8, 32, 16, b, 48, 32, c, 48, d, 16, e, 32, 0.1, None) == binding.E_ARG
    assert bdu(a, 16, 1, 8, 32, 16, b, 48, 32, c, 48, vp(d.value + 2), 32, e, 32, 0.1,
               None) == binding.E_ARG
    assert bdu(a, 16, 1, 8, 32, 16, b, 48, 32, c, 48, d, 32, vp(e.value + 2), 32, 0.1,
               None) == binding.E_ARG
    assert bdu(a, 16, 1, 8, 32, 16, b, 48, 32, c, 48, d, 32, e, 32, float("inf"),
               None) == binding.E_ARG
    assert bdu(a, 16, 1, 8, 32, 16, vp(b.value + 2), 48, 32, c, 48, d, 32, e, 32, 0.1,
               None) == binding.E_ARG
    # the pooling and upsampling adjoints through an activation need one
    assert lib.sur_pool2_backward_act(a, 16, 1, 8, 8, 16, b, 16, 1, None, 16, 0.1,
                                      None) == binding.E_ARG
    assert lib.sur_pool2_backward_act(a, 16, 1, 8, 8, 16, b, 16, 1, d, 16, float("inf"),
                                      None) == binding.E_ARG
    assert lib.sur_up2_backward_act(a, 16, 1, 4, 4, 16, b, 16, None, 16, 0.1,
                                    None) == binding.E_ARG
    assert lib.sur_up2_backward_act(a, 16, 1, 4, 4, 16, b, 16, d, 8, 0.1, None) == binding.E_ARG
    # weight gradient of an upsampled input: as the forward's checks, plus
    # the workspace; images under 8 x 32 pixels are left to the caller
    wu = lib.sur_conv3x3_backward_weight_up
    ws = lib.sur_conv3x3_backward_weight_workspace(1, 8, 32, 48, 32)
    wsp = vp(0x500000000)
    assert wu(a, 16, 16, d, 32, b, 32, 1, 8, 32, 48, 32, c, None, wsp, ws, None) == binding.E_ARG
    assert wu(a, 32, 32, d, 16, b, 32, 1, 8, 32, 32, 32, c, None, wsp, ws, None) == binding.E_ARG
    assert wu(a, 32, 32, d, 16, b, 32, 1, 9, 32, 48, 32, c, None, wsp, ws, None) == binding.E_ARG
    assert wu(a, 32, 32, d, 16, b, 32, 1, 8, 32, 48, 32, c, None, wsp, ws - 1,
              None) == binding.E_ARG
    ws6 = lib.sur_conv3x3_backward_weight_workspace(1, 6, 32, 48, 32)
    assert wu(a, 32, 32, d, 16, b, 32, 1, 6, 32, 48, 32, c, None, wsp, ws6,
              None) == binding.E_UNSUPPORTED
    ws16 = lib.sur_conv3x3_backward_weight_workspace(1, 8, 16, 48, 32)
    assert wu(a, 32, 32, d, 16, b, 32, 1, 8, 16, 48, 32, c, None, wsp, ws16,
              None) == binding.E_UNSUPPORTED
    # the split sums on another stream need an event; cu goes with xu
    wo = lib.sur_conv3x3_backward_weight_overlap
    st2 = vp(0x700000000)
    assert wo(None, 0, 0, d, 48, b, 32, 1, 8, 32, 48, 32, c, None, wsp, ws, None, st2,
              None) == binding.E_ARG
    assert wo(None, 0, 32, d, 48, b, 32, 1, 8, 32, 48, 32, c, None, wsp, ws, None, None,
              None) == binding.E_ARG
    assert wo(a, 32, 16, d, 32, b, 32, 1, 8, 32, 48, 32, c, None, wsp, ws, None, None,
              None) == binding.E_ARG
    assert wo(a, 32, 32, d, 16, b, 32, 1, 6, 32, 48, 32, c, None, wsp, ws6, None, None,
              None) == binding.E_UNSUPPORTED


def test_fd4_host_checks(lib):
    """The finite-difference reference solver: workspace size and argument
    errors, all decided on the host."""
    st, h = _init(lib, 130, 45, binding.F32)
    assert st == binding.OK
    state = 5 * 130 * 45 * 4
    try:
        assert lib.sslbm_fd4_workspace_bytes(h) == 3 * state
        assert lib.sslbm_fd4_workspace_bytes(None) == 0
        vp = ctypes.c_void_p
        a, w = vp(0x100000000), vp(0x200000000)
        ws = 3 * state
        assert lib.sslbm_fd4_run(None, a, w, ws, 1, None) == binding.E_ARG
        assert lib.sslbm_fd4_run(h, None, w, ws, 1, None) == binding.E_ARG
        assert lib.sslbm_fd4_run(h, a, None, ws, 1, None) == binding.E_ARG
        assert lib.sslbm_fd4_run(h, a, w, ws, -1, None) == binding.E_ARG
        assert lib.sslbm_fd4_run(h, a, w, ws - 1, 1, None) == binding.E_ARG      # short
        assert lib.sslbm_fd4_run(h, a, vp(w.value + 2), ws, 1, None) == binding.E_ARG  # misaligned
        assert lib.sslbm_fd4_run(h, a, vp(a.value + state // 2), ws, 1, None) == binding.E_ALIAS
        assert lib.sslbm_fd4_run(h, vp(w.value + ws - 4), w, ws, 1, None) == binding.E_ALIAS
        # nothing to do for zero steps: no GPU call is made
        assert lib.sslbm_fd4_run(h, a, w, ws, 0, None) == binding.OK
    finally:
        lib.sslbm_destroy(h)


def test_generic_model_host_checks(lib):
    """sslbm_model_create validates the model on the host."""
    from paper_2603_19789_amd.binding import Transition
    D = ctypes.c_double
    d = (D * 3)(0.1, 0.1, 0.0)
    counted = (ctypes.c_int * 3)(1, 1, 0)

    def create(lattice=9, m=3, trans=((0, 1, -1, 0, 0.5),), dd=d, dt=0.01, nx=16):
        arr = (Transition * max(len(trans), 1))(*[Transition(*t) for t in trans])
        h = ctypes.c_void_p()
        st = lib.sslbm_model_create(ctypes.byref(h), nx, 8, binding.F64, binding.PERIODIC,
                                    lattice, m, dd, counted, 1.0, dt, len(trans), arr)
        if h.value:
            lib.sslbm_model_destroy(h)
        return st

    assert create() == binding.OK
    assert create(lattice=5) == binding.OK
    assert create(lattice=7) == binding.E_ARG
    assert create(m=0) == binding.E_ARG
    assert create(m=9) == binding.E_ARG
    assert create(trans=((0, 0, -1, 0, 0.5),)) == binding.E_ARG      # src == dst
    assert create(trans=((3, 1, -1, 0, 0.5),)) == binding.E_ARG      # src out of range
    assert create(trans=((0, 1, 5, 1, 0.5),)) == binding.E_ARG       # catalyst out of range
    assert create(trans=((0, 1, -1, 2, 0.5),)) == binding.E_ARG      # frequency flag
    assert create(trans=((0, 1, -1, 0, -0.5),)) == binding.E_ARG     # negative rate
    assert create(trans=((0, -1, -1, 0, 0.5),)) == binding.OK        # sink
    # stability: D2Q5 allows d_lu <= 1/4, D2Q9 d_lu <= 3/8 (no sources)
    assert create(lattice=5, trans=(), dd=(D * 3)(30.0, 0, 0), dt=0.01) == binding.E_UNSTABLE
    assert create(lattice=9, trans=(), dd=(D * 3)(30.0, 0, 0), dt=0.01) == binding.OK
    assert create(lattice=9, trans=(), dd=(D * 3)(38.0, 0, 0), dt=0.01) == binding.E_UNSTABLE
    assert create(trans=((0, 1, -1, 0, 250.0),)) == binding.E_UNSTABLE  # dt * outflow > 2
    h = ctypes.c_void_p()
    assert lib.sslbm_model_create(None, 8, 8, 0, 0, 5, 1, d, counted, 1.0, 0.01, 0,
                                  None) == binding.E_ARG
    assert lib.sslbm_model_step(None, h, h, None) == binding.E_ARG


def test_generic_model_blocking_host(lib):
    """Steps per pass of sslbm_model_run: 0 (automatic) .. the maximum, set
    and read back on the host."""
    from paper_2603_19789_amd.binding import Transition
    header = (Path(__file__).resolve().parents[1] / "include" / "sslbm.h").read_text()
    assert f"#define SSLBM_MODEL_MAX_BLOCKING {binding.MODEL_MAX_BLOCKING}\n" in header
    d = (ctypes.c_double * 2)(0.1, 0.1)
    counted = (ctypes.c_int * 2)(1, 1)
    tr = (Transition * 1)(Transition(0, 1, -1, 0, 0.5))
    h = ctypes.c_void_p()
    assert lib.sslbm_model_create(ctypes.byref(h), 16, 8, binding.F32, binding.PERIODIC, 5, 2,
                                  d, counted, 1.0, 0.01, 1, tr) == binding.OK
    try:
        k = ctypes.c_int()
        assert lib.sslbm_model_get_blocking(h, ctypes.byref(k)) == binding.OK
        assert 1 <= k.value <= binding.MODEL_MAX_BLOCKING  # automatic choice, resolved
        for want in range(1, binding.MODEL_MAX_BLOCKING + 1):
            assert lib.sslbm_model_set_blocking(h, want) == binding.OK
            assert lib.sslbm_model_get_blocking(h, ctypes.byref(k)) == binding.OK
            assert k.value == want
        assert lib.sslbm_model_set_blocking(h, binding.MODEL_MAX_BLOCKING + 1) == binding.E_ARG
        assert lib.sslbm_model_set_blocking(h, -1) == binding.E_ARG
        assert lib.sslbm_model_get_blocking(h, None) == binding.E_ARG
        assert lib.sslbm_model_set_blocking(None, 1) == binding.E_ARG
    finally:
        lib.sslbm_model_destroy(h)


def test_run_plan_splits_evenly(lib):
    """sslbm_run's passes: the fewest of at most K steps, made even where every
    pass keeps a step, the steps spread evenly (host only)."""
    st, h = _init(lib, 64, 64, binding.F32)
    assert st == binding.OK
    n, hi, lo = ctypes.c_longlong(), ctypes.c_int(), ctypes.c_int()
    try:
        for K in range(1, 7):
            assert lib.sslbm_set_blocking(h, K) == binding.OK
            for nsteps in list(range(0, 130)) + [9999, 10000, 10001]:
                assert lib.sslbm_plan_run(h, nsteps, ctypes.byref(n), ctypes.byref(hi),
                                          ctypes.byref(lo)) == binding.OK
                count, longest, shortest = n.value, hi.value, lo.value
                if nsteps == 0:
                    assert count == 0
                    continue
                fewest = -(-nsteps // K)
                even = fewest + (fewest % 2 == 1 and fewest < nsteps)
                assert count == even, (K, nsteps)
                assert 1 <= shortest <= longest <= K and longest - shortest <= 1
                longer = nsteps - shortest * count
                assert (longer == 0) == (longest == shortest)
                assert 0 <= longer < count or (longer == 0)
        assert lib.sslbm_set_blocking(h, 6) == binding.OK
        lib.sslbm_plan_run(h, 20, ctypes.byref(n), ctypes.byref(hi), ctypes.byref(lo))
        assert (n.value, hi.value, lo.value) == (4, 5, 5)
        assert lib.sslbm_plan_run(h, -1, ctypes.byref(n), None, None) == binding.E_ARG
    finally:
        lib.sslbm_destroy(h)


def test_noalloc_adjoint_step_limit_before_any_device_call(lib):
    """Rows too long for the fixed slot array are refused on the host."""
    h = ctypes.c_void_p()
    params = Params.of(c1_params())
    assert lib.sslbm_init(ctypes.byref(h), 300000, 1, binding.F64, binding.PERIODIC,
                          ctypes.byref(params)) == binding.OK
    try:
        a, b, c, g = (ctypes.c_void_p(v << 28) for v in (1, 2, 3, 4))
        assert lib.sslbm_adjoint_step_noalloc(h, a, b, c, g, None) == binding.E_LIMIT
        assert b"fixed-size" in lib.sslbm_strerror(binding.E_LIMIT)
        assert lib.sslbm_adjoint_step_noalloc(h, a, b, a, g, None) == binding.E_ALIAS
        assert lib.sslbm_adjoint_step_noalloc(None, a, b, c, g, None) == binding.E_ARG
    finally:
        lib.sslbm_destroy(h)


def test_rate_notation_helpers(lib):
    """sslbm_params_from_rates builds the paper's (beta, alpha, gamma, phi)
    from (beta, sigma, gamma, mu) as inputs.from_sigma_mu does, and
    sslbm_rate_gradients is the chain rule of that map: checked against
    central differences of a linear functional of the mapped parameters."""
    from paper_2603_19789_amd import inputs
    dp = ctypes.POINTER(ctypes.c_double)
    d = (ctypes.c_double * 5)(1e-3, 2e-3, 3e-3, 4e-3, 0.0)
    out = binding.Params()
    rates = (0.55, 0.2, 0.1, 0.01)
    assert lib.sslbm_params_from_rates(*rates, d, 1.0, 0.01, ctypes.byref(out)) == binding.OK
    ref = inputs.from_sigma_mu(*rates, (0.0,) * 5)
    assert (out.beta, out.alpha, out.gamma) == (ref.beta, ref.alpha, ref.gamma)
    assert out.phi == pytest.approx(ref.phi, rel=1e-15)
    assert list(out.d) == list(d) and (out.dx, out.dt) == (1.0, 0.01)
    for bad in ((-0.1, 0.2, 0.1, 0.01), (0.5, float("nan"), 0.1, 0.01), (0.5, 0.2, 0.0, 0.0)):
        assert lib.sslbm_params_from_rates(*bad, d, 1.0, 0.01, ctypes.byref(out)) == binding.E_ARG
    assert lib.sslbm_params_from_rates(*rates, None, 1.0, 0.01, ctypes.byref(out)) == binding.E_ARG

    def mapped(b, s, g, m):
        p = binding.Params()
        assert lib.sslbm_params_from_rates(b, s, g, m, d, 1.0, 0.01, ctypes.byref(p)) == 0
        return np.array([p.beta, p.alpha, p.gamma, p.phi])

    rng = np.random.default_rng(4)
    for _ in range(5):
        r = rng.uniform(0.05, 0.6, 4)
        gp = rng.normal(size=4)
        fd = np.empty(4)
        for i in range(4):
            h = 1e-6 * r[i]
            up, dn = r.copy(), r.copy()
            up[i] += h
            dn[i] -= h
            fd[i] = (gp @ mapped(*up) - gp @ mapped(*dn)) / (2 * h)
        gin = (ctypes.c_double * 4)(*gp)
        gout = (ctypes.c_double * 4)()
        assert lib.sslbm_rate_gradients(gin, r[2], r[3], gout) == binding.OK
        assert np.allclose(list(gout), fd, rtol=1e-7, atol=1e-9)
        # in place
        assert lib.sslbm_rate_gradients(gin, r[2], r[3], gin) == binding.OK
        assert list(gin) == list(gout)
    gin = (ctypes.c_double * 4)(1, 2, 3, 4)
    assert lib.sslbm_rate_gradients(gin, -1.0, 0.1, gin) == binding.E_ARG
    assert lib.sslbm_rate_gradients(gin, 0.0, 0.0, gin) == binding.E_ARG
    assert lib.sslbm_rate_gradients(None, 0.1, 0.1, gin) == binding.E_ARG
