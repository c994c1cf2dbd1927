"""Ensemble entry points on the CPU: validation and the state layout."""
import ctypes

import pytest

from paper_2603_19789_amd import binding
from paper_2603_19789_amd.binding import Launch, Params
from paper_2603_19789_amd.inputs import c1_params, ensemble_workload


@pytest.fixture(scope="module")
def lib():
    return binding.library()


def _create(lib, sizes, params, dtype=binding.F32, bc=binding.PERIODIC):
    n = len(sizes)
    nx = (ctypes.c_int * n)(*[s[0] for s in sizes])
    ny = (ctypes.c_int * n)(*[s[1] for s in sizes])
    ps = (Params * n)(*[Params.of(p) for p in params])
    bad = ctypes.c_int(-7)
    h = ctypes.c_void_p()
    st = lib.sslbm_ensemble_create(ctypes.byref(h), n, nx, ny, dtype, bc, ps, ctypes.byref(bad))
    return st, h, bad.value


def test_layout_is_packed_and_aligned(lib):
    sizes = [(64, 64), (3, 5), (130, 71), (1, 1)]
    st, h, bad = _create(lib, sizes, [c1_params()] * 4)
    assert st == binding.OK and bad == -1
    offs = [lib.sslbm_ensemble_offset(h, i) for i in range(4)]
    total = lib.sslbm_ensemble_elements(h)
    assert offs[0] == 0
    for i, (nx, ny) in enumerate(sizes):
        assert offs[i] % 4 == 0
        end = offs[i] + 5 * nx * ny
        nxt = offs[i + 1] if i + 1 < 4 else total
        assert end <= nxt < end + 4
    assert lib.sslbm_ensemble_offset(h, 4) == -1
    assert lib.sslbm_ensemble_offset(h, -1) == -1
    lib.sslbm_ensemble_destroy(h)


def test_rejects_bad_instances(lib):
    good = c1_params()
    st, h, bad = _create(lib, [(8, 8), (0, 8)], [good, good])
    assert st == binding.E_ARG and bad == 1 and not h.value
    st, h, bad = _create(lib, [(8, 8), (8, 8), (8, 8)],
                         [good, good, good.with_(d=(100.0,) * 5)])
    assert st == binding.E_UNSTABLE and bad == 2
    st, h, bad = _create(lib, [(8, 8)], [good.with_(beta=-1.0)])
    assert st == binding.E_ARG and bad == 0
    st, h, bad = _create(lib, [(8, 8)], [good], dtype=5)
    assert st == binding.E_ARG
    h = ctypes.c_void_p()
    assert lib.sslbm_ensemble_create(ctypes.byref(h), 0, None, None, 0, 0, None, None) == binding.E_ARG


def test_launch_shape_and_run_arguments(lib):
    st, h, _ = _create(lib, [(64, 64), (128, 128)], [c1_params()] * 2)
    L = Launch
    assert lib.sslbm_ensemble_set_launch(h, ctypes.byref(L(9, 0, 0))) == binding.E_ARG
    assert lib.sslbm_ensemble_set_launch(h, ctypes.byref(L(7, 0, 2))) == binding.E_UNSUPPORTED
    assert lib.sslbm_ensemble_set_launch(h, ctypes.byref(L(4, 32, 2))) == binding.OK
    got = L()
    assert lib.sslbm_ensemble_get_launch(h, ctypes.byref(got)) == binding.OK
    assert got.as_dict() == L(4, 32, 2).as_dict()
    a, b = ctypes.c_void_p(0x100000), ctypes.c_void_p(0x100010)
    assert lib.sslbm_ensemble_run(h, a, b, 3, 0, None) == binding.E_ALIAS
    assert lib.sslbm_ensemble_run(h, a, None, 3, 0, None) == binding.E_ARG
    assert lib.sslbm_ensemble_run(h, a, ctypes.c_void_p(0x9000000), -1, 0, None) == binding.E_ARG
    assert lib.sslbm_ensemble_run(h, a, ctypes.c_void_p(0x9000000), 2, 4, None) == binding.E_ARG
    assert lib.sslbm_ensemble_run(h, a, ctypes.c_void_p(0x9000000), 0, 0, None) == binding.OK
    lib.sslbm_ensemble_destroy(h)


def test_odd_rows_use_one_column_per_lane(lib):
    st, h, _ = _create(lib, [(200, 64), (201, 64)], [c1_params()] * 2)
    got = Launch()
    assert lib.sslbm_ensemble_get_launch(h, ctypes.byref(got)) == binding.OK
    assert got.cols_per_lane == 1
    lib.sslbm_ensemble_destroy(h)


def test_uneven_workload_recipe():
    w = ensemble_workload(count=64, seed=3)
    assert len(w.sizes) == 64 and all(s in ((64, 64), (128, 128), (256, 256), (512, 512))
                                      for s in w.sizes)
    for p in w.params:
        assert 1.5 <= p.beta / p.gamma <= 5.0
    e = binding.Ensemble(w.sizes, w.params)
    assert e.elements >= sum(5 * nx * ny for nx, ny in w.sizes)


def test_size_classes():
    """Instances of at most 80 KiB go on chip; the others are grouped by the
    power-of-two bucket of their longest side, each with a shape of its own."""
    sizes = [(64, 64), (3, 5), (130, 71), (128, 128), (256, 64), (65, 64), (512, 512), (1, 1)]
    e = binding.Ensemble(sizes, [c1_params()] * len(sizes), dtype="f32")
    cls = e.classes()
    on_chip = [c for c in cls if c["on_chip"]]
    assert len(on_chip) == 1 and on_chip[0]["instances"] == 3
    assert on_chip[0]["cells"] == 64 * 64 + 15 + 1 and on_chip[0]["launch"]["steps_per_pass"] == 0
    # (65, 64) and (128, 128) share the bucket up to 128; (130, 71) and (256, 64) up to 256
    march = {c["max_side"]: c for c in cls if not c["on_chip"]}
    assert sorted(march) == [128, 256, 512]
    assert march[128]["instances"] == 2 and march[256]["instances"] == 2
    for i, (nx, ny) in enumerate(sizes):
        c = cls[e.instance_class(i)]
        assert c["on_chip"] == (5 * nx * ny * 4 <= 81920)
    for c in march.values():
        assert c["launch"]["steps_per_pass"] == 6 and c["launch"]["rows_per_wave"] >= 12
    # a shape for one class leaves the others automatic
    k512 = next(i for i, c in enumerate(cls) if c["max_side"] == 512 and not c["on_chip"])
    e.set_class_launch(k512, 3, 40, 1)
    after = e.classes()
    assert after[k512]["launch"] == {"steps_per_pass": 3, "rows_per_wave": 40, "cols_per_lane": 1}
    assert e.launch() == after[k512]["launch"]  # the class with the most cells
    k_chip = next(i for i, c in enumerate(cls) if c["on_chip"])
    with pytest.raises(binding.SSLBMError):
        e.set_class_launch(k_chip, 3, 0, 1)
    with pytest.raises(binding.SSLBMError):
        e.set_class_launch(len(cls), 3, 0, 1)
    # FP64: 64 x 64 is 160 KiB, too large for the on-chip class
    e64 = binding.Ensemble([(64, 64), (40, 40)], [c1_params()] * 2, dtype="f64")
    c64 = e64.classes()
    assert [c["on_chip"] for c in c64] == [False, True]
