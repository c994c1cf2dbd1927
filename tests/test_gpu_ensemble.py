"""Uneven ensembles on the GPU: every instance bit for bit equal to the
single-grid solver, within tolerance of the oracle; HIP graph replays equal
to eager runs; the tuner leaves the state untouched."""
import numpy as np
import pytest

import oracle
from gpu_util import TOL, max_rel_l2, to_gpu, to_np
from paper_2603_19789_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2603_19789_amd import Ensemble, Solver  # noqa: E402

SIZES = [(64, 64), (3, 5), (130, 71), (17, 9), (128, 128), (256, 64), (1, 1), (96, 40)]


def _params(i):
    base = inputs.c1_params()
    dl = (0.03, 0.015, 0.005, 0.02, 0.0) if i % 2 else (0.01, 0.02, 0.001, 0.004, 0.0)
    return base.with_(beta=0.3 + 0.1 * i, d=inputs.lattice_to_physical(dl, base.dx, base.dt))


def _same(ens, a, b) -> bool:
    """Bitwise equality of every instance (the gaps between instance blocks
    hold no data and are not compared)."""
    return all(torch.equal(x, y) for x, y in zip(ens.views(a), ens.views(b)))


def _load(ens, states, dtype):
    flat = ens.empty()
    flat.zero_()
    for v, s in zip(ens.views(flat), states):
        v.copy_(to_gpu(s, dtype))
    return flat


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("bc", ["periodic", "noflux"])
def test_instances_match_single_grid_and_oracle(dtype, bc):
    orc = oracle.load()
    params = [_params(i) for i in range(len(SIZES))]
    states = [inputs.random_state(nx, ny, seed=40 + i) for i, (nx, ny) in enumerate(SIZES)]
    ens = Ensemble(SIZES, params, dtype=dtype, bc=bc)
    flat = _load(ens, states, dtype)
    ens.run(flat, 13)
    for i, (v, s, p) in enumerate(zip(ens.views(flat), states, params)):
        nx, ny = SIZES[i]
        single = Solver(nx, ny, p, dtype=dtype, bc=bc)
        ref = to_gpu(s, dtype)
        single.run(ref, 13)
        assert torch.equal(v, ref), f"instance {i} ({nx}x{ny}) differs from the single grid"
        assert max_rel_l2(to_np(v), orc.sslbm_run(s, p, 13, bc=bc)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_every_shape_gives_the_same_bits(dtype):
    params = [_params(i) for i in range(len(SIZES))]
    sizes = [(nx + nx % 2, ny) for nx, ny in SIZES]  # even rows allow two columns per lane
    states = [inputs.random_state(nx, ny, seed=60 + i) for i, (nx, ny) in enumerate(sizes)]
    ens = Ensemble(sizes, params, dtype=dtype)
    start = _load(ens, states, dtype)
    ref = start.clone()
    ens.set_launch(1, 0, 1)
    ens.run(ref, 11)
    from paper_2603_19789_amd.binding import SSLBMError
    tried = 0
    for K in (2, 3, 5, 6):
        for V in (1, 2):
            for H in (0, 7, 64):
                try:
                    ens.set_launch(K, H, V)
                except SSLBMError:
                    continue
                got = start.clone()
                ens.run(got, 11)
                assert _same(ens, got, ref), f"K={K} V={V} H={H}"
                tried += 1
    assert tried >= 8


def test_graph_replays_match_eager_runs():
    """Replay the captured run several times with eager work in between; every
    replay must equal the eager result of the same number of steps."""
    params = [_params(i) for i in range(len(SIZES))]
    states = [inputs.random_state(nx, ny, seed=80 + i) for i, (nx, ny) in enumerate(SIZES)]
    ens = Ensemble(SIZES, params, dtype="f32")
    start = _load(ens, states, "f32")
    eager = start.clone()
    scratch = ens.empty()
    ens.run(eager, 9, scratch)
    for rep in range(4):
        got = start.clone()
        ens.run(got, 9, scratch, graph=True)
        torch.cuda.synchronize()
        assert _same(ens, got, eager), f"replay {rep}"
        # eager work between replays, on the same buffers
        tmp = start.clone()
        ens.run(tmp, 3, scratch)
        torch.cuda.synchronize()
    # a graph on other buffers is a different graph
    other = start.clone()
    ens.run(other, 9, graph=True)
    assert _same(ens, other, eager)


def test_tuner_keeps_state_and_results():
    params = [_params(i) for i in range(len(SIZES))]
    sizes = [(nx + nx % 2, ny) for nx, ny in SIZES]
    states = [inputs.random_state(nx, ny, seed=90 + i) for i, (nx, ny) in enumerate(sizes)]
    ens = Ensemble(sizes, params, dtype="f32")
    start = _load(ens, states, "f32")
    ref = start.clone()
    ens.run(ref, 10)
    state = start.clone()
    best = ens.tune(state)
    assert torch.equal(state, start)  # the tuner writes nothing, gaps included
    assert best == ens.launch()
    assert best["steps_per_pass"] >= 2
    ens.run(state, 10)
    assert _same(ens, state, ref)


def test_uneven_512_ensemble_sampled():
    """The 512-instance uneven workload, launched as the benchmark launches it
    (tuned shape, one graph): sampled instances bit for bit equal to the
    single-grid solver."""
    w = inputs.ensemble_workload(nsteps=12)
    ens = Ensemble(w.sizes, w.params, dtype="f32")
    flat = ens.empty()
    states = []
    for i, (v, s) in enumerate(zip(ens.views(flat), w.states())):
        v.copy_(to_gpu(s, "f32"))
        if i % 37 == 0:
            states.append((i, s))
    start = flat.clone()
    ens.tune(flat)
    ens.run(flat, w.nsteps, graph=True)
    views = ens.views(flat)
    for i, s in states:
        nx, ny = w.sizes[i]
        single = Solver(nx, ny, w.params[i], dtype="f32")
        ref = to_gpu(s, "f32")
        single.run(ref, w.nsteps)
        assert torch.equal(views[i], ref), f"instance {i}"
    assert not torch.equal(flat, start)
