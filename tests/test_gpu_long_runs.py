"""Long runs on the GPU: FP32 over 1000 BGK steps and 200 SSLBM steps of the
4096 x 4096 workload against the FP64 oracle, and the drift of FP32 from
FP64 over the 10 000 steps of that workload.

FP32 arithmetic rounds every stored value and every operation to 2^-24
relative; over a run the roundings of the linear (diffusion) part random-walk
while the epidemic's growth rate (the first eigenvalue of Eq. (eigenvalues),
0.2 to 0.5 per unit time here) amplifies those of the infection terms. The
SSLBM parity tests hold FP32 to 1e-5 per compartment up to 1000 steps, as
for shorter runs (BGK: see its test); over 10 000 steps the FP32-versus-FP64 difference is reported
and only held to a loose 1e-4 (an order of magnitude above the value a plain
FP32 model of the step gave before the kernels were written, 1.4e-5)."""
import numpy as np
import pytest

import oracle
from gpu_util import TOL, max_rel_l2, sample_nodes, to_gpu, to_np, windowed_oracle
from paper_2603_19789_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2603_19789_amd import BGK, Solver  # noqa: E402


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


def test_bgk_c1_fp32_1000_steps(orc):
    """The parity configuration (128 x 128, one focus, 1000 steps) with BGK in
    FP32 against the FP64 oracle's BGK. With d_lu = 1e-3, tau = 0.503 and the
    collision factor 1 - 1/tau = -0.988: the non-equilibrium parts of the 20
    populations are barely damped and flip sign every step, so FP32 roundings
    of the populations pile up there. A plain float32 NumPy model of the
    scheme (references.bgk_fp32_model) shows that floor, 5.7e-5 from FP64
    after 1000 steps, which no FP32 BGK can beat; the kernel is held to twice
    that model's error, computed here, and to 1e-4."""
    import references as ref
    w = inputs.c1_workload()
    b = BGK(w.nx, w.ny, w.params, dtype="f32")
    f, rd = b.init(to_gpu(w.rho0, "f32"))
    b.run(f, rd, w.nsteps)
    want = orc.bgk_run_density(w.rho0, w.params, w.nsteps, threads=oracle.host_threads())
    err = max_rel_l2(to_np(b.density(f, rd)), want)
    floor = max_rel_l2(ref.bgk_fp32_model(w.rho0, w.params, w.nsteps), want)
    print(f"BGK C1 FP32 1000 steps: {err:.3e} (plain float32 model {floor:.3e})")
    assert err <= min(2.0 * floor, 1e-4)


@pytest.mark.parametrize("bc", ["periodic", "noflux"])
def test_full_size_fp32_sampled_200_steps(orc, bc):
    """4096 x 4096, 64 foci, R0 = 5, 200 steps as the benchmark runs them
    (automatic pass shape): sampled nodes against the oracle on each node's
    dependence cone (a window of 2 x 200 + 3 cells)."""
    nsteps = 200
    w = inputs.c2_workload(r0=5.0, nsteps=nsteps)
    rho0 = w.rho0.copy()
    rng = np.random.default_rng(14)
    rho0[1] = rng.uniform(0, 0.02, size=rho0[1].shape)
    rho0[0] = 1.0 - rho0[1] - rho0[2]
    s = Solver(w.nx, w.ny, w.params, dtype="f32", bc=bc)
    rho = to_gpu(rho0, "f32")
    s.run(rho, nsteps)
    torch.cuda.synchronize()
    nodes = sample_nodes(w.nx, w.ny, 16, seed=5)
    want = windowed_oracle(orc, rho0, w.params, nsteps, bc, nodes, threads=oracle.host_threads())
    xs = torch.tensor([x for x, _ in nodes], device="cuda")
    ys = torch.tensor([y for _, y in nodes], device="cuda")
    got = rho[:, ys, xs].T.cpu().double().numpy()
    err = np.linalg.norm(got - want, axis=0) / np.linalg.norm(want, axis=0)
    print(f"4096^2 FP32 200 steps, sampled: {err}")
    assert np.all(err <= TOL["f32"]), err


def test_fp32_drift_over_10000_steps():
    """The 4096 x 4096 workload at R0 = 5 over 10 000 steps in FP32 and FP64
    on the GPU: the per-compartment relative L2 difference (reported)."""
    w = inputs.c2_workload(r0=5.0)
    assert w.nsteps == 10000
    out = {}
    for d in ("f32", "f64"):
        s = Solver(w.nx, w.ny, w.params, dtype=d)
        rho = to_gpu(w.rho0, d)
        s.run(rho, w.nsteps)
        out[d] = to_np(rho)
        del s, rho
    drift = [float(np.linalg.norm(out["f32"][c] - out["f64"][c]) / np.linalg.norm(out["f64"][c]))
             for c in range(5)]
    print("FP32 vs FP64 after 10000 steps (S, E, I, R, D): "
          + ", ".join(f"{v:.2e}" for v in drift))
    assert max(drift) <= 1e-4
