"""Helpers for the GPU tests: tensors, tolerances, and the oracle evaluated on
windows of a large grid (only the dependence cone of the sampled nodes)."""
from __future__ import annotations

import numpy as np

import references as ref

TOL = {"f64": 1e-12, "f32": 1e-5}


def torch_dtype(dtype):
    import torch
    return torch.float64 if dtype == "f64" else torch.float32


def to_gpu(a, dtype):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch_dtype(dtype), device="cuda")


def to_np(t) -> np.ndarray:
    return t.detach().cpu().double().numpy()


def max_rel_l2(got, want) -> float:
    """Largest per-compartment relative L2 error (absolute where the oracle is 0)."""
    return max(ref.rel_l2(got[c], want[c]) for c in range(got.shape[0]))


def _map(i, n, bc):
    if bc == "periodic":
        return np.mod(i, n)
    m = np.mod(i, 2 * n)
    return np.where(m < n, m, 2 * n - 1 - m)


def windowed_oracle(orc, rho0, params, nsteps, bc, samples, threads=1):
    """Oracle values after nsteps at the sampled (x, y) nodes. Each node depends
    only on nodes within nsteps cells, so the oracle runs on a periodic window
    of side 2 nsteps + 3 around it; no-flux walls are the mirror-image
    extension of the field (pinned in the oracle tests)."""
    _, ny, nx = rho0.shape
    half = nsteps + 1
    offs = np.arange(-half, half + 1)
    out = np.empty((len(samples), 5))
    for s, (x, y) in enumerate(samples):
        ys = _map(y + offs, ny, bc)
        xs = _map(x + offs, nx, bc)
        win = rho0[:, ys][:, :, xs]
        res = orc.sslbm_run(win, params, nsteps, bc="periodic", threads=threads)
        out[s] = res[:, half, half]
    return out


def sample_nodes(nx, ny, count, seed):
    rng = np.random.default_rng(seed)
    fixed = [(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1), (nx // 2, 0), (0, ny // 2),
             (nx - 1, ny // 2), (nx // 2, ny - 1)]
    rand = list(zip(rng.integers(0, nx, count).tolist(), rng.integers(0, ny, count).tolist()))
    return fixed + rand
