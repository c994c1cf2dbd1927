"""Build libsslbm.so in-tree with hipcc for gfx950.

Usage: python -m paper_2603_19789_amd.build   (or call ``build()``)
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
INCLUDE = ROOT / "include"
LIBRARY = PKG / "libsslbm.so"
ARCH = "gfx950"

SOURCES = ["sslbm_api.cpp", "ensemble_api.cpp", "adjoint_api.cpp", "surrogate_api.cpp",
           "model_api.cpp", "sslbm_kernels.hip", "ensemble_kernels.hip", "adjoint_kernels.hip",
           "surrogate_kernels.hip", "model_kernels.hip", "bgk_kernels.hip",
           "reduce_kernels.hip", "fd4_kernels.hip"]

# Sources compiled more than once, one object per set of definitions: the
# generic-model kernels per arithmetic type and lattice (four objects that
# compile in parallel instead of one long serial unit).
INSTANCES = [
    ("model_kernels_inst.hip", f"model_kernels_{t}_d2q{q}",
     [f"-DMODEL_FP64={int(t == 'f64')}", f"-DMODEL_Q={q}"])
    for t in ("f32", "f64") for q in (5, 9)
]

# -ffp-contract=off: only the fma() calls written in the kernels fuse, so every
# launch shape and blocking depth rounds identically.
# -packed-fp32-ops off: no packed FP32 instructions are generated.
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# Per-source additions. The MFMA kernels keep their accumulators in ordinary
# VGPRs: with the accumulation registers, this compiler copied the running
# sums of the two-deep convolution pipeline back and forth every step.
EXTRA_FLAGS = {
    "surrogate_kernels.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"],
}


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return str(Path(rocm) / "bin" / "hipcc")


def _run(cmd):
    """Run a compiler command; drop the host pass's notice that it does not
    know the device-only packed-fp32 feature, show everything else."""
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "'-packed-fp32-ops' is not a recognized feature"
    for line in (res.stdout + res.stderr).splitlines():
        if noise not in line:
            print(line, file=sys.stderr)
    if res.returncode != 0:
        raise subprocess.CalledProcessError(res.returncode, cmd)


def build(verbose: bool = False) -> Path:
    """Compile every source and link the shared library (always rebuilds)."""
    objdir = PKG / "_build"
    objdir.mkdir(exist_ok=True)
    cmds, objs = [], []
    units = [(name, Path(name).stem, []) for name in SOURCES] + INSTANCES
    for name, stem, defines in units:
        src = CSRC / name
        obj = objdir / (stem + ".o")
        cmds.append([hipcc(), *FLAGS, *EXTRA_FLAGS.get(name, []), *defines, "-x", "hip",
                     f"-I{INCLUDE}", f"-I{CSRC}", "-c", str(src),
                     "-o", str(obj)])
        objs.append(str(obj))
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as pool:
        list(pool.map(_run, cmds))
    tmp = LIBRARY.with_suffix(".so.tmp")
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    _run(cmd)
    os.replace(tmp, LIBRARY)
    return LIBRARY


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIBRARY)
