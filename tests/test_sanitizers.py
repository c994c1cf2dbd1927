"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

* The oracle (oracle.c) built with gcc's sanitizers runs the fast pins; a
  copy with a planted out-of-bounds read must be stopped by ASan, which shows
  the instrumentation is live.
* The library's host side (the argument checks, layouts, plans and tables of
  the *_api.cpp files) built with the sanitizers on the host pass only, linked
  with the kernel objects of the normal build, runs the CPU tests of the C ABI.
Python itself is not instrumented, so each run is a child process with the
sanitizer runtime preloaded; leak detection is off (the interpreter keeps
memory until exit)."""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

import pytest

import oracle

ROOT = Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2603_19789_amd" / "csrc"
OBJ = ROOT / "paper_2603_19789_amd" / "_build"
API = ["sslbm_api", "ensemble_api", "adjoint_api", "surrogate_api", "model_api"]
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0",
           "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _gcc_runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = out.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _child(code, preload, *args, timeout=300):
    env = dict(os.environ, **SAN_ENV, LD_PRELOAD=preload)
    return subprocess.run([sys.executable, "-c", code, *args], capture_output=True, text=True,
                          env=env, timeout=timeout, cwd=ROOT)


ORACLE_PINS = """
import sys
sys.path[:0] = ["{root}", "{root}/tests"]
import oracle, pins
o = oracle.Oracle(sys.argv[1])
for check in pins.FAST_SSLBM_CHECKS + pins.FAST_BGK_CHECKS:
    check(o)
print("pins ok")
"""


def test_oracle_under_sanitizers(tmp_path):
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    flags = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
             "-g", "-O1"]
    source = oracle.SOURCE.read_text()
    good = tmp_path / "oracle_san.c"
    good.write_text(source)
    lib = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", *flags, "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-o", str(lib), str(good), "-lm"], check=True)
    code = ORACLE_PINS.format(root=ROOT)
    res = _child(code, f"{asan}:{ubsan}", str(lib))
    assert res.returncode == 0 and "pins ok" in res.stdout, res.stderr[-2000:]
    # a planted read past the end of a field must be caught
    site = "            return field[(size_t)yc * nx + xc];\n        }\n    }\n    return field[(size_t)y * nx + x];"
    assert source.count(site) == 1
    bad = tmp_path / "oracle_oob.c"
    bad.write_text(source.replace(site, site[:-len("x];")] + "x + (size_t)nx * ny];"))
    badlib = tmp_path / "liboracle_oob.so"
    subprocess.run(["gcc", *flags, "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-o", str(badlib), str(bad), "-lm"], check=True)
    res = _child(code, f"{asan}:{ubsan}", str(badlib))
    assert res.returncode != 0 and "AddressSanitizer" in res.stderr, res.stderr[-2000:]


HOST_TESTS = """
import sys
from pathlib import Path
sys.path.insert(0, "{root}")
from paper_2603_19789_amd import binding
binding.LIBRARY = Path(sys.argv[1])
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", "{root}/tests/test_abi_host.py",
                      "{root}/tests/test_ensemble_host.py"]))
"""


def test_library_host_side_under_sanitizers(tmp_path):
    from paper_2603_19789_amd import build as hip_build
    # the device-code objects of the normal build: one per kernel source,
    # plus one per instantiation of a source compiled more than once
    kernels = [OBJ / f"{Path(n).stem}.o" for n in hip_build.SOURCES if n.endswith(".hip")]
    kernels += [OBJ / f"{stem}.o" for _, stem, _ in hip_build.INSTANCES]
    if not all(k.exists() for k in kernels):
        pytest.skip("kernel objects of the normal build are missing (run the build first)")
    runtimes = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not runtimes:
        pytest.skip("clang ASan runtime not installed")
    hipcc = str(Path(os.environ.get("ROCM_PATH", "/opt/rocm")) / "bin" / "hipcc")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]

    def compile_one(name):
        obj = tmp_path / f"{name}.o"
        subprocess.run([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                        "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
                        "-packed-fp32-ops", *san, "-x", "hip", f"-I{ROOT / 'include'}",
                        f"-I{CSRC}", "-c", str(CSRC / f"{name}.cpp"), "-o", str(obj)],
                       check=True, capture_output=True)
        return str(obj)

    with ThreadPoolExecutor(len(API)) as pool:
        objs = list(pool.map(compile_one, API))
    lib = tmp_path / "libsslbm_san.so"
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", str(lib), *objs,
                    *[str(k) for k in kernels]], check=True, capture_output=True)
    res = _child(HOST_TESTS.format(root=ROOT), runtimes[0], str(lib))
    assert res.returncode == 0, (res.stdout[-2000:], res.stderr[-2000:])
    assert "passed" in res.stdout
