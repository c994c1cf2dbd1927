"""The benchmark's contract on the host (no GPU): it refuses more than one
GPU with a message, and the HBM traffic it reports for the headline kernel
comes from a counter summary taken on the current kernel source."""
import subprocess
import sys
from pathlib import Path

ROOT = Path(__file__).resolve().parents[1]


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU" in (res.stdout + res.stderr)


def test_recorded_traffic_matches_the_kernel_source():
    sys.path.insert(0, str(ROOT))
    import bench
    for kernel in ("sslbm_march_kernel<float, 5, false, 2>",
                   "sslbm_march_kernel<float, 6, false, 2>"):
        traffic = bench.recorded_traffic(kernel)
        assert traffic is not None, f"no counter summary of {kernel} on the current source"
        # a pass moves its algorithmic bytes plus a few per cent of halo
        algorithmic = 40 * 4096 * 4096
        assert algorithmic <= traffic < 1.2 * algorithmic
        assert 0.0 < bench.recorded_valu_issue(kernel) < 1.0
