"""CPU checks of bench.py's contract: one GPU only, and the committed
rocprofv3 traffic summary belongs to the current step-kernel source."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_summary_matches_the_kernel_source():
    sys.path.insert(0, ROOT)
    import bench
    data = json.load(open(os.path.join(ROOT, "profiles", "step_kernel_traffic.json")))
    h = bench.kernel_source_hash()
    for key in ("cavity4096_f32", "cavity4096_f16", "cavity4096_mixed", "batch256_f32",
                "channel2048_f32"):
        assert data[key]["kernel_hash"] == h, key
        t = bench.measured_traffic(key)
        assert t is not None and 1.0 <= t / data[key]["algorithmic_bytes"] < 1.1, key
        assert os.path.exists(os.path.join(ROOT, "profiles", "step_kernel_%s.md" % key))
