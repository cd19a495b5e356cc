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
    for key in ("cavity4096_f32", "cavity4096_f32_single", "cavity4096_f32c",
                "cavity4096_f32c_single", "cavity4096_f16", "cavity4096_f16_single",
                "cavity4096_mixed",
                "cavity4096_mixed_single", "batch256_f32", "batch256_f32c",
                "channel2048_f32", "channel2048_f32c"):
        assert data[key]["kernel_hash"] == h, key
        t = bench.measured_traffic(key)
        # one step per launch: close to the populations read and written once;
        # two: the ring of every tile is read again (mostly from L2)
        hi = 1.1 if data[key]["steps_per_launch"] == 1 else 1.5
        assert t is not None and 1.0 <= t / data[key]["algorithmic_bytes"] < hi, key
        assert os.path.exists(os.path.join(ROOT, "profiles", "step_kernel_%s.md" % key))
    # the FP32 records of the default launch mode come from the two-step
    # kernel, the "single" one from the one-step kernel
    for key in ("cavity4096_f32", "cavity4096_f32c", "cavity4096_f16", "cavity4096_mixed",
                "batch256_f32", "batch256_f32c", "channel2048_f32", "channel2048_f32c"):
        assert data[key]["steps_per_launch"] == 2 and "step2_kernel" in data[key]["kernel"], key
    one, two = data["cavity4096_f32_single"], data["cavity4096_f32"]
    assert one["steps_per_launch"] == 1 and "step2_kernel" not in one["kernel"]
    # the work of one node update, counted on the one-step kernel; the two-step
    # kernel issues more per update (it also updates each tile's ring)
    assert one["fp64_flops_per_launch"] > 0 and one["valu_instr_per_launch"] > 0
    per_lu_one = one["valu_instr_per_launch"] / one["nodes"]
    per_lu_two = two["valu_instr_per_launch"] / (2 * two["nodes"])
    assert 1.0 < per_lu_two / per_lu_one < 660 / 512 + 0.05
    # the roofline of the measured launch time: algorithmic bytes of two node
    # updates per node per launch against 8 TB/s; issue and FP64 beside it
    r = bench.two_step_roofline("cavity4096_f32", "f32", two["nodes"], two["avg_launch_us"] / 2e3,
                                112)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    launch_s = two["avg_launch_us"] * 1e-6
    assert abs(r["achieved"] - 112 * 2 * two["nodes"] / launch_s / 1e9) < 0.1
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-4 and 0 < r["frac"] < 1.2
    assert r["traffic"] == two["bytes_per_launch"]
    assert abs(r["traffic_frac"] - two["bytes_per_launch"] / launch_s / 8e12) < 1e-4
    assert 0 < r["valu"]["frac"] <= r["valu"]["issued_frac"] < 1 and 0 < r["fp64"]["frac"] < 1
    # FP32 arithmetic: no FP64 work, fewer instructions per node update
    c1 = data["cavity4096_f32c_single"]
    assert c1["fp64_flops_per_launch"] == 0
    assert c1["valu_instr_per_launch"] < one["valu_instr_per_launch"]


def test_kernel_hash_ignores_comments_and_layout():
    sys.path.insert(0, ROOT)
    import bench
    a = "int f(int x) {\n  return x + 1;  // one more\n}\n/* note */"
    b = "int f(int x) { return x + 1; }"
    assert bench.code_only(a) == bench.code_only(b)
    assert bench.code_only(b) != bench.code_only(b.replace("1", "2"))


def test_main_prints_its_json_line():
    # The default line is printed at the end of main (a refactor once lost
    # the print and the bench exited 0 with no output).
    import ast
    src = open(os.path.join(ROOT, "bench.py")).read()
    main = next(n for n in ast.parse(src).body if isinstance(n, ast.FunctionDef) and n.name == "main")
    last = main.body[-1]
    assert isinstance(last, ast.Expr) and isinstance(last.value, ast.Call)
    assert ast.unparse(last.value).startswith("print(json.dumps(out)")
