"""Host logic of the benchmark script, no GPU: the one-GPU guard and the CPU
oracle leg (one copy, then independent copies at once)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_leg_reports_one_copy_and_all_cores():
    import bench

    out = bench.cpu_leg(2.0, 0.3, 2)
    assert out["kind"] == "oracle" and out["unit"] == "MLUPS" and out["cores"] == 1
    assert out["value"] > 0
    assert out["host"]["nproc"] >= 1 and out["host"]["affinity"] >= 1
    ac = out["all_cores"]
    assert ac["procs"] == 2 and ac["value"] > 0 and ac["unit"] == "MLUPS"


def test_cpu_leg_single_copy_has_no_all_cores_entry():
    import bench

    out = bench.cpu_leg(2.0, 0.2, 1)
    assert "all_cores" not in out
