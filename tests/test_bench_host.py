"""Host-side checks of the benchmark script (no GPU): it refuses more than one
GPU, and it reads a committed HBM-traffic line only when the line was taken on
the current source of the step kernels."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_lines_are_keyed_to_the_kernel_source(tmp_path, monkeypatch):
    src = tmp_path / "step_kernels.hip"
    src.write_bytes(b"// kernels\n")
    h = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    traffic = tmp_path / "traffic.txt"
    traffic.write_text(
        "# comment line traffic workload=pool-wave storage=f32 bytes_per_launch=1 kernel_src=x\n"
        f"traffic workload=pool-wave storage=f32 bytes_per_launch=3271391597 fetch=1 write=2 kernel_src={h}\n"
        "traffic workload=pool-wave storage=f16 bytes_per_launch=99 fetch=1 write=2 kernel_src=0000000000000000\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(src))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(traffic))
    assert bench.measured_traffic("pool-wave", "f32") == 3271391597.0
    # taken on another source: not used
    assert bench.measured_traffic("pool-wave", "f16") is None
    # no line for this workload or storage
    assert bench.measured_traffic("cyl-dam-break", "f32") is None
    assert bench.measured_traffic("pool-wave", "bf16") is None
    # the source changes: the line no longer applies
    src.write_bytes(b"// kernels, edited\n")
    assert bench.measured_traffic("pool-wave", "f32") is None
    # no traffic file at all
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "absent.txt"))
    assert bench.measured_traffic("pool-wave", "f32") is None
