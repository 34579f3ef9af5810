"""Host-side pieces of bench.py that need no GPU: the one-GPU guard, the lookup
of measured HBM traffic (valid only for the kernel sources it was taken on), and
the CPU-baseline leg (the FP64 oracle on a bounded sample)."""
import os
import subprocess
import sys

import bench
from paper_2009_04604_amd.profiling import kernel_source_sha

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _summary(root, sha, fetch=908e6, write=812e6):
    os.makedirs(os.path.join(root, "profiles"), exist_ok=True)
    with open(os.path.join(root, "profiles", "step_kernel_packing256_f32_counters.txt"), "w") as f:
        f.write("# counters\n")
        f.write(f"kernel_source_sha256: {sha}\n")
        f.write(f"kernel_bytes_per_launch.FETCH_SIZE: {fetch}\n")
        f.write(f"kernel_bytes_per_launch.WRITE_SIZE: {write}\n")


def test_traffic_only_for_the_current_kernel_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_from_profile("packing256", "f32") is None          # no summary
    _summary(str(tmp_path), kernel_source_sha())
    assert bench.traffic_from_profile("packing256", "f32") == 908e6 + 812e6
    _summary(str(tmp_path), "0123456789abcdef")                              # taken on other sources
    assert bench.traffic_from_profile("packing256", "f32") is None
    assert bench.traffic_from_profile("packing256", "bf16s") is None         # other storage: no summary


def test_cpu_baseline_is_the_oracle_on_one_core():
    r = bench.cpu_baseline("packing256", 0.5)
    assert r["kind"] == "oracle"
    assert r["cores"] == 1
    assert r["unit"] == "MLUPS"
    assert r["value"] > 0
    assert "64^3" in r["sample"]
