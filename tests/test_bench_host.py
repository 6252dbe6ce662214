"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic
bytes per sweep launch, and the rule that measured traffic is reported only
for the kernel source it was measured on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2305_19400_amd import inputs as I  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_exits_with_a_message(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_sweep_bytes_of_the_2d_workload():
    # 128 x 128 cells x 400 directions x 55 band entries: I^k and I^n read and
    # I^{k+1} written per update (8 B each in FP64, 4 B in FP32), plus the
    # per-(band, cell) equilibrium read and energy partial write (8 B each)
    inst = I.config_c2()
    n_dof = 128 * 128 * 400 * 55
    assert inst.n_dof == n_dof
    assert bench.sweep_bytes(inst, 8) == n_dof * 24 + 55 * 128 * 128 * 16
    assert bench.sweep_bytes(inst, 4) == n_dof * 12 + 55 * 128 * 128 * 16


def test_traffic_only_for_the_measured_source(tmp_path):
    src = tmp_path / "kernels.hip"
    src.write_text("// a kernel\n__global__ void k() {}  // empty\n")
    counters = tmp_path / "counters.json"
    counters.write_text(json.dumps({"kernel_code_sha256": bench.kernel_code_hash(str(src)),
                                    "traffic_bytes_per_launch": 1.25e9}))
    assert bench.measured_traffic(str(src), str(counters)) == 1.25e9
    # comments and blank lines do not count ...
    src.write_text("/* a kernel,\n   empty */\n\n__global__ void k() {}\n")
    assert bench.measured_traffic(str(src), str(counters)) == 1.25e9
    # ... code does
    src.write_text("__global__ void k() { }\n")
    assert bench.measured_traffic(str(src), str(counters)) is None
    assert bench.measured_traffic(str(src), str(tmp_path / "missing.json")) is None
    counters.write_text("not json")
    assert bench.measured_traffic(str(src), str(counters)) is None


def test_traffic_tracks_the_kernel_header(tmp_path):
    """The kernels compile from a header too: a change of its code voids the
    counters, a change of its comments does not."""
    src, hdr = tmp_path / "kernels.hip", tmp_path / "internal.h"
    src.write_text("__global__ void k() {}\n")
    hdr.write_text("constexpr int kBlock = 256;  // threads\n")
    counters = tmp_path / "counters.json"
    counters.write_text(json.dumps({"kernel_code_sha256": bench.kernel_code_hash(str(src), str(hdr)),
                                    "traffic_bytes_per_launch": 2.5e9}))
    files = (str(src), str(hdr))
    assert bench.measured_traffic(files, str(counters)) == 2.5e9
    hdr.write_text("// block size\nconstexpr int kBlock = 256;\n")
    assert bench.measured_traffic(files, str(counters)) == 2.5e9
    hdr.write_text("constexpr int kBlock = 128;\n")
    assert bench.measured_traffic(files, str(counters)) is None
    assert bench.measured_traffic(str(src), str(counters)) is None
    # the shipped sources are the kernels and their header
    assert [os.path.basename(f) for f in bench.KERNEL_SOURCES] == ["bte_kernels.hip",
                                                                   "bte_internal.h"]


def test_sweep_bytes_of_the_explicit_paper_demo():
    # forward Euler reads I^n once and writes I^{n+1}
    inst = I.config_f1()
    assert inst.n_dof == 120 * 120 * 20 * 55
    assert bench.sweep_bytes(inst, 8) == inst.n_dof * 16 + 55 * 120 * 120 * 16


def test_workload_defaults():
    """Every single-geometry workload has a generator; c3 and c4 default to
    FP32 storage (their configuration), c4's FP64 state does not fit one GPU,
    and the paper context quotes the paper's ~18x with its hardware."""
    for name, wl in bench.WORKLOADS.items():
        inst = I.CONFIGS[name]()
        assert wl["steps"] == inst.nsteps
    assert bench.WORKLOADS["c3"]["precision"] == "fp32"
    assert bench.WORKLOADS["c4"]["precision"] == "fp32" and not bench.WORKLOADS["c4"]["fp64_fits"]
    pc = bench.PAPER_CONTEXT
    assert pc["paper_speedup"] == 18.0 and "A6000" in pc["gpu"] and "Cascade Lake" in pc["cpu"]
    assert pc["precision"] == "FP64"
