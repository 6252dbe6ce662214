"""Static checks on the gfx950 assembly of the HIP kernels (runs on the CPU).

A workgroup barrier must be reached by every wave in uniform control flow.
The persistent batched sweep is the only kernel that executes barriers inside
a loop; if the compiler ever nests that loop (it does when a lane-divergent
condition is threaded across the back-edge), lanes other than the one that
claims work items spin on the inner loop's barrier and the kernel never
finishes.  The check: in every kernel, every s_barrier sits at loop depth
<= 1, and only the persistent sweep kernels have barriers inside a loop.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2305_19400_amd import build as B

SOURCES = ["bte_kernels.hip", "bte_nn.hip"]


def barrier_depths(asm: str):
    """{kernel symbol: [loop depth of each s_barrier]} from compiler assembly,
    using the loop annotations the AMDGPU backend writes on block labels."""
    out, fn, depth = {}, None, 0
    for line in asm.splitlines():
        m = re.match(r"^(_Z\w+):", line)
        if m:
            fn, depth = m.group(1), 0
            continue
        if re.match(r"^\.LBB\S+:|^; %bb\.\d+:", line):
            d = re.search(r"Depth=(\d+)", line)
            depth = int(d.group(1)) if d else 0
            continue
        h = re.search(r"Loop Header: Depth=(\d+)", line)
        if h:
            depth = int(h.group(1))
            continue
        if fn and re.search(r"\ts_barrier\b", line):
            out.setdefault(fn, []).append(depth)
    return out


def test_parser_sees_nested_loop_barriers():
    asm = "\n".join([
        "_ZN3bte1kEv:", "; %bb.0:", "\ts_barrier",
        ".LBB0_1:  ; =>This Loop Header: Depth=1", "\ts_barrier",
        ".LBB0_2:  ;   in Loop: Header=BB0_1 Depth=1",
        ".LBB0_3:  ; =>  This Loop Header: Depth=2", "\ts_barrier",
        ".LBB0_4:  ; %exit", "\ts_barrier"])
    assert barrier_depths(asm) == {"_ZN3bte1kEv": [0, 1, 2, 0]}


@pytest.mark.parametrize("src", SOURCES)
def test_barriers_stay_in_uniform_loops(src, tmp_path):
    if not os.path.exists(B.hipcc()):
        pytest.skip("hipcc not available")
    out = tmp_path / (src + ".s")
    flags = [f for f in B.HIPCC_FLAGS if f not in ("-fPIC", "-shared")]
    subprocess.run([B.hipcc()] + flags + ["--cuda-device-only", "-S", "-o", str(out),
                                          os.path.join(B.CSRC, src)],
                   check=True, capture_output=True)
    depths = barrier_depths(out.read_text())
    assert depths, "no barriers found: assembly format changed?"
    for fn, ds in depths.items():
        assert max(ds) <= 1, f"{fn}: barrier inside a nested loop (depths {ds})"
        if "batch_sweep_kernel" not in fn:
            assert max(ds) == 0, f"{fn}: unexpected barrier inside a loop (depths {ds})"
    if src == "bte_kernels.hip":
        persistent = [fn for fn in depths if "batch_sweep_kernel" in fn]
        assert len(persistent) == 12  # 3 work lists x 2 storage precisions x stored or decoded items
