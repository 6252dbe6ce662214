"""Static checks on the gfx950 assembly of the HIP kernels (runs on the CPU).

A workgroup barrier must be reached by every wave in uniform control flow.
The persistent batched sweep is the only kernel that executes barriers inside
a loop; if the compiler ever nests that loop (it does when a lane-divergent
condition is threaded across the back-edge), lanes other than the one that
claims work items spin on the inner loop's barrier and the kernel never
finishes.  The flattened-plane sweep also keeps one barrier inside its direction loop
(its tile's staging buffer), marked in the assembly by an inline-asm comment.
The check: the marked barrier sits exactly one loop level below the kernel's
other barriers; in the persistent sweep kernels every other s_barrier sits at
loop depth 1 (the work loop), and in every other kernel at depth 0.
"""
import os
import re
import shutil
import subprocess

import pytest

from paper_2305_19400_amd import build as B

SOURCES = ["bte_kernels.hip", "bte_nn.hip"]


MARK = "bte: direction-loop barrier"


def barrier_depths(asm: str):
    """{kernel symbol: [(loop depth, marked) of each s_barrier]} from compiler
    assembly, using the loop annotations the AMDGPU backend writes on block
    labels; a barrier is marked when the direction-loop marker comment is the
    last one seen before it."""
    out, fn, depth, marked = {}, None, 0, False
    for line in asm.splitlines():
        m = re.match(r"^(_Z\w+):", line)
        if m:
            fn, depth, marked = m.group(1), 0, False
            continue
        if re.match(r"^\.LBB\S+:|^; %bb\.\d+:", line):
            d = re.search(r"Depth=(\d+)", line)
            depth = int(d.group(1)) if d else 0
            continue
        h = re.search(r"Loop Header: Depth=(\d+)", line)
        if h:
            depth = int(h.group(1))
            continue
        if MARK in line:
            marked = True
            continue
        if fn and re.search(r"\ts_barrier\b", line):
            out.setdefault(fn, []).append((depth, marked))
            marked = False
    return out


def test_parser_sees_nested_loop_barriers():
    asm = "\n".join([
        "_ZN3bte1kEv:", "; %bb.0:", "\ts_barrier",
        ".LBB0_1:  ; =>This Loop Header: Depth=1", "\ts_barrier",
        ".LBB0_2:  ;   in Loop: Header=BB0_1 Depth=1",
        ".LBB0_3:  ; =>  This Loop Header: Depth=2", "\t;;#ASMSTART", "\t; " + MARK,
        "\t;;#ASMEND", "\ts_waitcnt lgkmcnt(0)", "\ts_barrier", "\ts_barrier",
        ".LBB0_4:  ; %exit", "\ts_barrier"])
    assert barrier_depths(asm) == {"_ZN3bte1kEv": [(0, False), (1, False), (2, True), (2, False),
                                                   (0, False)]}


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
        base = 1 if "batch_sweep_kernel" in fn else 0
        for depth, marked in ds:
            want = base + 1 if marked else base
            assert depth == want, f"{fn}: barrier at loop depth {depth}, expected {want} ({ds})"
        if "sweep3d_flat_kernel" not in fn and "batch_sweep_kernel" not in fn:
            assert not any(m for _, m in ds), f"{fn}: unexpected direction-loop barrier"
    flat = [fn for fn in depths if "sweep3d_flat_kernel" in fn]
    if src == "bte_kernels.hip":
        assert flat and all(any(m for _, m in depths[fn]) for fn in flat)
    if src == "bte_kernels.hip":
        persistent = [fn for fn in depths if "batch_sweep_kernel" in fn]
        assert len(persistent) == 12  # 3 work lists x 2 storage precisions x stored or decoded items
