"""The C-ABI library builds, loads and exports every symbol include/bte.h
declares; host-side validation rejects bad inputs before touching a device.
These run without a GPU (no kernel is launched)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2305_19400_amd import bte, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bte.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(bte_[a-z_]+)\s*\(", src)))


def test_header_matches_binding_exports():
    assert declared_functions() == sorted(bte.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = bte.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", bte.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    syms = {line.split()[-1] for line in out.splitlines() if line.strip()}
    for name in declared_functions():
        assert name in syms, name


def test_library_is_gfx950_code_object():
    """The fat binary embedded in libbte.so (built here) targets gfx950."""
    with open(bte.LIB_PATH, "rb") as f:
        blob = f.read()
    assert b"amdgcn-amd-amdhsa--gfx950" in blob


def test_workspace_size_c2():
    inst = inputs.config_c2()
    n = bte.bte_workspace_size(inst)
    field = inst.n_dof * 8
    assert 3 * field <= n < 3 * field * 1.02 + (1 << 28)  # fields + per-(group, band, cell) partials
    n32 = bte.bte_workspace_size(inst, precision=bte.BTE_FP32_MIXED)
    assert 3 * field // 2 <= n32 < n


def _create_status(inst, workspace=0x100000, nbytes=1 << 40, **opts):
    lib = bte.load_library()
    inp = bte._Inputs(inst, bte._resolve(inst, opts))
    inp.opt.workspace = C.c_void_p(workspace)
    inp.opt.workspace_bytes = nbytes
    ctx = C.c_void_p(0)
    rc = lib.bte_create(C.byref(inp.mesh), C.byref(inp.dirs), C.byref(inp.bands),
                        C.byref(inp.disp), C.byref(inp.opt), C.byref(ctx))
    return rc, lib.bte_last_error().decode()


def test_validation_rejects_bad_inputs_without_device():
    base = inputs.config_c1()
    # direction set not closed under a specular wall's mirror
    s, w = inputs.product_quadrature(1, 7)
    spec = base.copy(s=s, w=w, wall=[1, 1, 0, 0, 0, 0], wall_T=[None, None] + base.wall_T[2:])
    rc, msg = _create_status(spec)
    assert rc == bte.BTE_E_INVAL and "mirror" in msg
    # non-positive band data
    bad = base.copy()
    bad.tau[1] = 0.0
    rc, msg = _create_status(bad)
    assert rc == bte.BTE_E_INVAL and "band 1" in msg
    # bad dt / scheme / precision
    assert _create_status(base, dt=-1.0)[0] == bte.BTE_E_INVAL
    assert _create_status(base, scheme=7)[0] == bte.BTE_E_INVAL
    assert _create_status(base, precision=3)[0] == bte.BTE_E_INVAL
    # non-positive initial temperature
    cold = base.copy()
    cold.T_init[5] = -1.0
    rc, msg = _create_status(cold)
    assert rc == bte.BTE_E_INVAL and "T_init[5]" in msg
    # isothermal wall without temperatures
    nowall = base.copy()
    nowall.wall_T[2] = None
    assert _create_status(nowall)[0] == bte.BTE_E_INVAL
    # 2D mesh with nz != 1
    flat = base.copy(n=[16, 16, 2])
    assert _create_status(flat)[0] == bte.BTE_E_INVAL
    # more cells than 32-bit slab offsets reach (rejected before any array is read)
    huge = base.copy(dim=3, n=[700, 700, 700], h=[1e-8, 1e-8, 1e-8])
    rc, msg = _create_status(huge)
    assert rc == bte.BTE_E_INVAL and "too many cells" in msg
    # a 2D mesh whose cells fit but whose rows, padded to a 128-byte line
    # (16383 -> 16384 cells), do not
    padded = base.copy(n=[16383, 16384, 1])
    for prec in (bte.BTE_FP64, bte.BTE_FP32_MIXED):
        rc, msg = _create_status(padded, precision=prec)
        assert rc == bte.BTE_E_INVAL and "with padding" in msg, msg
    # wall tables past 32-bit offsets: 4 band entries x 10^8 faces of a z side
    wide = base.copy(dim=3, n=[10000, 10000, 2], h=[1e-8, 1e-8, 1e-8])
    rc, msg = _create_status(wide)
    assert rc == bte.BTE_E_INVAL and "wall faces" in msg


def test_workspace_checks_without_device():
    base = inputs.config_c1()
    need = bte.bte_workspace_size(base)
    rc, msg = _create_status(base, workspace=0)
    assert rc == bte.BTE_E_NOMEM
    rc, msg = _create_status(base, nbytes=need - 1)
    assert rc == bte.BTE_E_NOMEM and str(need) in msg
    rc, msg = _create_status(base, workspace=0x100001)
    assert rc == bte.BTE_E_INVAL and "aligned" in msg


def test_null_context_calls_fail_cleanly():
    lib = bte.load_library()
    T = np.zeros(4)
    assert lib.bte_step(None, 1, None, None) == bte.BTE_E_INVAL
    assert lib.bte_temperature(None, T.ctypes.data_as(C.POINTER(C.c_double)), 4) == bte.BTE_E_INVAL
    assert lib.bte_destroy(None) == bte.BTE_OK


def test_explicit_step_limit_without_device():
    """Forward Euler is refused where dt (1/tau_b + sum_a v_b |s_a| / h_a) > 1
    for some band and direction (the update would no longer be a convex
    combination of old values); the message names the largest stable dt."""
    base = inputs.config_c1()
    rate = max(1.0 / base.tau[b] + sum(base.vg[b] * abs(base.s[d, a]) / base.h[a] for a in range(2))
               for b in range(base.n_bands) for d in range(base.n_dirs))
    rc, msg = _create_status(base, scheme=bte.BTE_EXPLICIT_EULER, dt=1.01 / rate)
    assert rc == bte.BTE_E_INVAL and "explicit step too large" in msg
    assert f"{1.0 / rate:.6g}" in msg
    # the implicit scheme has no such limit (it fails later, at the fake workspace)
    rc, msg = _create_status(base, scheme=bte.BTE_IMPLICIT_JACOBI, dt=1.01 / rate)
    assert "explicit step" not in msg
    rc, msg = _create_status(base, scheme=bte.BTE_EXPLICIT_EULER, dt=0.99 / rate)
    assert "explicit step" not in msg


def test_state_header_layout_matches_binding(tmp_path):
    """The checkpoint header as the C compiler lays it out (include/bte.h) is
    the one the binding parses."""
    src = tmp_path / "hdr.c"
    fields = [name for name, _ in bte.bte_state_header._fields_]
    body = "".join(f'  printf("{f} %zu\\n", offsetof(bte_state_header, {f}));\n' for f in fields)
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "bte.h"\nint main(void) {\n'
                   + body + '  printf("size %zu\\n", sizeof(bte_state_header));\n  return 0;\n}\n')
    exe = tmp_path / "hdr"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), "-o", str(exe),
                    str(src)], check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    for f in fields:
        assert int(out[f]) == getattr(bte.bte_state_header, f).offset, f
    assert int(out["size"]) == C.sizeof(bte.bte_state_header)
