"""Every sweep layout the autotuner may choose gives the oracle's answer.

Ragged meshes that span two x tiles (the last one partly filled), row and
plane counts that are not multiples of a block, and a different wall kind on
each face, so every edge path of the column-walk sweeps (neighbouring tile,
isothermal table, mirrored direction; first and last rows, planes and lanes)
is exercised in every layout.  Narrow meshes (23 cells along x in 2D, 13 in
3D) leave most lanes of a column-walk tile idle, and put several rows, and
x walls, inside one wave of the flattened-plane layout.
FP64 within 1e-10 relative with the oracle's sweep schedule replayed; FP32
storage within 1e-5 relative in T.
"""
import sys

import numpy as np
import pytest

from paper_2305_19400_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2305_19400_amd import bte
    bte.load_library()
    return bte


def announce(msg):
    print(f"\n[case] {msg}", flush=True)
    sys.stdout.flush()


def mixed_walls(inst, seed):
    """Isothermal (random face temperatures), specular and symmetry walls mixed
    over the faces, and a random initial field."""
    rng = np.random.default_rng(seed)
    kinds = [I.WALL_ISOTHERMAL, I.WALL_SPECULAR, I.WALL_SYMMETRY, I.WALL_ISOTHERMAL,
             I.WALL_SPECULAR, I.WALL_ISOTHERMAL]
    inst.wall = kinds[:2 * inst.dim] + [I.WALL_ISOTHERMAL] * (6 - 2 * inst.dim)
    inst.wall_T = [rng.uniform(296.0, 330.0, inst.wall_face_count(f))
                   if f < 2 * inst.dim and inst.wall[f] == I.WALL_ISOTHERMAL else None
                   for f in range(6)]
    inst.T_init = rng.uniform(295.0, 325.0, inst.n_cells)
    return inst


def case_2d():
    inst = I.strip_2d(70, 37, 2, 8, 4, seed=51, nsteps=2)
    inst.name = "layouts2d_70x37"
    return mixed_walls(inst, 52)


def case_2d_narrow():
    inst = I.strip_2d(23, 30, 2, 8, 4, seed=58, nsteps=2)
    inst.name = "layouts2d_23x30"
    return mixed_walls(inst, 59)


def case_3d():
    # flattened plane: 4 plane tiles x 2 (4 planes) or 4 (2 planes) z blocks, a
    # tile count divisible by 8, so its launch takes the XCD-ordered tile mapping
    # (the narrow case below does not)
    inst = I.gaussian_3d(70, 11, 7, 2, 8, 3, seed=53, precision=I.PRECISION_FP64, nsteps=2)
    inst.h = [1e-8, 1.2e-8, 0.9e-8]
    inst.name = "layouts3d_70x11x7"
    return mixed_walls(inst, 54)


def case_3d_narrow():
    inst = I.gaussian_3d(13, 9, 10, 2, 8, 3, seed=55, precision=I.PRECISION_FP64, nsteps=2)
    inst.h = [1.1e-8, 0.8e-8, 1e-8]
    inst.name = "layouts3d_13x9x10"
    return mixed_walls(inst, 56)


def case_3d_wide():
    # rows longer than the flattened plane's 256-cell tile: every y-upwind
    # cell lies in the tile's halo, and tile ends fall inside rows
    inst = I.gaussian_3d(300, 3, 5, 2, 8, 3, seed=60, precision=I.PRECISION_FP64, nsteps=2)
    inst.h = [0.9e-8, 1.1e-8, 1e-8]
    inst.name = "layouts3d_300x3x5"
    return mixed_walls(inst, 61)


CASES = {"2d": case_2d, "2dn": case_2d_narrow, "3d": case_3d, "3dn": case_3d_narrow,
         "3dw": case_3d_wide}
KIND_WALK, KIND_FLAT = 1, 3  # kernel families (ry = 0: flattened (x, y) plane, 3D)
LAYOUTS = [("2d", 4, 0, 1), ("2d", 8, 0, 3), ("2d", 16, 0, 2),
           ("2dn", 4, 0, 2), ("2dn", 8, 0, 1),
           ("3d", 2, 2, 1), ("3d", 1, 4, 2), ("3d", 2, 4, 3), ("3d", 0, 4, 1), ("3d", 0, 2, 2),
           ("3dn", 2, 2, 1), ("3dn", 1, 4, 3), ("3dn", 0, 4, 2), ("3dn", 0, 2, 1),
           ("3dw", 0, 4, 1), ("3dw", 0, 2, 2)]


def set_layout(monkeypatch, ry, rz, ndg):
    monkeypatch.setenv("BTE_SWEEP_KIND", str(KIND_FLAT if ry == 0 else KIND_WALK))
    monkeypatch.setenv("BTE_SWEEP_RY", str(ry))
    monkeypatch.setenv("BTE_SWEEP_RZ", str(rz))
    monkeypatch.setenv("BTE_SWEEP_NDG", str(ndg))


@pytest.mark.parametrize("dim,ry,rz,ndg", LAYOUTS)
def test_layout_matches_oracle(gpu, monkeypatch, dim, ry, rz, ndg):
    from oracle import Oracle
    inst = CASES[dim]()
    set_layout(monkeypatch, ry, rz, ndg)
    ref = Oracle(inst)
    sched = [s["inner"] for s in ref.run(inst.nsteps)]
    announce(f"{inst.name} ry={ry} rz={rz} ndg={ndg} sched={sched}")
    with gpu.Solver(inst) as sol:
        kind = 1 if dim.startswith("2d") else (KIND_FLAT if ry == 0 else 2)
        assert sol.sweep_layout() == dict(kind=kind, ry=ry, rz=max(rz, 1), ndg=ndg)
        sol.step(inst.nsteps, fixed_inner=sched)
        T, Iq = sol.temperature(), sol.intensity()
    I_ref = np.ascontiguousarray(ref.intensity().transpose(2, 1, 0))
    errT = float(np.max(np.abs(T - ref.temperature()) / ref.temperature()))
    errI = float(np.max(np.abs(Iq - I_ref) / np.abs(I_ref)))
    print(f"T {errT:.2e} I {errI:.2e}", flush=True)
    assert errT <= 1e-10 and errI <= 1e-10


@pytest.mark.parametrize("dim,ry,rz,ndg", [("2d", 16, 0, 2), ("3d", 2, 2, 1), ("3d", 1, 4, 2),
                                             ("3d", 2, 4, 3), ("3d", 0, 4, 1), ("3d", 0, 2, 2),
                                             ("3dn", 1, 4, 1), ("3dw", 0, 4, 2)])
def test_explicit_layout_matches_oracle(gpu, monkeypatch, dim, ry, rz, ndg):
    """Forward-Euler steps (one sweep each, the update scaled by dt instead of
    the implicit diagonal) through every sweep family and layout."""
    from oracle import Oracle
    inst = CASES[dim]()
    dt = 2e-13  # inside the forward-Euler stability limit of these meshes
    set_layout(monkeypatch, ry, rz, ndg)
    ref = Oracle(inst, scheme=I.SCHEME_EXPLICIT_EULER, dt=dt)
    ref_st = ref.run(4)
    announce(f"{inst.name} explicit ry={ry} rz={rz} ndg={ndg}")
    with gpu.Solver(inst, scheme=I.SCHEME_EXPLICIT_EULER, dt=dt) as sol:
        st = sol.step(4)
        T, Iq = sol.temperature(), sol.intensity()
    assert all(s["inner"] == 1 for s in st) and all(s["inner"] == 1 for s in ref_st)
    I_ref = np.ascontiguousarray(ref.intensity().transpose(2, 1, 0))
    errT = float(np.max(np.abs(T - ref.temperature()) / ref.temperature()))
    errI = float(np.max(np.abs(Iq - I_ref) / np.abs(I_ref)))
    print(f"explicit T {errT:.2e} I {errI:.2e}", flush=True)
    assert errT <= 1e-10 and errI <= 1e-10
    assert float(np.max(np.abs(T - inst.T_init))) > 1e-3  # the steps changed the field


DEGENERATE = [(2, (1, 9), None), (2, (1, 9), (16, 0, 2)), (2, (11, 1), None), (2, (11, 1), "cell"),
              (2, (1, 1), None), (3, (1, 6, 5), None), (3, (1, 6, 5), (2, 2, 1)),
              (3, (7, 1, 4), (1, 4, 2)), (3, (7, 1, 4), (0, 4, 1)), (3, (6, 5, 1), (2, 4, 3)),
              (3, (6, 5, 1), None), (3, (1, 1, 1), None), (3, (1, 1, 1), (2, 2, 1)),
              (3, (1, 1, 7), (0, 4, 1)), (3, (1, 1, 7), (1, 4, 1))]


@pytest.mark.parametrize("dim,n,layout", DEGENERATE)
def test_degenerate_mesh_matches_oracle(gpu, monkeypatch, dim, n, layout):
    """Axes one cell wide (every cell between two walls of that axis) and
    single-cell meshes, in 2D and 3D, through the default and requested
    layouts, with the mixed wall kinds."""
    from oracle import Oracle
    seed = 70 + sum(n)
    if dim == 2:
        inst = I.strip_2d(n[0], n[1], 2, 8, 4, seed=seed, strip_cells=1, nsteps=2)
    else:
        inst = I.gaussian_3d(n[0], n[1], n[2], 2, 8, 3, seed=seed, sigma_cells=1.0,
                             precision=I.PRECISION_FP64, nsteps=2)
    inst.name = f"degenerate{dim}d_" + "x".join(str(v) for v in n)
    inst = mixed_walls(inst, seed + 10)
    if layout == "cell":
        monkeypatch.setenv("BTE_SWEEP_KIND", "0")
    elif layout is not None:
        set_layout(monkeypatch, *layout)
    ref = Oracle(inst)
    sched = [s["inner"] for s in ref.run(inst.nsteps)]
    announce(f"{inst.name} layout={layout} sched={sched}")
    with gpu.Solver(inst) as sol:
        if layout == "cell":
            assert sol.sweep_layout()["kind"] == 0
        sol.step(inst.nsteps, fixed_inner=sched)
        T, Iq = sol.temperature(), sol.intensity()
    I_ref = np.ascontiguousarray(ref.intensity().transpose(2, 1, 0))
    errT = float(np.max(np.abs(T - ref.temperature()) / ref.temperature()))
    errI = float(np.max(np.abs(Iq - I_ref) / np.abs(I_ref)))
    print(f"T {errT:.2e} I {errI:.2e}", flush=True)
    assert errT <= 1e-10 and errI <= 1e-10
    assert float(np.max(np.abs(T - inst.T_init))) > 1e-3


@pytest.mark.parametrize("dim,layout", [("2d", None), ("3d", None), ("3dn", None), ("3dw", None),
                                        ("2d", (8, 0, 3)), ("3d", (1, 4, 2)), ("3d", (0, 4, 1)),
                                        ("3dn", (2, 2, 2)), ("2d", "cell"), ("3dn", "cell")])
def test_fp32_explicit_matches_oracle(gpu, monkeypatch, dim, layout):
    """FP32 storage with forward-Euler steps, through every kernel family: the
    tiled kernels take the defect form of the update there (the direct form
    they use under backward Euler lacks the -(1/tau + sum c) I^n term), and
    every layout matches the FP64 oracle to the FP32 bar."""
    from oracle import Oracle
    inst = CASES[dim]()
    dt = 2e-13
    if layout == "cell":
        monkeypatch.setenv("BTE_SWEEP_KIND", "0")
    elif layout is not None:
        set_layout(monkeypatch, *layout)
    ref = Oracle(inst, scheme=I.SCHEME_EXPLICIT_EULER, dt=dt)
    ref.run(4)
    announce(f"{inst.name} fp32 explicit, layout {layout}")
    with gpu.Solver(inst, precision=gpu.BTE_FP32_MIXED, scheme=I.SCHEME_EXPLICIT_EULER,
                    dt=dt) as sol:
        lay = sol.sweep_layout()
        if layout == "cell":
            assert lay["kind"] == 0
        elif layout is not None:
            kind = 1 if dim.startswith("2d") else (KIND_FLAT if layout[0] == 0 else 2)
            assert lay == dict(kind=kind, ry=layout[0], rz=max(layout[1], 1), ndg=layout[2])
        else:
            assert lay["kind"] != 0
        st = sol.step(4)
        T, Iq = sol.temperature(), sol.intensity()
    assert all(s["inner"] == 1 for s in st)
    I_ref = np.ascontiguousarray(ref.intensity().transpose(2, 1, 0))
    errT = float(np.max(np.abs(T - ref.temperature()) / ref.temperature()))
    errI = float(np.max(np.abs(Iq - I_ref) / np.abs(I_ref)))
    print(f"fp32 explicit T {errT:.2e} I {errI:.2e}", flush=True)
    assert errT <= 1e-5 and errI <= 1e-5
    assert float(np.max(np.abs(T - inst.T_init))) > 1e-3


def test_fp32_explicit_autotunes(gpu):
    """FP32 storage with forward Euler is no longer tied to one kernel family:
    the autotuner searches the 3D layouts and the tuned layout still matches
    the oracle."""
    from oracle import Oracle
    inst = CASES["3dn"]()
    dt = 2e-13
    ref = Oracle(inst, scheme=I.SCHEME_EXPLICIT_EULER, dt=dt)
    ref.run(2)
    announce(f"{inst.name} fp32 explicit autotune")
    with gpu.Solver(inst, precision=gpu.BTE_FP32_MIXED, scheme=I.SCHEME_EXPLICIT_EULER,
                    dt=dt) as sol:
        ry, rz, ndg, ms = sol.autotune()
        assert ms > 0 and sol.sweep_layout()["kind"] in (2, KIND_FLAT)
        sol.step(2)
        T = sol.temperature()
    errT = float(np.max(np.abs(T - ref.temperature()) / ref.temperature()))
    print(f"tuned ({ry}, {rz}, {ndg}): T {errT:.2e}", flush=True)
    assert errT <= 1e-5


@pytest.mark.parametrize("dim,ry,rz,ndg", [("2d", 8, 0, 3), ("2dn", 4, 0, 1), ("3d", 1, 4, 2),
                                             ("3d", 0, 4, 1), ("3dn", 0, 2, 2), ("3dw", 0, 4, 1)])
def test_layout_fp32_matches_oracle(gpu, monkeypatch, dim, ry, rz, ndg):
    from oracle import Oracle
    inst = CASES[dim]()
    set_layout(monkeypatch, ry, rz, ndg)
    ref = Oracle(inst)
    sched = [s["inner"] for s in ref.run(inst.nsteps)]
    announce(f"{inst.name} fp32 ry={ry} rz={rz} ndg={ndg}")
    with gpu.Solver(inst, precision=gpu.BTE_FP32_MIXED) as sol:
        sol.step(inst.nsteps, fixed_inner=sched)
        T = sol.temperature()
    errT = float(np.max(np.abs(T - ref.temperature()) / ref.temperature()))
    print(f"fp32 T {errT:.2e}", flush=True)
    assert errT <= 1e-5


@pytest.mark.parametrize("dim", ["3d", "3dn", "3dw"])
def test_warm_start_shift_is_layout_independent(gpu, monkeypatch, dim):
    """The first sweep of a warm-started step adds the equilibrium shift at the
    guessed temperature to every inflow value (neighbour, edge, mirrored
    ghost).  The trained network is deterministic, so every 3D layout must
    give the same temperatures; the walk with 2 x 2 per wave is the one the
    oracle checks in the other tests."""
    inst = CASES[dim]()
    inst.nsteps = 6
    opts = dict(warm_start=gpu.BTE_WARM_T_SHIFT, nn_train_steps=3, nn_seed=4)
    results = {}
    for ry, rz in ((2, 2), (1, 4), (0, 4), (0, 2)):
        set_layout(monkeypatch, ry, rz, 1)
        announce(f"{inst.name} warm start with shift, layout ry={ry} rz={rz}")
        with gpu.Solver(inst, **opts) as sol:
            st = sol.step(6, fixed_inner=[8] * 6)
            assert all(x["warm"] for x in st[3:])
            results[(ry, rz)] = sol.temperature()
    ref = results[(2, 2)]
    for key, T in results.items():
        err = float(np.max(np.abs(T - ref) / ref))
        print(f"layout {key}: max rel diff {err:.2e}", flush=True)
        assert err <= 1e-12


@pytest.mark.parametrize("dim,ry,rz", [("2d", 4, 0), ("2dn", 8, 0), ("3d", 1, 4), ("3dn", 0, 2),
                                       ("3d", 0, 4)])
def test_fp32_reaches_tight_tolerance(gpu, monkeypatch, dim, ry, rz):
    """With FP32 storage the iterate must settle: the update is rounded once to
    the stored value and the norms use that value, so a converged sweep
    changes nothing and the increment norm falls to zero instead of stalling
    at rounding noise.  Each step must stop well before the sweep cap."""
    inst = CASES[dim]()
    set_layout(monkeypatch, ry, rz, 1)
    announce(f"{inst.name} fp32 tol 1e-10 ry={ry} rz={rz}")
    with gpu.Solver(inst, precision=gpu.BTE_FP32_MIXED, tol=1e-10, max_inner=200) as sol:
        st = sol.step(3)
    print([x["inner"] for x in st], flush=True)
    assert all(x["converged"] and x["inner"] < 100 for x in st)


def test_default_layouts(gpu, monkeypatch):
    """Without overrides: the flattened plane where 64-column tiles would leave
    lanes idle (4 planes with FP32 storage; with FP64, 4 once the 4-plane
    launch has 8192 workgroups per direction group, else 2), the column walk
    where x is a multiple of 64 (2 x 2 with FP64 storage, 1 x 4 with FP32)."""
    for name in ("BTE_SWEEP_KIND", "BTE_SWEEP_RY", "BTE_SWEEP_RZ", "BTE_SWEEP_NDG"):
        monkeypatch.delenv(name, raising=False)
    meshes = {
        "narrow": case_3d_narrow(),
        "full": I.gaussian_3d(64, 6, 5, 2, 8, 3, seed=57, precision=I.PRECISION_FP64, nsteps=1),
        # 157 plane tiles x 2 blocks of 4 planes x 27 band entries = 8478 workgroups
        "large": I.gaussian_3d(200, 200, 8, 2, 4, 20, seed=58, precision=I.PRECISION_FP64,
                               nsteps=1),
    }
    assert meshes["large"].n_bands == 27
    want = {("narrow", gpu.BTE_FP64): (KIND_FLAT, 0, 2), ("narrow", gpu.BTE_FP32_MIXED): (KIND_FLAT, 0, 4),
            ("full", gpu.BTE_FP64): (2, 2, 2), ("full", gpu.BTE_FP32_MIXED): (2, 1, 4),
            ("large", gpu.BTE_FP64): (KIND_FLAT, 0, 4)}
    for (which, prec), (kind, ry, rz) in want.items():
        with gpu.Solver(meshes[which], precision=prec) as sol:
            lay = sol.sweep_layout()
        assert (lay["kind"], lay["ry"], lay["rz"]) == (kind, ry, rz), (which, prec, lay)


@pytest.mark.parametrize("precision", [I.PRECISION_FP64, I.PRECISION_FP32_MIXED])
def test_2d_padded_rows_in_copies_and_checkpoint(gpu, precision):
    """2D slabs pad each row to a 128-byte line (45 cells: 48 in FP64, 64 in
    FP32 storage), while intensity(), set_fields and the checkpoint use the
    dense [b][d][P] order.  Six steps in one go equal three, a checkpoint
    restored into a fresh context and three more, bit for bit; the
    checkpoint's intensity section is intensity() in storage format; the
    intensity and temperature re-imported through set_fields come back (FP64:
    bit for bit, and the next steps take the same sweeps; FP32 storage
    re-rounds I - Iref, so to 1e-12)."""
    inst = I.strip_2d(45, 23, 2, 8, 4, seed=41, strip_cells=6, nsteps=6)
    nb, nd, nc = inst.n_bands, inst.n_dirs, inst.n_cells
    announce(f"2D padded rows, precision {precision}")
    with gpu.Solver(inst, precision=precision) as a:
        a.step(3)
        state = a.get_state()
        Ia3, Ta3 = a.intensity(), a.temperature()
        sa = a.step(3)
        Ta, Ia = a.temperature(), a.intensity()
    st = gpu.parse_state(state)
    dense = st["I"].astype(np.float64)
    if precision == I.PRECISION_FP32_MIXED:
        dense = st["Iref"][:, None, None] + dense
    assert np.array_equal(dense.reshape(Ia3.shape), Ia3)
    with gpu.Solver(inst, precision=precision) as b:
        b.set_state(state)
        assert np.array_equal(b.intensity(), Ia3)
        assert b.step(3) == sa
        assert np.array_equal(b.temperature(), Ta) and np.array_equal(b.intensity(), Ia)
    with gpu.Solver(inst, precision=precision) as c:
        c.set_fields(Ia3, Ta3)
        assert np.array_equal(c.temperature(), Ta3)
        if precision == I.PRECISION_FP64:
            assert np.array_equal(c.intensity(), Ia3)
            sc = c.step(3)
            assert [s["inner"] for s in sc] == [s["inner"] for s in sa]
        else:
            assert float(np.max(np.abs(c.intensity() - Ia3) / Ia3)) <= 1e-12
    assert Ia3.size == nb * nd * nc
