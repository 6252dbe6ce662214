"""Batched persistent stepping of uneven geometries (and its HIP graph), and
the sweep-layout autotuner.  Every geometry of a batch must give exactly the
results it gives when stepped alone (the batch runs the same arithmetic in
the same order), graph replays included."""
import os
import sys
import tempfile

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


def same(name, got, want, inst=None):
    """Bitwise comparison that reports where and by how much arrays differ."""
    got, want = np.asarray(got), np.asarray(want)
    if np.array_equal(got, want):
        return True
    bad = np.argwhere(got != want)
    rel = np.abs(got - want) / np.maximum(np.abs(want), 1e-300)
    print(f"{name}: {len(bad)} of {got.size} differ; max rel {rel.max():.3e}", flush=True)
    for idx in bad[:8]:
        where = tuple(int(v) for v in idx)
        if inst is not None:
            P = where[-1]
            nx, ny, _ = inst.n
            where = where + ((P % nx, (P // nx) % ny, P // (nx * ny)),)
        print(f"   at {where}: got {got[tuple(idx)]!r} want {want[tuple(idx)]!r}", flush=True)
    return False


def geometries(precision):
    g = [I.strip_2d(48, 40, 2, 8, 6, seed=1, nsteps=3),
         I.gaussian_3d(10, 9, 8, 2, 8, 4, seed=2, sigma_cells=2.0, precision=precision, nsteps=3),
         I.strip_2d(130, 70, 2, 12, 5, seed=3, strip_cells=10, nsteps=3),
         I.gaussian_3d(17, 12, 9, 4, 8, 3, seed=4, sigma_cells=2.5, precision=precision, nsteps=3),
         I.strip_2d(20, 33, 3, 8, 4, seed=5, nsteps=3)]
    for inst in g:
        inst.precision = precision
    return g


@pytest.mark.parametrize("use_graph", [True, False])
@pytest.mark.parametrize("precision", [I.PRECISION_FP64, I.PRECISION_FP32_MIXED])
def test_batch_equals_solo_runs(gpu, use_graph, precision):
    import torch
    insts = geometries(precision)
    stream = torch.cuda.Stream()
    nsteps = 3
    announce(f"batch of {len(insts)} geometries, graph={use_graph}, precision={precision}")
    solos = []
    for inst in insts:
        with gpu.Solver(inst, stream=stream) as s:
            st = s.step(nsteps)
            solos.append((st, s.temperature(), s.intensity()))
    with gpu.Solver(insts[0], stream=stream) as s:  # solo runs are reproducible
        st = s.step(nsteps)
        assert [x["inner"] for x in st] == [x["inner"] for x in solos[0][0]]
        assert same("solo rerun T", s.temperature(), solos[0][1])
        assert same("solo rerun I", s.intensity(), solos[0][2], insts[0])
    announce("solo runs done; creating the batch")
    sols = [gpu.Solver(inst, stream=stream) for inst in insts]
    with gpu.Batch(sols, use_graph=use_graph) as batch:
        per_step = []
        for k in range(nsteps):
            announce(f"batch step {k}")
            per_step.append(batch.step(1)[0])  # eager host work between graph replays
            for i, s in enumerate(sols):  # every step checked against the solo run
                assert per_step[-1][i]["converged"]
        ok = True
        for i, s in enumerate(sols):
            st, T, Iq = solos[i]
            assert [per_step[k][i]["inner"] for k in range(nsteps)] == [x["inner"] for x in st]
            ok &= same(f"geometry {i} T", s.temperature(), T, insts[i])
            ok &= same(f"geometry {i} I", s.intensity(), Iq, insts[i])
        assert ok
    # the contexts keep working on their own after the batch
    for s in sols:
        s.step(1)
        s.close()


WALK, FLAT = 1, 3  # kernel families: column walk, flattened (x, y) plane


@pytest.mark.parametrize("layout3d", [((WALK, 1, 4), (WALK, 2, 2)), ((FLAT, 0, 2), (FLAT, 0, 4))])
@pytest.mark.parametrize("precision", [I.PRECISION_FP64, I.PRECISION_FP32_MIXED])
def test_batch_mixes_3d_layouts(gpu, monkeypatch, precision, layout3d):
    """3D geometries of one batch may hold 2 rows x 2 planes or 1 row x 4
    planes per wave (column walk), or 2 or 4 planes of the flattened (x, y)
    plane (the default for these narrow meshes, used by the other batch
    tests; 4 planes run in a persistent launch of their own); each still
    gives its solo result bit for bit."""
    import torch
    insts = geometries(precision)
    layouts = [None, layout3d[0], None, layout3d[1], None]
    stream = torch.cuda.Stream()
    announce(f"batch with 3D layouts {layouts}, precision={precision}")

    def make(i):
        names = ("BTE_SWEEP_KIND", "BTE_SWEEP_RY", "BTE_SWEEP_RZ")
        for name, v in zip(names, layouts[i] or (None, None, None)):
            if v is None:
                monkeypatch.delenv(name, raising=False)
            else:
                monkeypatch.setenv(name, str(v))
        return gpu.Solver(insts[i], stream=stream)

    solos = []
    for i in range(len(insts)):
        with make(i) as s:
            st = s.step(3)
            solos.append(([x["inner"] for x in st], s.temperature(), s.intensity()))
    sols = [make(i) for i in range(len(insts))]
    with gpu.Batch(sols, use_graph=True) as batch:
        st = batch.step(3)
    ok = True
    for i, s in enumerate(sols):
        assert [st[k][i]["inner"] for k in range(3)] == solos[i][0]
        ok &= same(f"geometry {i} T", s.temperature(), solos[i][1], insts[i])
        ok &= same(f"geometry {i} I", s.intensity(), solos[i][2], insts[i])
        s.close()
    assert ok


def degenerate_geometries(precision):
    """One-cell-wide axes and single cells, 2D and 3D, with a wall mix per
    face, beside one ordinary mesh of each dimension."""
    rng = np.random.default_rng(90)
    g = [I.strip_2d(1, 9, 2, 8, 4, seed=91, strip_cells=1, nsteps=3),
         I.strip_2d(11, 1, 2, 8, 4, seed=92, strip_cells=1, nsteps=3),
         I.strip_2d(1, 1, 2, 8, 4, seed=93, strip_cells=1, nsteps=3),
         I.strip_2d(20, 33, 3, 8, 4, seed=94, nsteps=3)]
    g += [I.gaussian_3d(*n, 2, 8, 3, seed=95 + i, sigma_cells=1.0, precision=precision, nsteps=3)
          for i, n in enumerate([(1, 6, 5), (7, 1, 4), (6, 5, 1), (1, 1, 1), (1, 1, 7), (10, 9, 8)])]
    kinds = [I.WALL_ISOTHERMAL, I.WALL_SPECULAR, I.WALL_SYMMETRY, I.WALL_ISOTHERMAL,
             I.WALL_SPECULAR, I.WALL_ISOTHERMAL]
    for inst in g:
        inst.precision = precision
        inst.wall = kinds[:2 * inst.dim] + [I.WALL_ISOTHERMAL] * (6 - 2 * inst.dim)
        inst.wall_T = [rng.uniform(296.0, 330.0, inst.wall_face_count(f))
                       if f < 2 * inst.dim and inst.wall[f] == I.WALL_ISOTHERMAL else None
                       for f in range(6)]
        inst.T_init = rng.uniform(295.0, 325.0, inst.n_cells)
    return g


@pytest.mark.parametrize("precision", [I.PRECISION_FP64, I.PRECISION_FP32_MIXED])
def test_batch_of_degenerate_meshes(gpu, precision):
    import torch
    insts = degenerate_geometries(precision)
    stream = torch.cuda.Stream()
    nsteps = 3
    announce(f"batch of {len(insts)} degenerate geometries, precision={precision}")
    solos = []
    for inst in insts:
        with gpu.Solver(inst, stream=stream) as s:
            st = s.step(nsteps)
            solos.append(([x["inner"] for x in st], s.temperature(), s.intensity()))
    announce("solo runs done; creating the batch")
    sols = [gpu.Solver(inst, stream=stream) for inst in insts]
    with gpu.Batch(sols, use_graph=True) as batch:
        st = batch.step(nsteps)
    ok = True
    for i, s in enumerate(sols):
        assert [st[k][i]["inner"] for k in range(nsteps)] == solos[i][0]
        ok &= same(f"geometry {i} T", s.temperature(), solos[i][1], insts[i])
        ok &= same(f"geometry {i} I", s.intensity(), solos[i][2], insts[i])
        s.close()
    assert ok


@pytest.mark.parametrize("train_steps", [(3, 3, 3), (3, 4, 3)])
def test_batch_with_learned_warm_start(gpu, train_steps):
    """The networks of a batch train together when their training falls due
    in the same step (and in separate groups when it does not); each geometry
    still matches its solo run bit for bit, losses included."""
    import torch
    insts = geometries(I.PRECISION_FP32_MIXED)[:3]
    stream = torch.cuda.Stream()

    def opts(i):
        return dict(precision=gpu.BTE_FP32_MIXED, warm_start=gpu.BTE_WARM_T,
                    nn_train_steps=train_steps[i], nn_seed=2)
    announce(f"batch with warm start (train after {train_steps} steps)")
    ref = []
    for i, inst in enumerate(insts):
        with gpu.Solver(inst, stream=stream, **opts(i)) as s:
            st = s.step(7)
            ref.append(([x["inner"] for x in st], s.temperature(),
                        [x["nn_loss"] for x in st]))
    announce("solo runs done; batch of the same")
    sols = [gpu.Solver(inst, stream=stream, **opts(i)) for i, inst in enumerate(insts)]
    with gpu.Batch(sols) as batch:
        st = batch.step(7)
    for i, s in enumerate(sols):
        n = train_steps[i]
        assert [st[k][i]["inner"] for k in range(7)] == ref[i][0]
        assert st[n - 1][i]["trained"] == 1 and all(st[k][i]["warm"] for k in range(n, 7))
        assert [st[k][i]["nn_loss"] for k in range(7)] == ref[i][2]
        assert same(f"warm geometry {i} T", s.temperature(), ref[i][1], insts[i])
        s.close()


def test_batch_rejects_mixed_precision(gpu):
    import torch
    stream = torch.cuda.Stream()
    a = gpu.Solver(I.strip_2d(20, 20, 1, 8, 3, seed=1), stream=stream)
    b = gpu.Solver(I.strip_2d(20, 20, 1, 8, 3, seed=1), stream=stream, precision=gpu.BTE_FP32_MIXED)
    with pytest.raises(gpu.BteError) as e:
        gpu.Batch([a, b])
    assert e.value.code == gpu.BTE_E_INVAL
    a.close()
    b.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_autotune_picks_a_layout_and_caches_it(gpu, dim):
    from oracle import Oracle
    if dim == 2:
        inst = I.strip_2d(64, 48, 4, 8, 10, seed=6, nsteps=2)
        shapes = {(4, 1), (8, 1)}
    else:
        inst = I.gaussian_3d(20, 18, 11, 2, 8, 6, seed=6, sigma_cells=2.5,
                             precision=I.PRECISION_FP64, nsteps=2)
        shapes = {(2, 2), (1, 4), (2, 4), (0, 4), (0, 2)}  # 0 rows: flattened plane
    announce(f"autotune {dim}D")
    with tempfile.TemporaryDirectory() as d:
        cache = os.path.join(d, "tune.txt")
        with gpu.Solver(inst) as s:
            ry, rz, ndg, ms = s.autotune(cache)
            assert (ry, rz) in shapes and ndg >= 1 and ms > 0
            ref = Oracle(inst)
            sched = [x["inner"] for x in ref.run(2)]
            s.step(2, fixed_inner=sched)
            T = s.temperature()
        assert np.max(np.abs(T - ref.temperature()) / ref.temperature()) <= 1e-10
        text = open(cache).read()
        assert f"ry={ry} rz={rz} ndg={ndg}" in text
        with gpu.Solver(inst) as s2:
            assert s2.autotune(cache)[:3] == (ry, rz, ndg)  # read back from the cache
            with pytest.raises(gpu.BteError):
                s2.autotune(None, ry=3)  # no such layout
        assert open(cache).read() == text
        with gpu.Solver(inst) as s3:  # restricted to what a batch accepts
            rb, zb, gb, ms = s3.autotune(cache, batch=True)
            # one direction group; 4 rows in 2D, and 4 planes of the flattened
            # plane on this narrow 3D mesh (the batch fills the device)
            assert (rb, zb) == ((4, 1) if dim == 2 else (0, 4))
            assert gb == 1 and ms > 0
        # the batch choice is recorded apart from the single-geometry one
        assert f" batch -> ry={rb} rz={zb} ndg=1" in open(cache).read()
        with gpu.Solver(inst) as s4:
            assert s4.autotune(cache)[:3] == (ry, rz, ndg)


@pytest.mark.parametrize("precision", [I.PRECISION_FP64, I.PRECISION_FP32_MIXED])
def test_batch_matches_oracle(gpu, precision):
    """Every geometry of a graph-replayed batch against the FP64 oracle, both
    free-running to a tight tolerance (where any two correct solvers land on
    the unique fixed point): FP64 within 1e-10 (sweep counts within one of
    the oracle's), FP32 storage within 1e-5 in T."""
    import torch
    from oracle import Oracle
    tol = 1e-12 if precision == I.PRECISION_FP64 else 1e-10
    insts = [inst.copy(tol=tol) for inst in geometries(precision)]
    nsteps = 3
    stream = torch.cuda.Stream()
    announce(f"batch of {len(insts)} against the oracle, precision={precision}, tol={tol:g}")
    sols = [gpu.Solver(inst, stream=stream) for inst in insts]
    with gpu.Batch(sols, use_graph=True) as batch:
        st = batch.step(nsteps)
    worst_T, worst_I = 0.0, 0.0
    for i, (inst, s) in enumerate(zip(insts, sols)):
        ref = Oracle(inst)
        ref_st = ref.run(nsteps)
        T, Iq = s.temperature(), s.intensity()
        s.close()
        k_gpu = [st[k][i]["inner"] for k in range(nsteps)]
        k_ref = [x["inner"] for x in ref_st]
        errT = float(np.max(np.abs(T - ref.temperature()) / ref.temperature()))
        I_ref = np.ascontiguousarray(ref.intensity().transpose(2, 1, 0))
        errI = float(np.max(np.abs(Iq - I_ref) / np.abs(I_ref)))
        print(f"geometry {i} {inst.name}: sweeps {k_gpu} oracle {k_ref}, T {errT:.2e} "
              f"I {errI:.2e}", flush=True)
        if precision == I.PRECISION_FP64:  # FP32 rounding moves the tight stop by a few sweeps
            assert all(abs(a - b) <= 1 for a, b in zip(k_gpu, k_ref))
        worst_T, worst_I = max(worst_T, errT), max(worst_I, errI)
    if precision == I.PRECISION_FP64:
        assert worst_T <= 1e-10 and worst_I <= 1e-10
    else:
        assert worst_T <= 1e-5 and worst_I <= 1e-4
