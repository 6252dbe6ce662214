"""Full-size checks at the 3D and batched workloads' real shapes and launch
layouts, where the oracle cannot hold the state (64^3 x 400 x 55 in FP64 is
138 GB per field): properties that hold at any size.

* Symmetry.  A Gaussian hot spot centred in a cube with six isothermal 300 K
  walls, on a product quadrature that maps onto itself under reflection of
  any axis and under the exchange of x and y, keeps those symmetries: the
  temperature equals its mirror images to rounding.  A wrong halo, tile edge,
  z-block face or XCD tile mapping anywhere in the full-size launch breaks
  it by many orders more.
* Uniform state.  A body at 300 K with 300 K walls is the equilibrium: every
  step leaves the temperature bitwise unchanged.
* The batch (the 64-geometry draw at full size): each geometry equals its solo
  run bit for bit.
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


def centred(inst, sigma=6.0, peak=50.0):
    """The workload's mesh with its hot spot moved to the exact centre."""
    n = inst.n
    z, y, x = np.meshgrid(np.arange(n[2]) + 0.5, np.arange(n[1]) + 0.5, np.arange(n[0]) + 0.5,
                          indexing="ij")
    r2 = (x - n[0] / 2) ** 2 + (y - n[1] / 2) ** 2 + (z - n[2] / 2) ** 2
    out = inst.copy()
    out.T_init = (300.0 + peak * np.exp(-r2 / (2.0 * sigma ** 2))).reshape(-1)
    return out


def mirror_errors(T, n):
    """Largest |T - T'| / (T - 300 K) over the images T' of T under x, y and z
    reflection and the exchange of x and y."""
    f = T.reshape(n[2], n[1], n[0])
    rise = float(f.max()) - 300.0
    images = {"x": f[:, :, ::-1], "y": f[:, ::-1, :], "z": f[::-1, :, :],
              "xy": np.transpose(f, (0, 2, 1))}
    return {k: float(np.max(np.abs(f - g))) / rise for k, g in images.items()}


@pytest.mark.parametrize("workload,precision,tol", [("c4", "fp32", 1e-10), ("c3", "fp64", 1e-11)])
def test_fullsize_symmetry(gpu, workload, precision, tol):
    """Three steps in the default (benchmarked) layout.  The mirrored updates
    differ only in the order of the direction sums (measured: 1e-15 of the
    temperature rise with FP32 storage, whose compensated sums absorb it, and
    5e-14 in FP64)."""
    inst = centred(I.CONFIGS[workload]())
    prec = gpu.BTE_FP64 if precision == "fp64" else gpu.BTE_FP32_MIXED
    announce(f"{workload} full size {precision}: symmetry after 3 steps")
    with gpu.Solver(inst, precision=prec) as sol:
        layout = sol.sweep_layout()
        st = sol.step(3)
        T = sol.temperature()
    err = mirror_errors(T, inst.n)
    print(f"layout {layout}, sweeps {[s['inner'] for s in st]}, rise {T.max() - 300:.3f} K, "
          f"mirror errors (of the rise) {err}", flush=True)
    assert T.max() - 300.0 > 1.0 and T.min() >= 300.0 - 1e-9
    assert all(v <= tol for v in err.values()), err


def test_fullsize_uniform_state_bitwise(gpu):
    """c4's shape, FP32 storage, default layout: the 300 K equilibrium stays
    bitwise 300 K."""
    inst = I.config_c4()
    inst.T_init = np.full(inst.n_cells, 300.0)
    announce("c4 full size fp32: uniform 300 K state, 2 steps")
    with gpu.Solver(inst, precision=gpu.BTE_FP32_MIXED) as sol:
        st = sol.step(2)
        T = sol.temperature()
    print(f"sweeps {[s['inner'] for s in st]}", flush=True)
    assert np.array_equal(T, np.full(inst.n_cells, 300.0))


def test_c5_fullsize_batch_equals_solo(gpu, monkeypatch, tmp_path):
    """The c5 draw at full size (64 geometries, 2.19e10 DOF, 277 GB of
    workspace), FP32 storage, the layouts the autotuner picks for a batch, one
    persistent launch per inner iteration replayed from a HIP graph: after 2
    batched steps the largest 2D and 3D geometries and the smallest one equal
    solo runs in the same layouts bit for bit (solo runs are checked against
    the oracle on smaller meshes)."""
    import torch
    insts = I.config_c5(nsteps=2)
    assert sum(i.n_dof for i in insts) > 2.1e10
    stream = torch.cuda.Stream()
    cache = str(tmp_path / "layouts.txt")
    announce("c5 full draw: creating and tuning 64 contexts")
    sols = []
    for inst in insts:
        s = gpu.Solver(inst, stream=stream, precision=gpu.BTE_FP32_MIXED)
        s.autotune(cache, batch=True)
        sols.append(s)
    layouts = [s.sweep_layout() for s in sols]
    announce("c5 full draw: 2 batched steps")
    with gpu.Batch(sols, use_graph=True) as batch:
        st = batch.step(2)
    dofs = [i.n_dof for i in insts]
    pick = [max((k for k in range(64) if insts[k].dim == 2), key=dofs.__getitem__),
            max((k for k in range(64) if insts[k].dim == 3), key=dofs.__getitem__),
            min(range(64), key=dofs.__getitem__)]
    T_batch = {k: sols[k].temperature() for k in pick}
    for s in sols:
        s.close()
    del sols
    torch.cuda.empty_cache()
    for k in pick:
        lay = layouts[k]
        for name, v in (("BTE_SWEEP_KIND", lay["kind"]), ("BTE_SWEEP_RY", lay["ry"]),
                        ("BTE_SWEEP_RZ", lay["rz"]), ("BTE_SWEEP_NDG", lay["ndg"])):
            monkeypatch.setenv(name, str(v))
        announce(f"c5 geometry {k} ({insts[k].name}, {dofs[k]:.3e} DOF, layout {lay}) solo")
        with gpu.Solver(insts[k], stream=stream, precision=gpu.BTE_FP32_MIXED) as s:
            assert s.sweep_layout() == lay
            solo = s.step(2)
            T = s.temperature()
        assert [x["inner"] for x in solo] == [st[j][k]["inner"] for j in range(2)]
        assert np.array_equal(T, T_batch[k]), float(np.max(np.abs(T - T_batch[k])))
