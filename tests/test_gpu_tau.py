"""Temperature-dependent relaxation times on the GPU, against the oracle:
tau_b(T) = tau_b (300 K / T)^p_b with band-dependent exponents, so every
relaxation term takes tau at its cell's current temperature, the implicit
diagonal varies from cell to cell, and the relaxation-time-weighted
temperature solves sum_b (W I0_b(T) - e_b) / tau_b(T) = 0.

Every kernel family and layout (2D and 3D column walks, the flattened plane,
one cell per thread), implicit and explicit, FP64 within 1e-10 with the
oracle's sweep schedule replayed and FP32 storage within 1e-5 in T (both
schemes); the
uniform state stays bitwise unchanged; a specular box conserves energy to
round-off in explicit mode (only if the inversion and the relaxation term use
the same tau_b(T)); a checkpoint resumes bit for bit.
"""
import sys

import numpy as np
import pytest

from paper_2305_19400_amd import inputs as I
from tests.test_gpu_layouts import CASES, KIND_FLAT, set_layout

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


def with_law(inst, seed=7, lo=0.5, hi=2.5):
    out = inst.copy()
    out.tau_exp = np.random.default_rng(seed).uniform(lo, hi, inst.n_bands)
    out.tau_T0 = 300.0
    return out


def rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))


LAYOUTS = [("2d", 4, 0, 1), ("2d", 8, 0, 3), ("2dn", 4, 0, 2), ("3d", 2, 2, 1), ("3d", 1, 4, 2),
           ("3d", 2, 4, 3), ("3d", 0, 4, 1), ("3d", 0, 2, 2), ("3dn", 0, 4, 2), ("3dn", 1, 4, 1),
           ("2d", None, None, None), ("3dn", None, None, None)]


@pytest.mark.parametrize("dim,ry,rz,ndg", LAYOUTS)
@pytest.mark.parametrize("scheme", [I.SCHEME_IMPLICIT_JACOBI, I.SCHEME_EXPLICIT_EULER])
def test_tau_law_matches_oracle(gpu, monkeypatch, dim, ry, rz, ndg, scheme):
    """ry None: one cell per thread."""
    from oracle import Oracle
    inst = with_law(CASES[dim]())
    dt = 2e-13 if scheme == I.SCHEME_EXPLICIT_EULER else inst.dt
    if ry is None:
        monkeypatch.setenv("BTE_SWEEP_KIND", "0")
    else:
        set_layout(monkeypatch, ry, rz, ndg)
    ref = Oracle(inst, scheme=scheme, dt=dt)
    sched = [s["inner"] for s in ref.run(3)]
    const = Oracle(CASES[dim](), scheme=scheme, dt=dt)
    const.run(3, schedule=sched)
    announce(f"tau(T) {inst.name} layout {(ry, rz, ndg)} scheme {scheme} sched {sched}")
    with gpu.Solver(inst, scheme=scheme, dt=dt) as sol:
        if ry is None:
            assert sol.sweep_layout()["kind"] == 0
        else:
            kind = 1 if dim.startswith("2d") else (KIND_FLAT if ry == 0 else 2)
            assert sol.sweep_layout()["kind"] == kind
        sol.step(3, fixed_inner=sched)
        T, Iq = sol.temperature(), sol.intensity()
    errT = rel(T, ref.temperature())
    errI = rel(Iq, np.ascontiguousarray(ref.intensity().transpose(2, 1, 0)))
    print(f"T {errT:.2e} I {errI:.2e}; law moves T by {rel(ref.temperature(), const.temperature()):.2e}",
          flush=True)
    assert errT <= 1e-10 and errI <= 1e-10
    assert rel(ref.temperature(), const.temperature()) > 1e-7  # the law matters here


@pytest.mark.parametrize("dim", ["2d", "3d", "3dn"])
@pytest.mark.parametrize("scheme", [I.SCHEME_IMPLICIT_JACOBI, I.SCHEME_EXPLICIT_EULER])
def test_tau_law_fp32_matches_oracle(gpu, dim, scheme):
    from oracle import Oracle
    inst = with_law(CASES[dim]())
    dt = 2e-13 if scheme == I.SCHEME_EXPLICIT_EULER else inst.dt
    ref = Oracle(inst, scheme=scheme, dt=dt)
    ref.run(3)
    announce(f"tau(T) fp32 {inst.name} scheme {scheme}")
    with gpu.Solver(inst, precision=gpu.BTE_FP32_MIXED, scheme=scheme, dt=dt) as sol:
        st = sol.step(3)
        T = sol.temperature()
    err = rel(T, ref.temperature())
    print(f"fp32 T {err:.2e}, sweeps {[s['inner'] for s in st]}", flush=True)
    assert err <= 1e-5


@pytest.mark.parametrize("scheme", [I.SCHEME_IMPLICIT_JACOBI, I.SCHEME_EXPLICIT_EULER])
def test_tau_law_uniform_state_bitwise(gpu, scheme):
    inst = with_law(CASES["3dn"]())
    inst.T_init[:] = 310.0
    for f in range(6):
        if inst.wall_T[f] is not None:
            inst.wall_T[f][:] = 310.0
    announce(f"tau(T) uniform state, scheme {scheme}")
    with gpu.Solver(inst, scheme=scheme, dt=2e-13) as sol:
        I0, T0 = sol.intensity(), sol.temperature()
        sol.step(3)
        assert np.array_equal(sol.intensity(), I0) and np.array_equal(sol.temperature(), T0)


def test_tau_law_specular_box_conserves_energy(gpu):
    """All walls specular, forward Euler: sum_P E_P is conserved to round-off;
    with the plain energy sum as the temperature (which does not weight bands
    by tau_b(T)) it is not."""
    inst = with_law(I.gaussian_3d(12, 10, 9, 2, 8, 4, seed=9, sigma_cells=2.0,
                                  precision=I.PRECISION_FP64, nsteps=10))
    inst.wall = [I.WALL_SPECULAR] * 6
    inst.wall_T = [None] * 6
    announce("tau(T) specular box")
    drift = {}
    for tdef in (I.TDEF_TAU_WEIGHTED, I.TDEF_ENERGY):
        with gpu.Solver(inst, scheme=I.SCHEME_EXPLICIT_EULER, dt=2e-13, t_definition=tdef) as sol:
            E0 = sol.energy().sum()
            Es = []
            for _ in range(10):
                sol.step(1)
                Es.append(sol.energy().sum())
        drift[tdef] = max(abs(e - E0) / E0 for e in Es)
    print(f"energy drift: tau-weighted {drift[I.TDEF_TAU_WEIGHTED]:.2e}, "
          f"plain energy {drift[I.TDEF_ENERGY]:.2e}", flush=True)
    assert drift[I.TDEF_TAU_WEIGHTED] < 1e-13
    assert drift[I.TDEF_ENERGY] > 1e-10


@pytest.mark.parametrize("precision", [I.PRECISION_FP64, I.PRECISION_FP32_MIXED])
def test_tau_law_checkpoint_and_warm_start(gpu, precision):
    """With tau_b(T) and the learned warm start (which refreshes the rates at its
    guessed temperature): 7 steps equal 4 + checkpoint + 3 bit for bit; and a
    batch refuses the context."""
    import torch
    inst = with_law(I.gaussian_3d(13, 11, 9, 2, 4, 5, seed=29, sigma_cells=2.5,
                                  precision=precision, nsteps=7))
    opts = dict(precision=precision, warm_start=gpu.BTE_WARM_T, nn_train_steps=2, nn_epochs=2)
    announce(f"tau(T) checkpoint, precision {precision}")
    stream = torch.cuda.Stream()
    with gpu.Solver(inst, stream=stream, **opts) as a:
        a.step(4)
        state = a.get_state()
        sa = a.step(3)
        assert all(s["warm"] for s in sa)
        Ta, Ia = a.temperature(), a.intensity()
        with pytest.raises(gpu.BteError) as e:
            gpu.Batch([a])
        assert e.value.code == gpu.BTE_E_INVAL and "temperature law" in str(e.value)
    with gpu.Solver(inst, stream=stream, **opts) as b:
        b.set_state(state)
        assert b.step(3) == sa
        assert np.array_equal(b.temperature(), Ta) and np.array_equal(b.intensity(), Ia)
