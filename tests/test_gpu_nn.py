"""The learned warm start on the GPU: bf16 MFMA forward and backward against
the FP64 reference on identical (bf16-rounded) operands, on-device training,
the iterations it saves, and the fallback when the network is unusable.

Tolerances.  The GPU accumulates products in FP32 and rounds the first hidden
activation and the back-propagated pre-activation gradients to bf16, as the
reference emulates; they differ only where the FP32 and FP64 sums fall on
opposite sides of a bf16 rounding boundary (probability ~1e-6 / 2^-8 per
element), which moves a few outputs by ~2^-8 of one hidden unit's share.
Hence: the median output error is at FP32 round-off level, 99 % of outputs
are within 1e-4 of the output scale, all within 1e-2; gradients agree to
1e-3 in relative norm.  (Measured on MI355X: median ~4e-8, max ~1e-6,
gradients ~3e-6.)
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


def nn_instance(dim):
    if dim == 3:
        return I.gaussian_3d(12, 10, 9, 2, 8, 6, seed=7, sigma_cells=2.5,
                             precision=I.PRECISION_FP64, nsteps=4)
    return I.strip_2d(40, 30, 2, 8, 6, seed=7, nsteps=4)


def synthetic_sample(inst, seed):
    """Seeded (T_n, T_{n-1}, E_n, T_{n+1}) fields of a hot spot relaxing."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = inst.n
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    r2 = (x - nx / 2) ** 2 + (y - ny / 3) ** 2 + (z - nz / 2) ** 2
    Tn = (300 + 20 * np.exp(-r2 / 8.0) + rng.normal(0, 0.05, r2.shape)).reshape(-1)
    Tp = Tn + 0.3 * np.exp(-r2 / 8.0).reshape(-1) + rng.normal(0, 0.01, Tn.shape)
    E = 1.0e5 * (Tn / 300.0) ** 1.7 + rng.normal(0, 10.0, Tn.shape)
    Tx = Tn - 0.25 * np.exp(-r2 / 9.0).reshape(-1) + rng.normal(0, 0.01, Tn.shape)
    return Tn, Tp, E, Tx


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


@pytest.mark.parametrize("dim,n", [(2, None), (3, None), (2, (1, 9)), (3, (1, 6, 5)),
                                   (3, (7, 1, 4)), (3, (1, 1, 7))])
def test_forward_backward_vs_reference(gpu, dim, n):
    """Network forward and gradients against the numpy reference, also on
    one-cell-wide axes, where both patch neighbours along the axis are walls."""
    from oracle import mlp
    if n is None:
        inst = nn_instance(dim)
    elif dim == 2:
        inst = I.strip_2d(n[0], n[1], 2, 8, 6, seed=7, strip_cells=1, nsteps=4)
    else:
        inst = I.gaussian_3d(*n, 2, 8, 6, seed=7, sigma_cells=1.0, precision=I.PRECISION_FP64,
                             nsteps=4)
    Tn, Tp, E, Tx = synthetic_sample(inst, 11 + dim)
    norm = dict(muT=Tn.mean(), sT=Tn.std(), muE=E.mean(), sE=E.std(), sD=np.sqrt(np.mean((Tx - Tn) ** 2)))
    params = mlp.random_params(dim, seed=3 + dim)
    vec = mlp.pack(params, norm)
    announce(f"nn forward/backward dim={dim} cells={inst.n_cells}")
    with gpu.Solver(inst, warm_start=gpu.BTE_WARM_T) as sol:
        assert sol.nn_param_count() == vec.size
        sol.nn_set_params(vec)
        assert np.array_equal(sol.nn_params(), vec)
        loss_g, grad_g, y_g = sol.nn_gradient(Tn, Tp, E, Tx)
    # reference on the same float32 fields and parameters, bf16 rounding emulated
    p32, n32 = mlp.unpack(vec, dim)
    X = mlp.pad_features(mlp.gather(inst.n, dim, f32(Tn), f32(Tp), f32(E), n32), dim)
    t = f32((f32(Tx) - f32(Tn)) / n32["sD"])
    loss_r, grad_r = mlp.loss_and_grad(p32, X, t, emulate_bf16=True)
    y_r, _ = mlp.forward(p32, X, emulate_bf16=True)
    scale = np.sqrt(np.mean(y_r ** 2))
    err = np.abs(y_g - y_r) / scale
    print(f"y: median {np.median(err):.1e} p99 {np.quantile(err, 0.99):.1e} max {err.max():.1e}; "
          f"loss gpu {loss_g:.6e} ref {loss_r:.6e}", flush=True)
    assert np.median(err) <= 1e-6
    assert np.quantile(err, 0.99) <= 1e-4
    assert err.max() <= 1e-2
    assert abs(loss_g - loss_r) <= 1e-4 * loss_r
    gr, _ = mlp.unpack(grad_g, dim)
    for k in ("W1", "b1", "W2", "b2", "w3", "b3"):
        a, b = gr[k], grad_r[k]
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        print(f"grad {k}: rel {rel:.2e}", flush=True)
        assert rel <= 1e-3, k
    # padded feature columns get no gradient
    assert np.all(gr["W1"][:, mlp.n_features(dim):] == 0)


def test_training_lowers_loss_and_saves_iterations(gpu):
    inst = I.gaussian_3d(16, 16, 16, 4, 8, 8, seed=4, sigma_cells=3.0,
                         precision=I.PRECISION_FP64, nsteps=40)
    n_train, n_after = 20, 12
    announce("nn training on 20 solver steps, then warm-started steps")
    with gpu.Solver(inst, warm_start=gpu.BTE_WARM_T_SHIFT, nn_train_steps=n_train,
                    nn_seed=1) as sol:
        st = sol.step(n_train + n_after)
        T_warm = sol.temperature()
    with gpu.Solver(inst) as ref:
        st_ref = ref.step(n_train + n_after)
        T_ref = ref.temperature()
    assert st[n_train - 1]["trained"] == 1
    assert st[n_train - 1]["nn_loss"] < 0.1  # a zero predictor scores ~1
    warm = st[n_train:]
    assert all(s["warm"] == 1 for s in warm)
    k_warm = sum(s["inner"] for s in warm)
    k_plain = sum(s["inner"] for s in st_ref[n_train:])
    print(f"inner sweeps after training: warm {k_warm} vs plain {k_plain}; "
          f"loss {st[n_train - 1]['nn_loss']:.3e}; fallbacks {[s['fallbacks'] for s in warm]}",
          flush=True)
    assert k_warm < k_plain
    # both stop at the same step-relative residual tolerance (1e-4), so they
    # agree to a small fraction of the temperature rise
    rise = T_ref.max() - 300.0
    print(f"warm vs plain: max |dT| {np.max(np.abs(T_warm - T_ref)):.2e} K of a {rise:.1f} K rise",
          flush=True)
    assert np.max(np.abs(T_warm - T_ref)) <= 1e-3 * rise
    assert all(s["converged"] for s in st)


def test_unusable_network_falls_back_to_plain(gpu):
    from oracle import mlp
    inst = nn_instance(2)
    announce("nan network: every cell falls back")
    params = mlp.random_params(2, seed=1)
    params["w3"][:] = np.nan
    vec = mlp.pack(params, dict(muT=300.0, sT=1.0, muE=1.0, sE=1.0, sD=0.01))
    with gpu.Solver(inst, warm_start=gpu.BTE_WARM_T) as sol:
        sol.nn_set_params(vec)
        st = sol.step(3)
        T1, I1 = sol.temperature(), sol.intensity()
    with gpu.Solver(inst) as ref:
        st0 = ref.step(3)
        T0, I0 = ref.temperature(), ref.intensity()
    assert all(s["warm"] == 1 and s["fallbacks"] == inst.n_cells for s in st)
    assert [s["inner"] for s in st] == [s["inner"] for s in st0]
    assert np.array_equal(T1, T0) and np.array_equal(I1, I0)


def test_training_is_deterministic(gpu):
    inst = nn_instance(2)
    announce("nn training determinism")
    out = []
    for _ in range(2):
        with gpu.Solver(inst, warm_start=gpu.BTE_WARM_T, nn_train_steps=3, nn_seed=5) as sol:
            sol.step(4)
            out.append((sol.nn_params(), sol.temperature()))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_guard_switches_off_a_guess_that_costs_sweeps(gpu):
    """A plausible but wrong network (every guess 5 s_D off) costs sweeps; after
    nn_guard warm steps the plain iteration's verdict switches the guess off."""
    from oracle import mlp
    inst = I.gaussian_3d(16, 16, 16, 4, 8, 8, seed=4, sigma_cells=3.0,
                         precision=I.PRECISION_FP64, nsteps=16)
    announce("guard against a harmful guess")
    with gpu.Solver(inst, warm_start=gpu.BTE_WARM_T_SHIFT, nn_train_steps=4, nn_seed=1,
                    nn_guard=4) as sol:
        st = sol.step(4)  # plain steps, recorded; trained after the 4th
        assert st[3]["trained"] == 1
        p = mlp.random_params(3, seed=1)
        p["w3"][:] = 0.0
        p["b3"][:] = 5.0  # y = 5: guess T_n + 5 s_D everywhere
        vec = sol.nn_params().copy()
        _, norm = mlp.unpack(vec, 3)
        sol.nn_set_params(mlp.pack(p, norm))
        st2 = sol.step(8)
    plain = sum(s["inner"] for s in st[:4])
    warm = sum(s["inner"] for s in st2[:4])
    print(f"plain {plain} warm {warm}; warm flags {[s['warm'] for s in st2]}", flush=True)
    assert all(s["warm"] == 1 for s in st2[:4])
    assert warm > plain
    assert all(s["warm"] == 0 for s in st2[4:])
    assert all(s["converged"] for s in st2)
