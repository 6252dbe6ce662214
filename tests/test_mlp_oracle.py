"""Pins of the FP64 reference of the learned warm start (oracle/mlp.py):
bf16 rounding against torch's bfloat16 conversion, hand-written
backpropagation against central finite differences, and the patch gather
against explicit loops."""
import numpy as np
import pytest
import torch

from oracle import mlp


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e6, 1000),
                        np.array([0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9,
                                  -1.5, 65504.0, 1e-30, 3.0e38])])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)


def test_gather_replicate_padding():
    n = (4, 3, 2)
    rng = np.random.default_rng(1)
    Tn, Tp, E = (rng.normal(size=24) for _ in range(3))
    norm = dict(muT=0.5, sT=2.0, muE=-1.0, sE=4.0)
    X = mlp.gather(n, 3, Tn, Tp, E, norm)
    assert X.shape == (24, 81)
    nx, ny, nz = n
    for P in range(24):
        x, y, z = P % nx, (P // nx) % ny, P // (nx * ny)
        k = 0
        for ch, f, mu, s in ((0, Tn, 0.5, 2.0), (1, Tp, 0.5, 2.0), (2, E, -1.0, 4.0)):
            for dz in (-1, 0, 1):
                for dy in (-1, 0, 1):
                    for dx in (-1, 0, 1):
                        qx = min(max(x + dx, 0), nx - 1)
                        qy = min(max(y + dy, 0), ny - 1)
                        qz = min(max(z + dz, 0), nz - 1)
                        Q = qx + nx * (qy + ny * qz)
                        assert X[P, k] == (f[Q] - mu) / s
                        k += 1
    X2 = mlp.gather((5, 4, 1), 2, rng.normal(size=20), rng.normal(size=20), rng.normal(size=20),
                    norm)
    assert X2.shape == (20, 27)


@pytest.mark.parametrize("dim", [2, 3])
def test_backprop_matches_finite_differences(dim):
    rng = np.random.default_rng(2 + dim)
    params = mlp.random_params(dim, seed=5)
    M = 37
    X = mlp.pad_features(rng.normal(size=(M, mlp.n_features(dim))), dim)
    t = rng.normal(size=M)
    loss, g = mlp.loss_and_grad(params, X, t)
    for key, arr in params.items():
        idx = [np.unravel_index(i, arr.shape) for i in rng.choice(arr.size, min(arr.size, 12), replace=False)]
        if key == "W1":  # padded feature columns have no effect
            idx = [i for i in idx if i[1] < mlp.n_features(dim)] or [(0, 0)]
        for i in idx:
            h = 1e-6 * max(1.0, abs(arr[i]))
            old = arr[i]
            arr[i] = old + h
            lp, _ = mlp.loss_and_grad(params, X, t)
            arr[i] = old - h
            lm, _ = mlp.loss_and_grad(params, X, t)
            arr[i] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[key][i]) <= 1e-6 * max(abs(fd), 1e-3), (key, i, fd, g[key][i])


def test_pack_unpack_round_trip():
    params = mlp.random_params(3, seed=9)
    norm = dict(muT=301.0, sT=2.5, muE=1.0e6, sE=3.0e4, sD=0.01)
    v = mlp.pack(params, norm)
    p2, n2 = mlp.unpack(v, 3)
    for k in params:
        assert np.allclose(p2[k], params[k].astype(np.float32))
    assert n2["sD"] == np.float32(0.01)


# ---------------------------------------------------------------- training rules
def test_adam_first_step_closed_form():
    """At t = 1 both bias corrections undo the moment decay exactly, so the
    update is -lr g / (|g| + eps): a step of lr against the sign of g."""
    rng = np.random.default_rng(11)
    g = np.concatenate([rng.normal(0, 1, 200), rng.normal(0, 1e-6, 20)])
    p0 = rng.normal(0, 1, g.size)
    lr = 3e-3
    p, m, v = mlp.adam_step(p0, g, np.zeros_like(g), np.zeros_like(g), 1, lr)
    assert np.allclose(p - p0, -lr * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)
    assert np.allclose(m, 0.1 * g, rtol=1e-15) and np.allclose(v, 0.001 * g * g, rtol=1e-15)


def test_adam_constant_gradient():
    """A constant gradient c keeps both bias-corrected moments at c and c^2,
    so every step is -lr c / (|c| + eps)."""
    p, m, v = np.array([0.5]), np.zeros(1), np.zeros(1)
    for t in range(1, 8):
        p, m, v = mlp.adam_step(p, np.array([-2.0]), m, v, t, 0.01)
    assert abs(p[0] - (0.5 + 7 * 0.01 * 2.0 / (2.0 + 1e-8))) <= 1e-15


def test_adam_hand_sequence():
    """Gradients 1, 2, -1 at lr 0.01: moments and steps computed by hand from
    m_t = 0.9 m + 0.1 g, v_t = 0.999 v + 0.001 g^2, step = -lr (m_t/(1-0.9^t)) /
    (sqrt(v_t/(1-0.999^t)) + 1e-8) (30-digit decimal arithmetic)."""
    hand = [(0.1, 0.001, -0.00999999990000000099999999),
            (0.29, 0.004999, -0.00965182019718343498145186),
            (0.161, 0.005994001, -0.00420089300599795335101968)]
    p, m, v = np.zeros(1), np.zeros(1), np.zeros(1)
    for t, (g, (mh, vh, dh)) in enumerate(zip((1.0, 2.0, -1.0), hand), start=1):
        p_old = p.copy()
        p, m, v = mlp.adam_step(p, np.array([g]), m, v, t, 0.01)
        assert abs(m[0] - mh) <= 1e-15 and abs(v[0] - vh) <= 1e-17
        assert abs((p - p_old)[0] - dh) <= 1e-16


def test_adam_leaves_frozen_entries():
    mask = mlp.trainable_mask(2)
    n = mask.size
    assert n == 128 * 32 + 128 + 128 * 128 + 128 + 128 + 4 + 8
    k = mlp.n_features(2)
    W1 = mask[:128 * 32].reshape(128, 32)
    assert W1[:, :k].all() and not W1[:, k:].any()
    assert not mask[-12 + 1:-8].any() and not mask[-8:].any() and mask[-12]
    g = np.ones(n)
    p, m, v = mlp.adam_step(np.zeros(n), g, np.zeros(n), np.zeros(n), 1, 0.1, mask)
    assert np.all(p[~mask] == 0) and np.all(m[~mask] == 0) and np.all(p[mask] < 0)


def test_normalisation_closed_forms():
    nc = 6
    hist = np.zeros((2, 4, nc), dtype=np.float32)
    hist[0, 0, :3], hist[0, 0, 3:] = 299.0, 301.0     # T_n: mean 300, population std 1
    hist[1, 0, :] = [299.0, 301.0] * 3
    hist[:, 2, :] = 5.0e5 + np.array([-0.0625, 0.0625] * 3)  # std 1/16 < 1e-6 |mean|: floor
    hist[:, 3, :] = hist[:, 0, :] + 0.5                # every step moves T by 0.5
    nm = mlp.normalisation(hist)
    assert nm["muT"] == 300.0 and nm["sT"] == 1.0 and nm["sD"] == 0.5
    assert nm["muE"] == 5.0e5
    assert nm["sE"] == float(np.float32(np.float32(1e-6) * np.float32(5.0e5) + np.float32(1e-30)))
    hist[:, 0, :] = 300.0  # no spread and no change: scales of 1
    hist[:, 2, :] = 5.0e5
    hist[:, 3, :] = 300.0
    nm = mlp.normalisation(hist)
    assert nm["sD"] == 1.0 and nm["sT"] == 1.0 and nm["sE"] == 1.0


@pytest.mark.parametrize("N", [1, 7, 64, 8192, 8193, 24576, 100003])
def test_schedule_visits_every_sample_once_per_epoch(N):
    from math import gcd
    a, ups = mlp.schedule(N, epochs=3)
    assert gcd(a, N) == 1 and a % 2 == 1
    per = (N + mlp.BATCH - 1) // mlp.BATCH
    assert len(ups) == 3 * per
    for e in range(3):
        seen = np.concatenate([(a * np.arange(b0, b0 + sz, dtype=np.int64) + c) % N
                               for b0, c, sz in ups[e * per:(e + 1) * per]])
        assert np.array_equal(np.sort(seen), np.arange(N))
        assert all(c == (e * 7919) % N for _, c, _ in ups[e * per:(e + 1) * per])
    # default: at least two passes and at least 300 updates
    assert len(mlp.schedule(N)[1]) == per * max(2, -(-300 // per))


def test_accept_guess_rules():
    Tn = np.array([300.0, 300.0, 300.0, 300.0, 300.0, 2.0])
    Tp = np.array([299.0, 300.0, 300.0, 300.0, 300.0, 2.0])
    y = np.array([1.0, 5.0, 10.5, np.nan, -9.9, -10.0])
    T0, bad = mlp.accept_guess(Tn, Tp, y, 0.5)
    # limits: 10 max(0.5, |Tn - Tp|) = 10, 5, 5, 5, 5, 5
    assert list(bad) == [False, False, True, True, False, True]
    assert T0[0] == 300.5 and T0[1] == 302.5 and T0[2] == 300.0 and T0[3] == 300.0
    assert T0[4] == 300.0 - 4.95 and T0[5] == 2.0  # a guess of -3 K is not positive


def test_training_reduces_loss_on_a_smooth_target():
    """Sanity of the replayed training on a small synthetic history: the
    minibatch loss falls over the updates."""
    rng = np.random.default_rng(4)
    n, dim, nrec = (12, 10, 1), 2, 3
    nc = 120
    hist = np.zeros((nrec, 4, nc), dtype=np.float32)
    x = np.arange(nc) % 12
    for s in range(nrec):
        hist[s, 0] = 300 + np.sin(x / 3.0 + s)
        hist[s, 1] = 300 + np.sin(x / 3.0 + s - 1)
        hist[s, 2] = 1e5 * (1 + 0.01 * np.cos(x / 3.0 + s))
        hist[s, 3] = hist[s, 0] + 0.1 * (hist[s, 0] - hist[s, 1])
    vec0 = mlp.pack(mlp.random_params(dim, seed=1), dict(muT=0, sT=1, muE=0, sE=1, sD=1))
    P, m, v, t, losses = mlp.train(vec0, hist, n, dim, epochs=60, lr=3e-3)
    assert t == 60 and losses[-1] < 0.2 * losses[0]
