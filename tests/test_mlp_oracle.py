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
