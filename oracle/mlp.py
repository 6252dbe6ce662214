"""FP64 reference for the learned warm start -- TEST INFRASTRUCTURE ONLY.

Plain numpy: patch gather, the 3-layer MLP, the mean-squared-error loss and
its gradient by hand-written backpropagation, with optional emulation of the
BF16 rounding points of the GPU kernels (inputs, weights of the two hidden
layers, first hidden activation, and the backpropagated pre-activation
gradients are rounded to bfloat16 where the GPU feeds them to its matrix
cores).  Used only by the tests; shares nothing with the GPU library.

Model (per cell P, step n -> n+1):
  x = features of the 3^dim neighbourhood of P (replicate padding at mesh
      edges) of three channels, in the order [channel][dz][dy][dx]:
      (T_n - mu_T)/s_T, (T_{n-1} - mu_T)/s_T, (E_n - mu_E)/s_E
  h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3
  guess T_{n+1} = T_n + s_D * y
  loss = mean over samples of (y - (T_{n+1} - T_n)/s_D)^2
"""
from __future__ import annotations

import numpy as np

HIDDEN = 128


def bf16(a):
    """Round float values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64).reshape(np.shape(a))


def n_features(dim):
    return 3 * 3 ** dim


def padded_features(dim):
    k = n_features(dim)
    return (k + 31) // 32 * 32


def stencil(dim):
    if dim == 2:
        return [(0, dy, dx) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def gather(n, dim, Tn, Tp, E, norm):
    """Feature matrix [N_c, 3 * 3^dim] (unpadded), float64."""
    nx, ny, nz = n
    muT, sT, muE, sE = norm["muT"], norm["sT"], norm["muE"], norm["sE"]
    P = np.arange(nx * ny * nz)
    x, y, z = P % nx, (P // nx) % ny, P // (nx * ny)
    cols = []
    for ch, field in enumerate((Tn, Tp, E)):
        mu, s = (muT, sT) if ch < 2 else (muE, sE)
        for dz, dy, dx in stencil(dim):
            Q = (np.clip(x + dx, 0, nx - 1) + nx * (np.clip(y + dy, 0, ny - 1) +
                                                    ny * np.clip(z + dz, 0, nz - 1)))
            cols.append((field[Q] - mu) / s)
    return np.stack(cols, axis=1)


def forward(params, X, emulate_bf16=False):
    """Returns y and the intermediates (z1, h1, z2, h2)."""
    W1, b1, W2, b2, w3, b3 = (params[k] for k in ("W1", "b1", "W2", "b2", "w3", "b3"))
    r = bf16 if emulate_bf16 else (lambda a: a)
    Xq, W1q, W2q = r(X), r(W1), r(W2)
    z1 = Xq @ W1q.T + b1
    h1 = np.maximum(z1, 0.0)
    h1q = r(h1)
    z2 = h1q @ W2q.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, dict(Xq=Xq, W1q=W1q, W2q=W2q, z1=z1, h1=h1q, z2=z2, h2=h2)


def loss_and_grad(params, X, t, emulate_bf16=False):
    """Mean squared error and its gradient with respect to every parameter."""
    r = bf16 if emulate_bf16 else (lambda a: a)
    y, c = forward(params, X, emulate_bf16)
    M = X.shape[0]
    e = y - t
    loss = float(np.mean(e * e))
    dy = 2.0 * e / M
    g = {}
    g["w3"] = c["h2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    dz2 = np.outer(dy, params["w3"]) * (c["z2"] > 0)
    g["b2"] = dz2.sum(axis=0)
    dz2q = r(dz2)
    g["W2"] = dz2q.T @ c["h1"]
    dh1 = dz2q @ c["W2q"]
    dz1 = dh1 * (c["z1"] > 0)
    g["b1"] = dz1.sum(axis=0)
    dz1q = r(dz1)
    g["W1"] = dz1q.T @ c["Xq"]
    return loss, g


def random_params(dim, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    k = n_features(dim)
    kp = padded_features(dim)
    W1 = np.zeros((HIDDEN, kp))
    W1[:, :k] = rng.uniform(-1, 1, (HIDDEN, k)) * np.sqrt(6.0 / k) * scale
    return dict(W1=W1, b1=rng.uniform(-0.1, 0.1, HIDDEN),
                W2=rng.uniform(-1, 1, (HIDDEN, HIDDEN)) * np.sqrt(6.0 / HIDDEN) * scale,
                b2=rng.uniform(-0.1, 0.1, HIDDEN),
                w3=rng.uniform(-1, 1, HIDDEN) * np.sqrt(6.0 / HIDDEN) * scale,
                b3=np.array([rng.uniform(-0.1, 0.1)]))


def pad_features(X, dim):
    out = np.zeros((X.shape[0], padded_features(dim)))
    out[:, :X.shape[1]] = X
    return out


def pack(params, norm):
    """Flat FP32 parameter vector in the library's order (see include/bte.h)."""
    parts = [params["W1"].ravel(), params["b1"], params["W2"].ravel(), params["b2"],
             params["w3"], np.array([params["b3"][0], 0.0, 0.0, 0.0]),
             np.array([norm["muT"], norm["sT"], norm["muE"], norm["sE"], norm["sD"], 0.0, 0.0, 0.0])]
    return np.concatenate(parts).astype(np.float32)


def unpack(vec, dim):
    kp = padded_features(dim)
    o = 0

    def take(n):
        nonlocal o
        a = np.asarray(vec[o:o + n], dtype=np.float64)
        o += n
        return a

    W1 = take(HIDDEN * kp).reshape(HIDDEN, kp)
    b1 = take(HIDDEN)
    W2 = take(HIDDEN * HIDDEN).reshape(HIDDEN, HIDDEN)
    b2 = take(HIDDEN)
    w3 = take(HIDDEN)
    b3 = take(4)[:1]
    nm = take(8)
    return (dict(W1=W1, b1=b1, W2=W2, b2=b2, w3=w3, b3=b3),
            dict(muT=nm[0], sT=nm[1], muE=nm[2], sE=nm[3], sD=nm[4]))
