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


# ---------------------------------------------------------------- training and use
# The steps below follow the warm-start rules the library documents (they are
# not in the paper): recorded samples, normalisation, the minibatch order, Adam
# and the plausibility test of a guess.  FP64 arithmetic; with emulate=True
# the FP32 storage points of the library (recorded fields, normalisation
# constants, master parameters and Adam moments) are rounded to float32.

ADAM_BETA1 = 0.9
ADAM_BETA2 = 0.999
ADAM_EPS = 1e-8
BATCH = 8192  # minibatch size


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def normalisation(hist):
    """Normalisation constants of a recorded history hist[step][4][N_c]
    (channels T_n, T_{n-1}, E_n, T_{n+1}): mean and population standard
    deviation of the T_n channel and of the E_n channel over every recorded
    sample, and the root mean square of T_{n+1} - T_n.  A non-positive
    variance gives a scale of 1; a T or E scale at or below 1e-6 |mean| is
    raised to 1e-6 |mean| + 1e-30; a zero RMS change gives 1."""
    h = np.asarray(hist, dtype=np.float64)
    t, e = h[:, 0, :].ravel(), h[:, 2, :].ravel()
    d = (h[:, 3, :] - h[:, 0, :]).ravel()
    muT, muE = t.mean(), e.mean()
    vT, vE = np.mean((t - muT) ** 2), np.mean((e - muE) ** 2)
    sD = np.sqrt(np.mean(d * d))
    sT = np.sqrt(vT) if vT > 0 else 1.0
    sE = np.sqrt(vE) if vE > 0 else 1.0
    sT, sE, muT32, muE32 = float(np.float32(sT)), float(np.float32(sE)), float(np.float32(muT)), float(np.float32(muE))
    if not sT > 1e-6 * abs(muT32):
        sT = float(np.float32(np.float32(1e-6) * np.float32(abs(muT32)) + np.float32(1e-30)))
    if not sE > 1e-6 * abs(muE32):
        sE = float(np.float32(np.float32(1e-6) * np.float32(abs(muE32)) + np.float32(1e-30)))
    return dict(muT=muT32, sT=sT, muE=muE32, sE=sE, sD=float(np.float32(sD if sD > 0 else 1.0)))


def schedule(nsamples, epochs=0):
    """Minibatch order of one training: sample position i of an epoch maps to
    recorded sample (a i + c_e) mod N, a = floor(0.6180339887 N) | 1 raised by 2
    until gcd(a, N) = 1, c_e = 7919 e mod N; each epoch is cut into minibatches
    of BATCH consecutive positions; epochs <= 0 means max(2, ceil(300 /
    minibatches per epoch)).  Returns (a, [(first position, c_e, size), ...])."""
    from math import gcd
    N = int(nsamples)
    a = int(0.6180339887 * float(N)) | 1
    while gcd(a, N) != 1:
        a += 2
    per_epoch = (N + BATCH - 1) // BATCH
    if epochs <= 0:
        epochs = max(2, (300 + per_epoch - 1) // per_epoch)
    ups = []
    for e in range(epochs):
        c = (e * 7919) % N
        for b0 in range(0, N, BATCH):
            ups.append((b0, c, min(BATCH, N - b0)))
    return a, ups


def adam_step(p, g, m, v, t, lr, trainable=None):
    """One Adam update (Kingma and Ba 2015, Algorithm 1) with beta1 0.9, beta2
    0.999, eps 1e-8 and bias correction at step t >= 1; entries outside
    `trainable` keep their parameter and moments."""
    m_new = ADAM_BETA1 * m + (1.0 - ADAM_BETA1) * g
    v_new = ADAM_BETA2 * v + (1.0 - ADAM_BETA2) * g * g
    mhat = m_new / (1.0 - ADAM_BETA1 ** t)
    vhat = v_new / (1.0 - ADAM_BETA2 ** t)
    p_new = p - lr * mhat / (np.sqrt(vhat) + ADAM_EPS)
    if trainable is not None:
        p_new = np.where(trainable, p_new, p)
        m_new = np.where(trainable, m_new, m)
        v_new = np.where(trainable, v_new, v)
    return p_new, m_new, v_new


def trainable_mask(dim):
    """Entries of the flat parameter vector that training updates: every weight
    and bias except the zero-padded feature columns of W1, the padding after b3
    and the normalisation constants."""
    k, kp = n_features(dim), padded_features(dim)
    W1 = np.zeros((HIDDEN, kp), dtype=bool)
    W1[:, :k] = True
    parts = [W1.ravel(), np.ones(HIDDEN, bool), np.ones(HIDDEN * HIDDEN, bool),
             np.ones(HIDDEN, bool), np.ones(HIDDEN, bool), np.array([True, False, False, False]),
             np.zeros(8, bool)]
    return np.concatenate(parts)


def _flat_to_params(vec, dim):
    params, _ = unpack(vec, dim)
    return params


def _grad_to_flat(g, dim):
    return np.concatenate([g["W1"].ravel(), g["b1"], g["W2"].ravel(), g["b2"], g["w3"],
                           np.array([g["b3"][0], 0.0, 0.0, 0.0]), np.zeros(8)])


def minibatch(hist, n, dim, norm, a, b0, c, size):
    """Features and targets of one minibatch: positions b0 .. b0+size-1 of the
    permuted order, sample i = (a pos + c) mod N = step i // N_c, cell i % N_c."""
    h = np.asarray(hist, dtype=np.float64)
    nrec, _, nc = h.shape
    N = nrec * nc
    pos = np.arange(b0, b0 + size, dtype=np.int64)
    idx = (a * pos + c) % N
    steps, cells = idx // nc, idx % nc
    X = np.empty((size, n_features(dim)))
    for st in np.unique(steps):
        sel = steps == st
        Xs = gather(n, dim, h[st, 0], h[st, 1], h[st, 2], norm)
        X[sel] = Xs[cells[sel]]
    t = (h[steps, 3, cells] - h[steps, 0, cells]) / norm["sD"]
    return X, t


def train(vec0, hist, n, dim, epochs=0, lr=1e-3, emulate=True, t0=0, m0=None, v0=None):
    """Replays one training of the warm-start network from the flat parameter
    vector vec0 on the recorded history hist[step][4][N_c]: normalisation, then
    one Adam update per minibatch of the schedule on the mean squared error.
    Returns (parameter vector, m, v, Adam step count, per-update losses)."""
    r32 = f32 if emulate else (lambda x: np.asarray(x, dtype=np.float64))
    norm = normalisation(hist)
    P = np.asarray(vec0, dtype=np.float64).copy()
    ko = padded_features(dim) * HIDDEN + HIDDEN * HIDDEN + 3 * HIDDEN + 4  # norm offset
    P[ko:ko + 5] = [norm["muT"], norm["sT"], norm["muE"], norm["sE"], norm["sD"]]
    P[ko + 5:] = 0.0
    m = np.zeros_like(P) if m0 is None else np.asarray(m0, dtype=np.float64).copy()
    v = np.zeros_like(P) if v0 is None else np.asarray(v0, dtype=np.float64).copy()
    mask = trainable_mask(dim)
    h = np.asarray(hist, dtype=np.float64)
    a, ups = schedule(h.shape[0] * h.shape[2], epochs)
    t = t0
    losses = []
    for b0, c, size in ups:
        X, tgt = minibatch(h, n, dim, norm, a, b0, c, size)
        if emulate:
            X, tgt = f32(X), f32(tgt)
        params = _flat_to_params(P, dim)
        loss, g = loss_and_grad(params, pad_features(X, dim), tgt, emulate_bf16=emulate)
        gf = _grad_to_flat(g, dim)
        t += 1
        P, m, v = adam_step(P, gf, m, v, t, lr, mask)
        P, m, v = r32(P), r32(m), r32(v)
        losses.append(loss)
    return P, m, v, t, losses


def accept_guess(Tn, Tprev, y, sD, max_step=10.0):
    """Plausibility test of a warm-start guess T_n + s_D y per cell: kept if the
    change is finite, at most max_step * max(s_D, |T_n - T_{n-1}|) in size and
    the guess is positive; otherwise the cell starts from T_n.  Returns the
    starting temperature and the mask of rejected cells."""
    Tn = np.asarray(Tn, dtype=np.float64)
    dT = float(sD) * np.asarray(y, dtype=np.float64)
    lim = max_step * np.maximum(float(sD), np.abs(Tn - np.asarray(Tprev, dtype=np.float64)))
    with np.errstate(invalid="ignore"):
        T0 = Tn + dT
        bad = ~np.isfinite(dT) | (np.abs(dT) > lim) | ~(T0 > 0.0)
    return np.where(bad, Tn, T0), bad
