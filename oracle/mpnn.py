"""Message-passing surrogate of the smooth vector -- TEST INFRASTRUCTURE ONLY.

Plain numpy (float64) reference of the network the GPU library runs: it
predicts log w, with w the algebraically smooth vector that drives the
matching weights (Sec. 3.1 leaves the smooth vector's source open; the
method's own relaxation, RELAX(20), provides the training targets).

Node features (8 per row i, from A alone):
    1, log(a_ii) / 4, s_i / a_ii with s_i = sum_{j!=i} |a_ij|,
    w1_i, w2_i  (two l1-Jacobi sweeps on A w = 0 from w = 1),
    log(max_{j!=i} |a_ij| / min_{j!=i} |a_ij|) / 4  (0 without off-diagonals),
    (number of off-diagonals) / 6, 0.
Aggregation: (Ahat X)_i = sum_{j!=i} |a_ij| X_j / s_i.
Layers:  h1 = ReLU([X | Ahat X] W1 + b1),  h2 = ReLU([h1 | Ahat h1] W2 + b2),
head:    y = h2 wh + bh   (prediction of log w).
Parameters, flat in this order: W1 (16 x 32, row-major), b1 (32), W2 (64 x 32),
b2 (32), wh (32), bh (1): 2657 values.

With bf16=True the inputs of every dense product (features, aggregated
features, hidden activations, W1, W2) are rounded to bfloat16 (round to
nearest even) as the GPU stores them; accumulation stays in float64 here.
"""
from __future__ import annotations

import numpy as np

F0, HID = 8, 32
SHAPES = [("W1", (2 * F0, HID)), ("b1", (HID,)), ("W2", (2 * HID, HID)), ("b2", (HID,)),
          ("wh", (HID,)), ("bh", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        m = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + m], dtype=np.float64).reshape(shp)
        o += m
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def round_bf16(x):
    """Round float values to bfloat16 (nearest, ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _rows(A):
    return np.repeat(np.arange(A.n), np.diff(A.row_ptr))


def features(A):
    rows = _rows(A)
    off = A.col != rows
    aabs = np.abs(A.val)
    d = np.zeros(A.n)
    d[rows[~off]] = A.val[~off]
    s = np.bincount(rows[off], weights=aabs[off], minlength=A.n)
    l1 = np.bincount(rows, weights=aabs, minlength=A.n)
    dinv = 1.0 / l1
    S = A.scipy()
    w1 = 1.0 - dinv * (S @ np.ones(A.n))
    w2 = w1 - dinv * (S @ w1)
    noff = np.bincount(rows[off], minlength=A.n)
    mx = np.full(A.n, 0.0)
    mn = np.full(A.n, np.inf)
    np.maximum.at(mx, rows[off], aabs[off])
    np.minimum.at(mn, rows[off], aabs[off])
    contrast = np.where(noff > 0, np.log(np.where(noff > 0, mx / np.where(noff > 0, mn, 1.0), 1.0)) / 4.0, 0.0)
    X = np.zeros((A.n, F0))
    X[:, 0] = 1.0
    X[:, 1] = np.log(d) / 4.0
    X[:, 2] = s / d
    X[:, 3] = w1
    X[:, 4] = w2
    X[:, 5] = contrast
    X[:, 6] = noff / 6.0
    return X, s


def _ahat(A, X, s):
    rows = _rows(A)
    off = A.col != rows
    out = np.zeros_like(X)
    np.add.at(out, rows[off], np.abs(A.val[off])[:, None] * X[A.col[off]])
    return out / np.where(s > 0, s, 1.0)[:, None]


def _ahat_t(A, G, s):
    rows = _rows(A)
    off = A.col != rows
    sc = np.abs(A.val[off]) / np.where(s > 0, s, 1.0)[A.col[off]]
    out = np.zeros_like(G)
    np.add.at(out, rows[off], sc[:, None] * G[A.col[off]])
    return out


def forward(theta, A, X=None, bf16=False):
    """Returns (y, cache).  y = predicted log w per row."""
    p = unpack(theta)
    r = round_bf16 if bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    if X is None:
        X, s = features(A)
    else:
        s = features(A)[1]
    X0 = r(X)
    N0 = r(_ahat(A, X0, s))
    U1 = np.concatenate([X0, N0], axis=1)
    Z1 = U1 @ r(p["W1"]) + p["b1"]
    h1 = r(np.maximum(Z1, 0.0))
    N1 = r(_ahat(A, h1, s))
    U2 = np.concatenate([h1, N1], axis=1)
    Z2 = U2 @ r(p["W2"]) + p["b2"]
    h2 = r(np.maximum(Z2, 0.0))
    y = h2 @ p["wh"] + p["bh"][0]
    cache = dict(p=p, s=s, U1=U1, Z1=Z1, h1=h1, U2=U2, Z2=Z2, h2=h2, r=r)
    return y, cache


def loss_and_grad(theta, A, target, X=None, bf16=False):
    """Mean squared error of y against target (log w) and its gradient."""
    y, c = forward(theta, A, X, bf16)
    n = A.n
    diff = y - target
    loss = float(np.mean(diff * diff))
    dy = 2.0 * diff / n
    p, r = c["p"], c["r"]
    g = {}
    g["wh"] = c["h2"].T @ dy
    g["bh"] = np.array([dy.sum()])
    dZ2 = np.outer(dy, p["wh"]) * (c["Z2"] > 0)
    g["W2"] = c["U2"].T @ dZ2
    g["b2"] = dZ2.sum(axis=0)
    dU2 = dZ2 @ r(p["W2"]).T
    dh1 = dU2[:, :HID] + _ahat_t(A, dU2[:, HID:], c["s"])
    dZ1 = dh1 * (c["Z1"] > 0)
    g["W1"] = c["U1"].T @ dZ1
    g["b1"] = dZ1.sum(axis=0)
    return loss, pack(g)


def init_params(seed=0):
    """Scaled uniform initial weights (He-style fan-in), zero biases except bh."""
    rng = np.random.default_rng(seed)
    p = {}
    p["W1"] = rng.uniform(-1, 1, (2 * F0, HID)) * np.sqrt(6.0 / (2 * F0))
    p["b1"] = np.zeros(HID)
    p["W2"] = rng.uniform(-1, 1, (2 * HID, HID)) * np.sqrt(6.0 / (2 * HID))
    p["b2"] = np.zeros(HID)
    p["wh"] = rng.uniform(-1, 1, HID) * np.sqrt(3.0 / HID)
    p["bh"] = np.zeros(1)
    return pack(p)
