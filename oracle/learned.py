"""Learned passive-set proposals on the CPU (oracle side) -- TEST INFRASTRUCTURE ONLY.

The paper starts every NNLS solve from x = 0 (Section 4.1).  The learned form
proposes an initial passive set instead: per-column features of the sketched
problem go through a small perceptron whose output is the probability that
the column is passive (x_j > 0) at the optimum.  This module is the plain FP64
definition of the features, of the network, of its loss and gradient and of
one Adam step, written out so that a reader can check it by eye.

Features of column j from the Gram form (G = SA^T SA, q = SA^T Sb, c = Sb^T Sb)
with C_jk = G_jk / sqrt(G_jj G_kk) (0 when either diagonal entry is 0):
    f0 = q_j / sqrt(G_jj c)          (0 when G_jj c = 0)
    f1 = q_j / max_k |q_k|           (0 when q = 0)
    f2 = (q_j - mean q) / std q      (population std; 0 when it is 0)
    f3 = mean_{k != j} C_jk          (0 when d = 1)
    f4 = max_{k != j} C_jk           (0 when d = 1)
    f5 = mean_{k != j} C_jk f0_k     (0 when d = 1)
    f6 = log(G_jj / mean_k G_kk) clamped to [-30, 30] (-30 when G_jj = 0)
    f7 = d / 128

Network (width 128): h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2),
z = w3 . h2 + b3, p = sigmoid(z).  The weights W1, W2, w3 are used rounded to
bfloat16 (round to nearest, ties to even); biases stay as given.  Loss: mean
over rows of softplus(z) - y z.  Parameters travel as one flat vector in the
order W1 (128 x 8 row-major), b1, W2 (128 x 128 row-major), b2, w3, b3.
"""
from __future__ import annotations

import numpy as np

F = 8
H = 128
SHAPES = [("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)),
          ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
WEIGHTS = ("W1", "W2", "w3")


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (nearest, ties to even); returned as
    float32 values.  Written from the format's definition: keep the top 16
    bits of the IEEE single, rounding on the 16 dropped bits."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lower = u & 0xFFFF
    upper = u >> 16
    round_up = (lower > 0x8000) | ((lower == 0x8000) & ((upper & 1) == 1))
    upper = upper + round_up.astype(np.uint64)
    finite = (u & 0x7F800000) != 0x7F800000
    upper = np.where(finite, upper, u >> 16)
    return ((upper & 0xFFFF) << 16).astype(np.uint32).view(np.float32).reshape(a.shape)


def unpack(theta: np.ndarray) -> dict:
    theta = np.asarray(theta)
    out, off = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = theta[off:off + size].reshape(shape)
        off += size
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1)
                           for name, _ in SHAPES])


def features(G: np.ndarray, q: np.ndarray, c: float) -> np.ndarray:
    """(d, 8) features of every column, FP64, straight from the definitions."""
    G = np.asarray(G, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    d = len(q)
    diag = np.diag(G).copy()
    X = np.zeros((d, F))
    cos = np.array([q[j] / np.sqrt(diag[j] * c) if diag[j] > 0 and c > 0 else 0.0
                    for j in range(d)])
    qmax = np.max(np.abs(q))
    qmean = np.mean(q)
    qstd = np.sqrt(np.mean((q - qmean) ** 2))
    dmean = np.mean(diag)
    for j in range(d):
        C = []
        for k in range(d):
            if k == j:
                continue
            ok = diag[j] > 0 and diag[k] > 0
            C.append((G[j, k] / np.sqrt(diag[j] * diag[k]) if ok else 0.0, cos[k]))
        X[j, 0] = cos[j]
        X[j, 1] = q[j] / qmax if qmax > 0 else 0.0
        X[j, 2] = (q[j] - qmean) / qstd if qstd > 0 else 0.0
        if C:
            X[j, 3] = np.mean([ck for ck, _ in C])
            X[j, 4] = np.max([ck for ck, _ in C])
            X[j, 5] = np.mean([ck * cosk for ck, cosk in C])
        lg = np.log(diag[j] / dmean) if diag[j] > 0 and dmean > 0 else -30.0
        X[j, 6] = min(30.0, max(-30.0, lg))
        X[j, 7] = d / 128.0
    return X


def _softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def forward(theta: np.ndarray, X: np.ndarray, bf16: bool = True) -> dict:
    """All activations of the network for the rows of X, FP64."""
    P = unpack(theta)
    W = {k: (bf16_round(P[k]).astype(np.float64) if bf16 and k in WEIGHTS else P[k])
         for k in P}
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ W["W1"].T + W["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W["W2"].T + W["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ W["w3"] + W["b3"][0]
    p = 1.0 / (1.0 + np.exp(-z))
    return {"W": W, "X": X, "a1": a1, "h1": h1, "a2": a2, "h2": h2, "z": z, "p": p}


def loss(theta: np.ndarray, X: np.ndarray, y: np.ndarray, bf16: bool = True) -> float:
    f = forward(theta, X, bf16)
    return float(np.mean(_softplus(f["z"]) - np.asarray(y, np.float64) * f["z"]))


def gradient(theta: np.ndarray, X: np.ndarray, y: np.ndarray, bf16: bool = True) -> np.ndarray:
    """d loss / d theta by the chain rule, layer by layer.  With bf16=True
    the forward pass uses the rounded weights and their gradient is returned
    for the unrounded parameters (straight-through)."""
    f = forward(theta, X, bf16)
    W = f["W"]
    N = len(f["z"])
    dz = (f["p"] - np.asarray(y, np.float64)) / N           # (N,)
    g = {"w3": f["h2"].T @ dz, "b3": np.array([dz.sum()])}
    da2 = np.outer(dz, W["w3"]) * (f["a2"] > 0)              # (N, H)
    g["W2"] = da2.T @ f["h1"]
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ W["W2"]) * (f["a1"] > 0)
    g["W1"] = da1.T @ f["X"]
    g["b1"] = da1.sum(axis=0)
    return pack(g)


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam step (Kingma & Ba 2015); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mhat = m / (1 - beta1 ** step)
    vhat = v / (1 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
