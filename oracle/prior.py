"""CPU oracle of the learned edge prior -- TEST INFRASTRUCTURE ONLY.

The prior is an addition of this project, not part of the paper: a small MLP
scores each candidate edge (i, j) -- j the r-th nearest neighbour of i,
r < 16 -- and the score replaces eta^beta of that candidate in Eq. 1 and
Eq. 2 (Sec. 3); the fallback over all unvisited cities keeps eta^beta.

Definitions computed here, plainly and in float64:

* features of edge (i, r): (dx / s_i, dy / s_i, d_ij / s_i, r / 15) with
  dx, dy = coordinates of j minus those of i, d_ij the exact integer EUC_2D
  distance and s_i = d(i, 16th nearest neighbour) (1 if that is 0);
* MLP 4 -> 64 -> 64 -> 1, ReLU after the two hidden layers, logit z;
  score = max(sigmoid(z), 1e-6);
* training loss: mean binary cross-entropy with logits against soft labels.

``forward``/``grads`` take ``bf16=True`` to round every matrix-product
operand (inputs, weights, hidden activations, back-propagated deltas) to
bfloat16 before multiplying, which is what the GPU kernels feed their
BF16 matrix cores; products and sums stay in float64 here.
"""
from __future__ import annotations

import numpy as np

K_NN = 16
HID = 64
SCORE_MIN = 1e-6


def bf16(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), as float64."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    rounding = ((u >> 16) & 1) + 0x7FFF
    r = ((u + rounding) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def features(xy: np.ndarray, cand: np.ndarray, dist: np.ndarray) -> np.ndarray:
    """Edge features of the first 16 candidates of every city, shape (n*16, 4),
    row i*16 + r.  cand: (n, >=16) candidate lists sorted by (d, j);
    dist: exact integer distances (n, n)."""
    n = xy.shape[0]
    out = np.zeros((n * K_NN, 4), dtype=np.float32)
    for i in range(n):
        s = float(dist[i, cand[i, K_NN - 1]])
        if s == 0.0:
            s = 1.0
        for r in range(K_NN):
            j = cand[i, r]
            out[i * K_NN + r, 0] = np.float32((xy[j, 0] - xy[i, 0]) / s)
            out[i * K_NN + r, 1] = np.float32((xy[j, 1] - xy[i, 1]) / s)
            out[i * K_NN + r, 2] = np.float32(dist[i, j] / s)
            out[i * K_NN + r, 3] = np.float32(r / 15.0)
    return out


def init_params(seed: int = 0) -> dict:
    """He-uniform initial weights (float32), zero biases."""
    g = np.random.default_rng(seed)

    def he(fan_in, shape):
        lim = np.sqrt(6.0 / fan_in)
        return g.uniform(-lim, lim, size=shape).astype(np.float32)

    return {"W1": he(4, (4, HID)), "b1": np.zeros(HID, np.float32),
            "W2": he(HID, (HID, HID)), "b2": np.zeros(HID, np.float32),
            "W3": he(HID, (HID, 1)), "b3": np.zeros(1, np.float32)}


def _q(x, on):
    """Operand of a matrix product: float32 then bfloat16 (as the GPU holds it),
    or the exact float64 value."""
    return bf16(np.asarray(x, dtype=np.float32)) if on else np.asarray(x, dtype=np.float64)


def forward(p: dict, X: np.ndarray, bf16_ops: bool = False):
    """Logits z (float64) and the intermediate values needed by ``grads``."""
    x = _q(X, bf16_ops)
    a1 = x @ _q(p["W1"], bf16_ops) + p["b1"].astype(np.float64)
    h1 = np.maximum(a1, 0.0)
    a2 = _q(h1, bf16_ops) @ _q(p["W2"], bf16_ops) + p["b2"].astype(np.float64)
    h2 = np.maximum(a2, 0.0)
    z = _q(h2, bf16_ops) @ _q(p["W3"], bf16_ops) + p["b3"].astype(np.float64)
    return z[:, 0], (x, a1, h1, a2, h2)


def score(z: np.ndarray) -> np.ndarray:
    return np.maximum(1.0 / (1.0 + np.exp(-z)), SCORE_MIN)


def loss(p: dict, X: np.ndarray, y: np.ndarray, bf16_ops: bool = False) -> float:
    z, _ = forward(p, X, bf16_ops)
    # mean of log(1 + exp(-z)) for y=1 parts and log(1 + exp(z)) for y=0 parts
    return float(np.mean(np.logaddexp(0.0, z) - y * z))


def grads(p: dict, X: np.ndarray, y: np.ndarray, bf16_ops: bool = False) -> dict:
    """Gradients of ``loss`` by back-propagation (float64)."""
    z, (x, a1, h1, a2, h2) = forward(p, X, bf16_ops)
    R = X.shape[0]
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / R
    dz = dz[:, None]
    h2q = _q(h2, bf16_ops)
    g = {"W3": h2q.T @ dz, "b3": dz.sum(axis=0)}
    dh2 = (dz @ _q(p["W3"], bf16_ops).T) * (a2 > 0)
    dh2q = _q(dh2, bf16_ops)
    h1q = _q(h1, bf16_ops)
    g["W2"] = h1q.T @ dh2q
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2q @ _q(p["W2"], bf16_ops).T) * (a1 > 0)
    g["W1"] = x.T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return g


def adam_step(p: dict, g: dict, m: dict, v: dict, step: int, lr: float = 1e-3,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    """One Adam step (Kingma and Ba, ICLR 2015, Algorithm 1) in float64, in
    place on every array of p, m and v: first and second moment estimates,
    bias correction by 1 - beta^step, then p -= lr * m_hat / (sqrt(v_hat) + eps)."""
    for k in p:
        gk = np.asarray(g[k], dtype=np.float64).reshape(p[k].shape)
        m[k] = beta1 * m[k] + (1.0 - beta1) * gk
        v[k] = beta2 * v[k] + (1.0 - beta2) * gk * gk
        m_hat = m[k] / (1.0 - beta1 ** step)
        v_hat = v[k] / (1.0 - beta2 ** step)
        p[k] = p[k] - lr * m_hat / (np.sqrt(v_hat) + eps)
