"""fp64 oracle of the learned early exit: trajectory features, the
65 -> 64 -> 64 -> 1 ReLU MLP with binary cross-entropy on logits, its
backward pass, Adam, and a bfloat16 inference emulation.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  Written from the
textbook definitions: a dense layer is y = W x + b, ReLU(a) = max(a, 0),
BCE with logits l(z, y) = max(z, 0) - z y + log(1 + exp(-|z|)) whose
derivative is sigmoid(z) - y, backpropagation by the chain rule, and Adam
(Kingma & Ba, ICLR 2015).  The physics the classifier predicts is the BML
phase transition (Marzolla, arXiv:1804.07981, Sec. 2): free flow below a
critical density, a global jam above it, both possible near it.

Parameter vector layout (row-major, out x in):
W1[64][65] | b1[64] | W2[64][64] | b2[64] | W3[64] | b3.
"""
from __future__ import annotations

import numpy as np

NI, NH = 65, 64
SIZES = [("W1", (NH, NI)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
         ("W3", (NH,)), ("b3", (1,))]
NP = sum(int(np.prod(s)) for _, s in SIZES)
assert NP == 8449


def unpack(params: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in SIZES:
        k = int(np.prod(shape))
        out[name] = np.asarray(params[o:o + k], dtype=np.float64).reshape(shape)
        o += k
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel()
                           for name, _ in SIZES])


def forward(params: np.ndarray, X: np.ndarray):
    """Logits and the intermediate values of every sample (fp64)."""
    p = unpack(params)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["W3"] + p["b3"][0]
    return z, (X, a1, h1, a2, h2)


def bce_with_logits(z: np.ndarray, y: np.ndarray) -> np.ndarray:
    return np.maximum(z, 0.0) - z * y + np.log1p(np.exp(-np.abs(z)))


def loss(params: np.ndarray, X: np.ndarray, y: np.ndarray) -> float:
    z, _ = forward(params, X)
    return float(np.mean(bce_with_logits(z, np.asarray(y, dtype=np.float64))))


def sigmoid(z):
    z = np.asarray(z, dtype=np.float64)
    return np.where(z >= 0, 1.0 / (1.0 + np.exp(-np.abs(z))),
                    np.exp(-np.abs(z)) / (1.0 + np.exp(-np.abs(z))))


def grad(params: np.ndarray, X: np.ndarray, y: np.ndarray):
    """(mean loss, gradient of the mean loss) by backpropagation."""
    p = unpack(params)
    y = np.asarray(y, dtype=np.float64)
    z, (X, a1, h1, a2, h2) = forward(params, X)
    n = len(y)
    dz = (sigmoid(z) - y) / n                 # d mean-loss / dz
    g = {"W3": h2.T @ dz, "b3": np.array([dz.sum()])}
    d2 = np.outer(dz, p["W3"]) * (a2 > 0)     # d / d a2
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ p["W2"]) * (a1 > 0)            # d / d a1
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(axis=0)
    return float(np.mean(bce_with_logits(z, y))), pack(g)


def finite_difference(params: np.ndarray, X, y, indices, h: float = 1e-6) -> np.ndarray:
    """Central differences of the mean loss for the given parameter indices."""
    out = np.empty(len(indices))
    for k, i in enumerate(indices):
        pp = np.array(params, dtype=np.float64)
        pm = pp.copy()
        pp[i] += h
        pm[i] -= h
        out[k] = (loss(pp, X, y) - loss(pm, X, y)) / (2 * h)
    return out


def adam_step(params, m, v, g, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; returns new (params, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v


# --- bfloat16 inference emulation -------------------------------------------

def to_bf16(x) -> np.ndarray:
    """float32 -> bfloat16 (kept in float32) by round to nearest, ties to
    even, on the bit pattern: add 0x7fff plus the lowest kept bit, then
    truncate the low 16 bits."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    finite = (u & 0x7f800000) != 0x7f800000
    r = np.where(finite, (u + 0x7fff + ((u >> 16) & 1)) & 0xffff0000, u & 0xffff0000)
    return r.astype(np.uint32).view(np.float32)


def infer_bf16(params: np.ndarray, X: np.ndarray) -> np.ndarray:
    """Logits with weights and each layer's input rounded to bfloat16;
    biases, products and sums in float32 (products of two bfloat16 values are
    exact in float32).  One rounding site per line: the three weight
    matrices, the input, and the two hidden activations; the biases are never
    rounded."""
    p = unpack(np.asarray(params, dtype=np.float32))
    f32 = lambda a: np.asarray(a, dtype=np.float32)   # noqa: E731
    W1 = to_bf16(f32(p["W1"]))
    W2 = to_bf16(f32(p["W2"]))
    W3 = to_bf16(f32(p["W3"]))
    b1 = f32(p["b1"])
    b2 = f32(p["b2"])
    b3 = f32(p["b3"])
    x = to_bf16(f32(X))
    h1 = to_bf16(np.maximum(x @ W1.T + b1, np.float32(0)))
    h2 = to_bf16(np.maximum(h1 @ W2.T + b2, np.float32(0)))
    return (h2 @ W3 + b3[0]).astype(np.float32)


# --- features and labels from per-step counts ---------------------------------

def mobile_fraction(moved_lr, moved_tb, cars) -> np.ndarray:
    """v_t = (LR moved + TB moved) / cars per step (1 without cars)."""
    m = np.asarray(moved_lr, dtype=np.float64) + np.asarray(moved_tb, dtype=np.float64)
    return m / cars if cars else np.ones_like(m)


def features(moved_lr, moved_tb, cars: int, rho: float, window: int = 8,
             n_windows: int = 64) -> np.ndarray:
    """f_m = mean of v_t over steps window*m+1 .. window*m+window (double,
    then rounded to float32), m < n_windows; last entry rho (float32)."""
    out = np.empty(n_windows + 1, dtype=np.float32)
    mlr = np.asarray(moved_lr, dtype=np.int64)
    mtb = np.asarray(moved_tb, dtype=np.int64)
    for m in range(n_windows):
        s = slice(window * m, window * (m + 1))
        tot = int(mlr[s].sum() + mtb[s].sum())
        out[m] = np.float32(tot / (window * cars)) if cars else np.float32(1.0)
    out[n_windows] = np.float32(rho)
    return out


def jam_label(moved_lr, moved_tb, cars: int, last: int = 1000,
              threshold: float = 0.05) -> int:
    """1 (jammed) if the mean mobile fraction over the last `last` steps is
    below `threshold`, else 0 (free flow)."""
    v = mobile_fraction(np.asarray(moved_lr)[-last:], np.asarray(moved_tb)[-last:], cars)
    return int(v.mean() < threshold)
