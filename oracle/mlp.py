"""FP64 oracle of the learned warm start (TEST INFRASTRUCTURE ONLY).

Not from the paper: the paper has no learned component.  It recurs daily
solves on slowly drifting inputs (Sections 1 and 6) and warm-starts each
continuation stage from the previous dual iterate; the learned warm start
predicts today's duals from per-item features and yesterday's duals.  Parity
with the paper is therefore unpinned; these functions are pinned against
finite differences and closed forms in tests/test_oracle_mlp.py.

Network: x (n_in, zero-padded to 16) -> 256 -> 256 -> 1 with ReLU, i.e.
    h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), y = h2 w3 + b3.
Loss: L = (1 / 2n) sum_i (y_i - t_i)^2.
Optimiser: AdamW (Loshchilov & Hutter) with decoupled weight decay on the
weight matrices.
"""
from __future__ import annotations

import numpy as np

N_IN = 16
HIDDEN = 256


def param_sizes(n_in: int = N_IN, hidden: int = HIDDEN):
    """Flat layout: W1 [n_in, H], b1 [H], W2 [H, H], b2 [H], w3 [H], b3 [1]."""
    return [("W1", (n_in, hidden)), ("b1", (hidden,)), ("W2", (hidden, hidden)), ("b2", (hidden,)),
            ("w3", (hidden,)), ("b3", (1,))]


def unflatten(flat: np.ndarray, n_in: int = N_IN, hidden: int = HIDDEN) -> dict:
    out, off = {}, 0
    for name, shape in param_sizes(n_in, hidden):
        size = int(np.prod(shape))
        out[name] = np.asarray(flat[off:off + size], dtype=np.float64).reshape(shape)
        off += size
    assert off == flat.size
    return out


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in param_sizes(
        p["W1"].shape[0], p["W1"].shape[1])])


def forward(p: dict, x: np.ndarray):
    """Returns (y [n], cache)."""
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ p["W1"] + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["w3"] + p["b3"][0]
    return y, (x, z1, h1, z2, h2)


def backward(p: dict, cache, dy: np.ndarray) -> dict:
    """Gradient of sum_i dy_i * y_i with respect to every parameter (chain rule)."""
    x, z1, h1, z2, h2 = cache
    dy = np.asarray(dy, dtype=np.float64)
    g = {}
    g["w3"] = h2.T @ dy
    g["b3"] = np.array([dy.sum()])
    dh2 = np.outer(dy, p["w3"]) * (z2 > 0)
    g["W2"] = h1.T @ dh2
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ p["W2"].T) * (z1 > 0)
    g["W1"] = x.T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return g


def mse(y: np.ndarray, t: np.ndarray):
    """(L, dL/dy) with L = (1 / 2n) sum (y - t)^2."""
    r = np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    n = max(r.size, 1)
    return 0.5 * float(r @ r) / n, r / n


def adamw_step(p: dict, g: dict, m: dict, v: dict, step: int, lr: float, beta1: float = 0.9,
               beta2: float = 0.999, eps: float = 1e-8, wd: float = 0.0):
    """One AdamW update (step counts from 1); decay applies to W1, W2, w3 only."""
    out = {}
    for k in p:
        m[k] = beta1 * m[k] + (1 - beta1) * g[k]
        v[k] = beta2 * v[k] + (1 - beta2) * g[k] * g[k]
        mh = m[k] / (1 - beta1 ** step)
        vh = v[k] / (1 - beta2 ** step)
        decay = wd * p[k] if k in ("W1", "W2", "w3") else 0.0
        out[k] = p[k] - lr * (mh / (np.sqrt(vh) + eps) + decay)
    return out


def init_params(seed: int, n_in: int = N_IN, hidden: int = HIDDEN, n_used: int = 12) -> dict:
    """He-normal weights (rows of W1 past the used inputs are zero), zero biases."""
    rng = np.random.default_rng(seed)
    W1 = np.zeros((n_in, hidden))
    W1[:n_used] = rng.normal(size=(n_used, hidden)) * np.sqrt(2.0 / n_used)
    return {"W1": W1, "b1": np.zeros(hidden), "W2": rng.normal(size=(hidden, hidden)) * np.sqrt(2.0 / hidden),
            "b2": np.zeros(hidden), "w3": rng.normal(size=hidden) * np.sqrt(1.0 / hidden), "b3": np.zeros(1)}


# -------------------------------------------------------------------------- #
# Per-item features of a day's instance                                       #
# -------------------------------------------------------------------------- #
N_FEAT = 12


def item_features(inst, lam_prev, slack_prev, b_prev) -> np.ndarray:
    """[J, 16] features of every item (one family), FP64, columns:
    0 b/n, 1 log1p(n)/10, 2 mean c, 3 std c, 4 max c, 5 min c over the item's
    eligible users, 6 lam_prev, 7 [lam_prev > 0], 8 b_prev/n,
    9 clip(g_prev/b_prev, -1, 1) with g_prev a gradient A x - b taken at
    lam_prev (the warm-start pipeline uses today's instance there, giving
    today's relative over-subscription at yesterday's duals),
    10 10 (b/b_prev - 1), 11 n / mean n; 12..15 zero.  Items with no eligible
    user get n = 0 and c statistics 0."""
    J = inst.n_items
    idx = inst.item_idx
    c = inst.c.astype(np.float64)
    n = np.bincount(idx, minlength=J).astype(np.float64)
    s1 = np.bincount(idx, weights=c, minlength=J)
    s2 = np.bincount(idx, weights=c * c, minlength=J)
    mx = np.full(J, -np.inf)
    mn = np.full(J, np.inf)
    np.maximum.at(mx, idx, c)
    np.minimum.at(mn, idx, c)
    nn = np.maximum(n, 1.0)
    mean = s1 / nn
    var = np.maximum(s2 / nn - mean * mean, 0.0)
    has = n > 0
    b = inst.b.reshape(-1).astype(np.float64)
    bp = np.asarray(b_prev, dtype=np.float64).reshape(-1)
    lp = np.asarray(lam_prev, dtype=np.float64).reshape(-1)
    sp = np.asarray(slack_prev, dtype=np.float64).reshape(-1)
    F = np.zeros((J, 16))
    F[:, 0] = b / nn
    F[:, 1] = np.log1p(n) / 10.0
    F[:, 2] = np.where(has, mean, 0.0)
    F[:, 3] = np.where(has, np.sqrt(var), 0.0)
    F[:, 4] = np.where(has, mx, 0.0)
    F[:, 5] = np.where(has, mn, 0.0)
    F[:, 6] = lp
    F[:, 7] = (lp > 0).astype(np.float64)
    F[:, 8] = bp / nn
    F[:, 9] = np.clip(sp / np.maximum(bp, 1e-12), -1.0, 1.0)
    F[:, 10] = 10.0 * (b / np.maximum(bp, 1e-12) - 1.0)
    F[:, 11] = n / max(n.mean(), 1e-12)
    return F
