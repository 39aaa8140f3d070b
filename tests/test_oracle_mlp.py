"""Pins of the learned-warm-start oracle (oracle/mlp.py).

The paper has no learned part, so nothing here is pinned to the paper; the
pins are mathematical: finite differences of the forward map for every
backward gradient, the closed-form first AdamW step, and the feature map
against direct per-item loops."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def mlp():
    from oracle import mlp
    return mlp


def small_params(mlp, seed=0, n_in=16, hidden=8):
    rng = np.random.default_rng(seed)
    return {"W1": rng.normal(size=(n_in, hidden)), "b1": rng.normal(size=hidden) * 0.1,
            "W2": rng.normal(size=(hidden, hidden)) / 3, "b2": rng.normal(size=hidden) * 0.1,
            "w3": rng.normal(size=hidden), "b3": rng.normal(size=1)}


def test_backward_matches_finite_differences(mlp):
    rng = np.random.default_rng(1)
    p = small_params(mlp)
    x = rng.normal(size=(7, 16))
    t = rng.normal(size=7)

    def loss(q):
        return mlp.mse(mlp.forward(q, x)[0], t)[0]

    y, cache = mlp.forward(p, x)
    _, dy = mlp.mse(y, t)
    g = mlp.backward(p, cache, dy)
    h = 1e-6
    for name in p:
        for flat_i in range(min(p[name].size, 12)):
            q = {k: v.copy() for k, v in p.items()}
            q[name].reshape(-1)[flat_i] += h
            lp = loss(q)
            q[name].reshape(-1)[flat_i] -= 2 * h
            lm = loss(q)
            fd = (lp - lm) / (2 * h)
            assert g[name].reshape(-1)[flat_i] == pytest.approx(fd, rel=1e-5, abs=1e-8), (name, flat_i)


def test_forward_is_composition(mlp):
    """Explicit per-row loops reproduce the vectorised forward."""
    rng = np.random.default_rng(2)
    p = small_params(mlp, hidden=5)
    x = rng.normal(size=(4, 16))
    y, _ = mlp.forward(p, x)
    for i in range(4):
        h1 = [max(0.0, sum(x[i, k] * p["W1"][k, j] for k in range(16)) + p["b1"][j]) for j in range(5)]
        h2 = [max(0.0, sum(h1[k] * p["W2"][k, j] for k in range(5)) + p["b2"][j]) for j in range(5)]
        assert y[i] == pytest.approx(sum(h2[k] * p["w3"][k] for k in range(5)) + p["b3"][0], rel=1e-12)


def test_adamw_first_step_closed_form(mlp):
    """At step 1 the bias-corrected moments are g and g^2, so the update is
    lr * (g / (|g| + eps) + wd * p) = lr * (sign(g) + wd * p) up to eps."""
    p = small_params(mlp)
    g = {k: np.random.default_rng(3).normal(size=v.shape) for k, v in p.items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    lr, wd = 1e-3, 0.01
    q = mlp.adamw_step(p, g, m, v, 1, lr, eps=0.0, wd=wd)
    for k in p:
        decay = wd * p[k] if k in ("W1", "W2", "w3") else 0.0
        np.testing.assert_allclose(q[k], p[k] - lr * (np.sign(g[k]) + decay), rtol=0, atol=1e-15)


def test_training_reduces_loss(mlp):
    rng = np.random.default_rng(4)
    x = rng.normal(size=(256, 16))
    t = np.tanh(x[:, 0]) + 0.5 * x[:, 1]
    p = mlp.init_params(0, hidden=32)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    l0 = mlp.mse(mlp.forward(p, x)[0], t)[0]
    for step in range(1, 301):
        y, cache = mlp.forward(p, x)
        _, dy = mlp.mse(y, t)
        p = mlp.adamw_step(p, mlp.backward(p, cache, dy), m, v, step, 3e-3)
    assert mlp.mse(mlp.forward(p, x)[0], t)[0] < 0.1 * l0


def test_item_features_against_loops(mlp, wl):
    inst = wl.tiny_plain(seed=5, binding=True, n_users=500, n_items=20)
    rng = np.random.default_rng(5)
    lam_prev = np.maximum(0, rng.normal(size=20) * 0.1)
    slack = rng.normal(size=20)
    b_prev = inst.b[0] * (1 + 0.05 * rng.uniform(-1, 1, size=20))
    F = mlp.item_features(inst, lam_prev, slack, b_prev)
    for j in range(20):
        cj = [float(inst.c[e]) for e in range(inst.nnz) if inst.item_idx[e] == j]
        n = len(cj)
        assert F[j, 0] == pytest.approx(inst.b[0, j] / n)
        assert F[j, 1] == pytest.approx(np.log1p(n) / 10)
        assert F[j, 2] == pytest.approx(np.mean(cj))
        assert F[j, 3] == pytest.approx(np.std(cj), abs=1e-12)
        assert F[j, 4] == max(cj) and F[j, 5] == min(cj)
        assert F[j, 7] == (1.0 if lam_prev[j] > 0 else 0.0)
        assert F[j, 9] == pytest.approx(np.clip(slack[j] / b_prev[j], -1, 1))
        assert F[j, 10] == pytest.approx(10 * (inst.b[0, j] / b_prev[j] - 1))
    assert np.all(F[:, 12:] == 0)
