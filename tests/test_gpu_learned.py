"""The learned warm start end to end on the GPU: training from solver-produced
duals, prediction, the judged solve and its fallback, and the gain over the
cold start on held-out drifting days.

Iteration counts are deterministic (the library's reductions are exact), so
the comparisons below are stable from run to run."""
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2606_07777_amd", "weights", "warmstart.npz")
COLD = dict(gammas=[1e-1, 1e-2, 1e-3], iters=[300, 300, -1], tol=1e-4, max_iters=20000, check_every=10)
FINAL = dict(gammas=[1e-3], iters=[-1], tol=1e-4, max_iters=20000, check_every=10)


@pytest.fixture(scope="module")
def dl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_07777_amd as dl
    dl.load()
    return dl


def _days(dl, wl, chain, n_users, n_items, days):
    """Yields (problem updated to day d, yesterday's instance, today's instance, yesterday's duals)."""
    inst = wl.cadence_base(chain, n_users=n_users, n_items=n_items)
    prob = dl.Problem.from_instance(inst)
    lam, st = prob.solve(**COLD)
    assert st["status"] == 0
    for d in range(1, days + 1):
        today = wl.cadence_next(inst, d)
        prob.update(c=today.c, b=today.b)
        lam_today = yield prob, inst, today, lam
        inst, lam = today, lam_today


def _evaluate(dl, wl, ws, chain, n_users, n_items, days):
    out = []
    gen = _days(dl, wl, chain, n_users, n_items, days)
    step = next(gen)
    while True:
        prob, yday, today, lam = step
        _, sc = prob.solve(**COLD)
        _, sp = prob.solve(lam0=lam, **FINAL)
        ll, sl, info = ws.solve(prob, lam, yday.b, **FINAL)
        assert sc["status"] == sp["status"] == sl["status"] == 0 and sl["rel_gap"] <= 1e-4
        out.append((sc["iters"], sp["iters"], sl["iters"], info["chosen"]))
        try:
            step = gen.send(ll)
        except StopIteration:
            return out


def test_train_and_beat_cold_start(dl, wl):
    """Train on 6 small chains x 6 days, evaluate on a held-out chain."""
    from paper_2606_07777_amd.learned import WarmStart
    ws = WarmStart(hidden=128, seed=1)
    X, T = [], []
    for chain in range(7000, 7006):
        gen = _days(dl, wl, chain, 30000, 200, 6)
        step = next(gen)
        while True:
            prob, yday, today, lam = step
            F, _ = ws.features(prob, lam, yday.b)
            lam_new, st = prob.solve(lam0=lam, **FINAL)
            X.append(F.cpu().numpy())
            T.append((lam_new - lam).cpu().numpy())
            try:
                step = gen.send(lam_new)
            except StopIteration:
                break
    X, T = np.concatenate(X), np.concatenate(T)
    hist = ws.fit(X, T, epochs=40, batch=512, lr=2e-3)
    print(f"loss {hist[0]:.3f} -> {hist[-1]:.3f}")
    assert hist[-1] < 0.5 * hist[0]
    res = _evaluate(dl, wl, ws, 7100, 30000, 200, 3)
    print("cold / previous / learned iterations:", res)
    for cold, prev, learned, chosen in res:
        assert learned < cold
    assert sum(r[2] for r in res) < sum(r[1] for r in res)


def test_judge_falls_back_when_the_prediction_is_bad(dl, wl):
    """A network whose output is blown up by the target scale loses the judge."""
    from paper_2606_07777_amd.learned import WarmStart
    ws = WarmStart(hidden=64, seed=2)
    ws.s = 1e3
    gen = _days(dl, wl, 7200, 20000, 100, 1)
    prob, yday, today, lam = next(gen)
    lam_l = ws.predict(prob, lam, yday.b)
    assert bool((lam_l >= 0).all())
    ll, sl, info = ws.solve(prob, lam, yday.b, **FINAL)
    print(info)
    assert info["chosen"] == "previous" and info["duals"]["learned"] < info["duals"]["previous"]
    _, sp = prob.solve(lam0=lam, **FINAL)
    assert sl["iters"] == sp["iters"]


@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained warm-start weights")
def test_shipped_weights_beat_cold_start(dl, wl):
    """The stored network (trained on 1M x 5k chains) on a held-out 200k x 1k chain."""
    from paper_2606_07777_amd.learned import WarmStart
    ws = WarmStart.load(WEIGHTS)
    res = _evaluate(dl, wl, ws, 6100, 200_000, 1000, 2)
    print("cold / previous / learned iterations:", res)
    for cold, prev, learned, chosen in res:
        assert chosen == "learned" and learned < prev < cold
