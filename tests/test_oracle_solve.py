"""Pins for the oracle's Maximizer: accelerated projected dual ascent with
Jacobi scaling and gamma continuation (Sections 4.4 and 6, Appendix C).

Independent references: a generic QP solver on the regularized primal (eq. 1),
strong and weak duality (Section 3.2), KKT conditions, a closed-form
one-dimensional case, the degree-1 case (per-item bisection), the all-slack
case, a hand-derived worked example (tests/golden/fista_1d.json), the FISTA
rate bound of Beck and Teboulle, and the projection bound on drift.
"""
import json
import os

import numpy as np
import pytest

from tests.test_oracle_dual import dense_A

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def qp_solve(inst, gamma):
    """Regularized primal (eq. 1) by a generic SQP solver, independent of the dual method."""
    from scipy.optimize import minimize
    A = dense_A(inst)
    b = inst.b.reshape(-1)
    c = inst.c.astype(np.float64)
    n = inst.nnz
    rp = inst.row_ptr
    eqr = np.zeros(A.shape[0], dtype=bool)
    for k in range(inst.n_families):
        if (getattr(inst, "eq_families", 0) >> k) & 1:
            eqr[k * inst.n_items:(k + 1) * inst.n_items] = True
    cons = []
    if (~eqr).any():
        cons.append({"type": "ineq", "fun": lambda x: b[~eqr] - A[~eqr] @ x, "jac": lambda x: -A[~eqr]})
    if eqr.any():
        cons.append({"type": "eq", "fun": lambda x: b[eqr] - A[eqr] @ x, "jac": lambda x: -A[eqr]})
    if inst.proj != "box":
        S = np.zeros((inst.n_users, n))
        for i in range(inst.n_users):
            S[i, rp[i]:rp[i + 1]] = 1.0
        kind = "eq" if inst.proj == "simplex_eq" else "ineq"
        cons.append({"type": kind, "fun": lambda x: inst.radius - S @ x, "jac": lambda x: -S})
        bounds = [(0, inst.upper if inst.proj == "boxcut" else None)] * n
    else:
        bounds = [(0, inst.radius)] * n
    res = minimize(lambda x: c @ x + 0.5 * gamma * x @ x, np.zeros(n), jac=lambda x: c + gamma * x,
                   method="SLSQP", bounds=bounds, constraints=cons,
                   options={"ftol": 1e-14, "maxiter": 2000})
    # status 8 (no descent direction left) means SLSQP stopped at its precision floor
    assert res.success or res.status == 8, res.message
    return res.x, res.fun


@pytest.mark.parametrize("kw", [
    dict(seed=21, n_users=25, n_items=5, max_degree=4, b_scale=0.3),
    dict(seed=22, n_users=20, n_items=4, max_degree=4, n_families=2, a_ones=False, b_scale=0.35),
    dict(seed=23, n_users=20, n_items=5, max_degree=4, proj="box", b_scale=0.3),
    dict(seed=24, n_users=20, n_items=5, max_degree=4, proj="boxcut", radius=1.0, upper=0.4, b_scale=0.3),
])
def test_converged_matches_qp(orc, wl, kw):
    inst = wl.random_small(**kw)
    gamma = 0.1
    lam, st, _, _ = orc.solve(inst, [gamma], [-1], tol=1e-13, max_iters=400_000, check_every=50,
                              jacobi=True)
    assert st["status"] == 0
    g, grad, x, _ = orc.dual_grad(inst, lam, gamma)
    xq, pq = qp_solve(inst, gamma)
    np.testing.assert_allclose(x, xq, atol=2e-6)
    # strong duality (Section 3.2): g(lam*) = P(x*)
    assert abs(g - pq) <= 1e-7 * max(1.0, abs(pq))
    # KKT: dual feasibility, primal feasibility, complementary slackness
    assert np.all(lam >= 0)
    assert grad.max() <= 1e-6
    assert np.abs(lam * grad).max() <= 1e-6


def test_equality_rows_free_duals_match_qp(orc, wl):
    """Equality rows A_1 x = b_1 next to capacity rows A_0 x <= b_0: the duals of
    the equality family are free (they may be negative); the converged oracle
    solve matches a generic SQP solve of the primal with the equality
    constraints, and its gradient on those rows vanishes."""
    import dataclasses
    base = wl.random_small(25, 30, 5, 4, n_families=2, a_ones=False, b_scale=0.25)
    inst = dataclasses.replace(base, eq_families=0b10)
    # equality targets reachable by construction: b_1 = A_1 x0 for a feasible x0 (half of each row's share)
    x0 = np.zeros(inst.nnz)
    for i in range(inst.n_users):
        s, e = inst.row_ptr[i], inst.row_ptr[i + 1]
        x0[s:e] = 0.5 / max(e - s, 1)
    A = dense_A(inst)
    inst.b[1] = (A[inst.n_items:] @ x0)
    gamma = 0.1
    lam, st, _, _ = orc.solve(inst, [gamma], [300_000], max_iters=300_000, check_every=0, jacobi=True)
    assert np.isnan(st["rel_gap"])
    g, grad, x, _ = orc.dual_grad(inst, lam, gamma)
    xq, pq = qp_solve(inst, gamma)
    np.testing.assert_allclose(x, xq, atol=2e-6)
    assert abs(g - pq) <= 1e-7 * max(1.0, abs(pq))
    J = inst.n_items
    assert np.abs(grad[J:]).max() <= 1e-6           # equality rows hold
    assert np.all(lam[:J] >= 0) and grad[:J].max() <= 1e-6
    assert (lam[J:] < 0).any() or (lam[J:] > 0).any()


def test_all_slack_literal_capacities(orc, wl):
    """b = 0.5 nnz/J leaves every capacity slack: lam stays exactly 0 and x = Pi_C(-c/gamma)."""
    inst = wl.tiny_plain(seed=0, binding=False)
    gamma = 1e-2
    lam, st, snaps, _ = orc.solve(inst, [gamma], [200], jacobi=False, check_every=0, snap_iters=[1, 50, 200])
    assert np.all(lam == 0.0) and np.all(snaps == 0.0)
    _, grad, x, _ = orc.dual_grad(inst, np.zeros(inst.n_items), gamma)
    assert grad.max() < 0
    np.testing.assert_array_equal(x, orc.project_rows(inst, -inst.c.astype(np.float64) / gamma))


def test_degree_one_decouples_per_item(orc, wl):
    """With one item per user the dual splits per item; lam_j* solves a monotone 1-D equation."""
    inst = wl.random_small(31, 300, 6, 1, b_scale=0.3)
    assert np.all(inst.degrees() == 1)
    gamma = 0.1
    lam, st, _, _ = orc.solve(inst, [gamma], [-1], tol=1e-14, max_iters=200_000, check_every=20, jacobi=True)
    u = -inst.c.astype(np.float64)
    for j in range(inst.n_items):
        sel = inst.item_idx == j
        load = lambda l: np.clip((u[sel] - l) / gamma, 0.0, 1.0).sum()
        bj = inst.b[0, j]
        if load(0.0) <= bj:
            ref = 0.0
        else:
            lo, hi = 0.0, 2.0
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                lo, hi = (mid, hi) if load(mid) > bj else (lo, mid)
            ref = 0.5 * (lo + hi)
        assert lam[j] == pytest.approx(ref, abs=1e-7)


def test_weak_duality_and_repair(orc, wl):
    """Along the trajectory g(lam_t) <= P(x~_t) and x~_t is feasible (Section 3.2, Table 4)."""
    inst = wl.tiny_plain(seed=0, binding=True, n_users=2000, n_items=40)
    A = dense_A(inst)
    gamma = 1e-2
    its = [1, 5, 20, 60, 150]
    _, _, snaps, _ = orc.solve(inst, [gamma], [150], jacobi=False, check_every=0, snap_iters=its)
    for lam in snaps:
        cert = orc.certificate(inst, lam, gamma)
        assert cert["dual_obj"] <= cert["primal_obj"] + 1e-9 * abs(cert["primal_obj"])
        assert cert["rel_gap"] >= -1e-12
        _, _, x, ax = orc.dual_grad(inst, lam, gamma)
        r = np.minimum(1.0, inst.b[0] / np.maximum(ax, 1e-300))
        xt = r[inst.item_idx] * x
        assert np.all(A @ xt <= inst.b[0] * (1 + 1e-12))
        for i in range(0, inst.n_users, 97):
            assert xt[inst.row_ptr[i]:inst.row_ptr[i + 1]].sum() <= 1 + 1e-12
        p, _ = orc.primal(inst, xt, gamma)
        assert p == pytest.approx(cert["primal_obj"], rel=1e-12)
        assert cert["max_slack"] == pytest.approx(max(0.0, (ax - inst.b[0]).max()), abs=1e-12)


def _one_by_one():
    from workloads import Instance
    return Instance("one_by_one", 1, 1, 1, np.array([0, 1], dtype=np.int64), np.array([0], dtype=np.int32),
                    np.array([-1.0], dtype=np.float32), np.array([[2.0]], dtype=np.float32),
                    np.array([[0.2]]), "simplex_le", 1.0)


def test_fista_worked_example(orc):
    ref = json.load(open(os.path.join(GOLDEN, "fista_1d.json")))
    inst = _one_by_one()
    for key, scale in (("step_scale_1", 1.0), ("step_scale_half", 0.5)):
        _, _, snaps, _ = orc.solve(inst, [1.0], [3], jacobi=False, check_every=0, step_scale=scale,
                                   snap_iters=[1, 2, 3])
        np.testing.assert_allclose(snaps[:, 0], ref[key]["lam"], atol=ref["tolerance"])


def test_fista_rate_bound(orc, wl):
    """g* - g(lam_k) <= 2 L ||lam_0 - lam*||^2 / (k+1)^2 (Beck-Teboulle, Thm 4.4) with L = Lhat/gamma
    in the scaled dual; plain projected ascent with the same step is slower."""
    inst = wl.tiny_plain(seed=3, binding=True, n_users=3000, n_items=30)
    gamma = 0.05
    D, Lhat = orc.scaling(inst, False)
    lam_star, st, _, _ = orc.solve(inst, [gamma], [-1], tol=1e-14, max_iters=300_000, check_every=100,
                                   jacobi=False)
    gstar = orc.dual_grad(inst, lam_star, gamma, want_x=False)[0]
    K = 400
    _, _, _, tr = orc.solve(inst, [gamma], [K], jacobi=False, check_every=0, trace=True, max_iters=K)
    R2 = np.sum(lam_star ** 2)
    L = Lhat / gamma
    k = np.arange(1, K + 1)
    assert np.all(gstar - tr[:K] <= 2 * L * R2 / (k + 1) ** 2 + 1e-9 * abs(gstar))
    # plain projected gradient ascent with the same step, for contrast
    lam = np.zeros(inst.n_items)
    for _ in range(K):
        _, grad, _, _ = orc.dual_grad(inst, lam, gamma, want_x=False)
        lam = np.maximum(0.0, lam + gamma / Lhat * grad)
    g_gd = orc.dual_grad(inst, lam, gamma, want_x=False)[0]
    assert gstar - tr[K - 1] < 0.5 * (gstar - g_gd)


def test_stage_switch_is_warm_start(orc, wl):
    """Continuation keeps lam and restarts the momentum (Section 6): two equal-gamma stages equal two
    separate solves chained through lam."""
    inst = wl.tiny_plain(seed=4, binding=True, n_users=1500, n_items=25)
    g = 0.05
    lam_ab, _, _, _ = orc.solve(inst, [g, g], [30, 40], jacobi=True, check_every=0)
    lam_a, _, _, _ = orc.solve(inst, [g], [30], jacobi=True, check_every=0)
    lam_b, _, _, _ = orc.solve(inst, [g], [40], jacobi=True, check_every=0, lam0=lam_a)
    np.testing.assert_allclose(lam_ab, lam_b, rtol=1e-15, atol=0)
    # without the reset the momentum carries over and the result differs
    lam_nr, _, _, _ = orc.solve(inst, [g, g], [30, 40], jacobi=True, check_every=0, reset_momentum=False)
    assert np.abs(lam_nr - lam_ab).max() > 1e-9


def test_drift_bound(orc, wl):
    """||x*_gamma(c) - x*_gamma(c')|| <= ||c - c'|| / gamma (projection onto a fixed convex set
    is non-expansive); the bound that makes gamma a stability control."""
    inst = wl.random_small(41, 60, 6, 4, b_scale=0.3)
    rng = np.random.default_rng(8)
    gamma = 0.2
    inst2 = wl.Instance(inst.name + "'", inst.n_users, inst.n_items, 1, inst.row_ptr, inst.item_idx,
                        (inst.c + 0.05 * rng.normal(size=inst.nnz)).astype(np.float32), None, inst.b)
    xs = []
    for I_ in (inst, inst2):
        lam, st, _, _ = orc.solve(I_, [gamma], [-1], tol=1e-13, max_iters=300_000, check_every=50)
        xs.append(orc.dual_grad(I_, lam, gamma)[2])
    dc = np.linalg.norm(inst.c.astype(np.float64) - inst2.c.astype(np.float64))
    dx = np.linalg.norm(xs[0] - xs[1])
    assert 0 < dx <= dc / gamma * (1 + 1e-6) + 1e-6
