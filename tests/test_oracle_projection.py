"""Pins for the oracle's per-user projections (ProjectionMap, Table 1).

The simplex projection follows the sort-based method the paper cites in
Section 4.3; the box projection is the box variant of the per-user set
(Section 3.3).  Each check here is independent of that algorithm: brute force
over every candidate support, a generic constrained solver, closed-form
special cases, and the defining optimality conditions.
"""
import itertools

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st


def brute_simplex(v, z, eq):
    """argmin 1/2||x - v||^2 over {x >= 0, sum x <= z} (or = z) by enumerating supports.

    For every support S the only stationary point with that support is
    x_S = v_S - t with t = (sum v_S - z)/|S| (the constraint is tight), or, for
    the inequality set, x = max(v, 0) with the constraint loose.  The minimiser
    is the best feasible candidate.
    """
    v = np.asarray(v, dtype=float)
    d = v.size
    cands = []
    if not eq:
        x = np.maximum(v, 0.0)
        if x.sum() <= z + 1e-15:
            cands.append(x)
    for r in range(1, d + 1):
        for S in itertools.combinations(range(d), r):
            S = list(S)
            t = (v[S].sum() - z) / r
            x = np.zeros(d)
            x[S] = v[S] - t
            if np.all(x >= -1e-15) and (x.sum() <= z + 1e-12):
                cands.append(np.maximum(x, 0.0))
    best = min(cands, key=lambda x: 0.5 * np.sum((x - v) ** 2))
    return best


@pytest.mark.parametrize("eq", [False, True])
@pytest.mark.parametrize("d", [1, 2, 3, 5, 8])
def test_simplex_matches_support_enumeration(orc, eq, d):
    rng = np.random.default_rng(100 + d + 10 * eq)
    for trial in range(40):
        scale = [0.1, 1.0, 10.0][trial % 3]
        v = rng.normal(size=d) * scale
        z = [1.0, 0.5, 2.0][trial % 3]
        x = orc.project_simplex(v, z, eq)
        xb = brute_simplex(v, z, eq)
        np.testing.assert_allclose(x, xb, atol=1e-12, rtol=0)


def test_simplex_matches_generic_solver(orc):
    from scipy.optimize import minimize
    rng = np.random.default_rng(7)
    for trial in range(5):
        d = 15
        v = rng.normal(size=d) * 2
        z = 1.0
        res = minimize(lambda x: 0.5 * np.sum((x - v) ** 2), np.full(d, z / d), jac=lambda x: x - v,
                       method="SLSQP", bounds=[(0, None)] * d,
                       constraints=[{"type": "ineq", "fun": lambda x: z - x.sum(), "jac": lambda x: -np.ones(d)}],
                       options={"ftol": 1e-15, "maxiter": 500})
        x = orc.project_simplex(v, z)
        np.testing.assert_allclose(x, res.x, atol=1e-7)


def test_simplex_special_cases(orc):
    # every coordinate non-positive: the projection is 0
    np.testing.assert_array_equal(orc.project_simplex([-1.0, -0.5, 0.0], 1.0), [0, 0, 0])
    # one coordinate: clamp to [0, z]
    for v in (-3.0, 0.25, 0.999, 7.5):
        assert orc.project_simplex([v], 1.0)[0] == min(max(v, 0.0), 1.0)
    # constant vector with d*alpha > z: mass z/d each
    np.testing.assert_allclose(orc.project_simplex([3.0] * 4, 1.0), [0.25] * 4, rtol=0, atol=1e-15)
    # positive part inside the simplex: early exit returns max(v, 0) exactly
    v = np.array([0.2, -1.0, 0.3, 0.1])
    np.testing.assert_array_equal(orc.project_simplex(v, 1.0), np.maximum(v, 0))
    # equality set moves a feasible-inequality point onto the face
    x = orc.project_simplex(v, 1.0, eq=True)
    assert abs(x.sum() - 1.0) < 1e-15
    # a dominant coordinate takes everything: v = (10, 0, -1) -> (1, 0, 0)
    np.testing.assert_allclose(orc.project_simplex([10.0, 0.0, -1.0], 1.0), [1, 0, 0], atol=0)
    # two-point closed form: v=(a, b) with a-b < z and a+b > z -> ((z+a-b)/2, (z-a+b)/2)
    a, b = 0.9, 0.6
    np.testing.assert_allclose(orc.project_simplex([a, b], 1.0), [(1 + a - b) / 2, (1 - a + b) / 2], atol=1e-15)


vec = st.lists(st.floats(-50, 50, allow_nan=False, allow_infinity=False), min_size=1, max_size=40)


@settings(max_examples=200, deadline=None)
@given(vec, st.sampled_from([0.5, 1.0, 3.0]), st.booleans())
def test_simplex_kkt_and_invariants(orc, v, z, eq):
    v = np.array(v)
    x = orc.project_simplex(v, z, eq)
    tol = 1e-9 * (1 + np.abs(v).max())
    # feasibility
    assert np.all(x >= 0)
    if eq:
        assert abs(x.sum() - z) <= tol
    else:
        assert x.sum() <= z + tol
    # optimality conditions: x = max(v - theta, 0) with theta >= 0 for the
    # inequality set and theta = 0 unless the budget is tight
    act = x > 0
    if act.any():
        theta = np.mean(v[act] - x[act])
        np.testing.assert_allclose(v[act] - x[act], theta, atol=tol)
        assert np.all(v[~act] <= theta + tol)
        if not eq:
            assert theta >= -tol
            if x.sum() < z - tol:
                assert abs(theta) <= tol
    # idempotence
    np.testing.assert_allclose(orc.project_simplex(x, z, eq), x, atol=tol)


@settings(max_examples=100, deadline=None)
@given(st.integers(1, 30), st.integers(0, 10_000), st.booleans())
def test_simplex_nonexpansive(orc, d, seed, eq):
    rng = np.random.default_rng(seed)
    v, w = rng.normal(size=d) * 3, rng.normal(size=d) * 3
    px, pw = orc.project_simplex(v, 1.0, eq), orc.project_simplex(w, 1.0, eq)
    assert np.linalg.norm(px - pw) <= np.linalg.norm(v - w) * (1 + 1e-12) + 1e-12


def test_box_closed_form(orc):
    rng = np.random.default_rng(3)
    v = rng.normal(size=1000) * 2
    for u in (0.5, 1.0, 2.0):
        x = orc.project_box(v, u)
        # coordinate-wise minimiser of 1/2(x - v)^2 on [0, u]
        for xi, vi in zip(x[:50], v[:50]):
            grid = np.array([0.0, u, min(max(vi, 0.0), u)])
            assert xi == grid[np.argmin((grid - vi) ** 2)]
        assert np.all((x >= 0) & (x <= u))


def test_project_rows_blockwise(orc, wl):
    inst = wl.random_small(5, 200, 30, 12, proj="simplex_le")
    rng = np.random.default_rng(5)
    v = rng.normal(size=inst.nnz) * 2
    x = orc.project_rows(inst, v)
    rp = inst.row_ptr
    for i in range(0, inst.n_users, 7):
        s, e = rp[i], rp[i + 1]
        np.testing.assert_allclose(x[s:e], brute_simplex(v[s:e], 1.0, False) if e - s <= 8
                                   else orc.project_simplex(v[s:e], 1.0), atol=1e-12)


def brute_boxcut(v, u, z):
    """argmin 1/2||x - v||^2 over {0 <= x <= u, sum x <= z} by enumerating, for
    every coordinate, whether it sits at 0, at u or strictly between.  With the
    sum constraint loose the candidate is clamp(v, 0, u); with it tight the free
    coordinates F and capped coordinates C fix the multiplier
    t = (|C| u + sum_F v - z) / |F| and x_F = v_F - t.  Every feasible candidate
    is scored; the strictly convex problem has its minimiser among them."""
    v = np.asarray(v, dtype=float)
    d = v.size
    cands = []
    x0 = np.clip(v, 0.0, u)
    if x0.sum() <= z + 1e-12:
        cands.append(x0)
    for states in itertools.product((0, 1, 2), repeat=d):
        F = [e for e in range(d) if states[e] == 1]
        C = [e for e in range(d) if states[e] == 2]
        if not F:
            continue
        t = (len(C) * u + v[F].sum() - z) / len(F)
        x = np.zeros(d)
        x[C] = u
        x[F] = v[F] - t
        if t >= -1e-12 and np.all(x >= -1e-12) and np.all(x <= u + 1e-12) and x.sum() <= z + 1e-9:
            cands.append(np.clip(x, 0.0, u))
    return min(cands, key=lambda x: 0.5 * np.sum((x - v) ** 2))


@pytest.mark.parametrize("d", [1, 2, 3, 5, 6])
def test_boxcut_matches_state_enumeration(orc, d):
    rng = np.random.default_rng(100 + d)
    for _ in range(40):
        v = rng.normal(size=d) * 2
        u = float(rng.uniform(0.1, 1.5))
        z = float(rng.uniform(0.2, 3.0))
        np.testing.assert_allclose(orc.project_boxcut(v, u, z), brute_boxcut(v, u, z), atol=1e-10)


def test_boxcut_special_cases(orc):
    rng = np.random.default_rng(7)
    for _ in range(50):
        d = int(rng.integers(1, 40))
        v = rng.normal(size=d) * 3
        z = float(rng.uniform(0.1, 2.0))
        # u >= z: the cap is implied by the sum, the set is the simplex <= z
        np.testing.assert_allclose(orc.project_boxcut(v, z * 1.5, z), orc.project_simplex(v, z), atol=1e-12)
        # z >= d u: the sum is implied by the cap, the set is the box
        u = float(rng.uniform(0.1, 1.0))
        np.testing.assert_allclose(orc.project_boxcut(v, u, d * u + 1.0), orc.project_box(v, u), atol=0)


def test_boxcut_kkt_and_generic_solver(orc):
    from scipy.optimize import minimize
    rng = np.random.default_rng(8)
    for trial in range(30):
        d = int(rng.integers(2, 30))
        v = rng.normal(size=d) * 2 + 0.5
        u, z = float(rng.uniform(0.2, 1.0)), float(rng.uniform(0.5, 4.0))
        x = orc.project_boxcut(v, u, z)
        # KKT: x = clamp(v - t, 0, u) for one t >= 0, complementary to the sum constraint
        assert np.all(x >= 0) and np.all(x <= u) and x.sum() <= z + 1e-12
        free = (x > 1e-12) & (x < u - 1e-12)
        if free.any():
            t = np.mean(v[free] - x[free])
            np.testing.assert_allclose(v[free] - x[free], t, atol=1e-10)
            assert t >= -1e-10
            np.testing.assert_allclose(np.clip(v - t, 0, u), x, atol=1e-10)
            if t > 1e-10:
                assert abs(x.sum() - z) <= 1e-10
        if trial < 10:
            r = minimize(lambda y: 0.5 * np.sum((y - v) ** 2), np.full(d, min(u, z / d) * 0.5),
                         jac=lambda y: y - v, bounds=[(0, u)] * d,
                         constraints=[{"type": "ineq", "fun": lambda y: z - y.sum(), "jac": lambda y: -np.ones(d)}],
                         method="SLSQP", options={"ftol": 1e-14, "maxiter": 500})
            np.testing.assert_allclose(x, r.x, atol=1e-6)
