"""Pins for the oracle's global-count row (Section 5's example of a new coupling
constraint: sum over all eligible (i, j) of x_ij <= M, one more dual coordinate,
one more term in A^T lam, one more gradient entry).

Independent references: the same instance without the row and with c shifted
by the row's dual (the extra term of A^T lam is a constant shift of every cost),
dense eigenvalues of the scaled A A^T on tiny instances (the step bound), a
generic QP solve of the regularized primal with the extra constraint, and
feasibility / weak duality of the certificate's repaired point.
"""
import dataclasses

import numpy as np
import pytest

from tests.test_oracle_dual import dense_A
from tests.test_oracle_solve import qp_solve


def _with_cap(inst, frac):
    """The instance with a global-count row whose cap is frac x the count at lam = 0."""
    return dataclasses.replace(inst, global_cap=float(frac * inst.n_users * inst.radius))


@pytest.mark.parametrize("kw", [
    dict(seed=31, n_users=300, n_items=12, max_degree=6, b_scale=0.4),
    dict(seed=32, n_users=300, n_items=10, max_degree=6, n_families=2, a_ones=False, proj="box", b_scale=0.4),
    dict(seed=33, n_users=300, n_items=10, max_degree=6, proj="boxcut", radius=1.0, upper=0.3, b_scale=0.4),
])
def test_global_term_is_a_cost_shift(orc, wl, kw):
    """With lam = (lam_items, lam_g): x*(lam) equals the projection for the instance
    without the row at costs c + lam_g; the item gradients agree; the extra gradient
    entry is sum x - M; g differs by lam_g (sum-x term absorbed in c) minus lam_g M."""
    base = wl.random_small(**kw)
    # costs on a 1/64 grid so that c + lam_g (lam_g = 1/8) is exact in the FP32 the instance stores
    base = dataclasses.replace(base, c=(-np.floor(-base.c.astype(np.float64) * 64) / 64).astype(np.float32))
    inst = _with_cap(base, 0.3)
    gamma = 0.05
    rng = np.random.default_rng(1)
    mJ = base.n_families * base.n_items
    lam = np.concatenate([rng.uniform(0, 0.3, mJ), [0.125]])
    g, grad, x, ax = orc.dual_grad(inst, lam, gamma)
    assert grad.size == mJ + 1 and ax.size == mJ + 1
    shifted = dataclasses.replace(base, c=(base.c.astype(np.float64) + lam[mJ]).astype(np.float32))
    assert np.array_equal(shifted.c.astype(np.float64), base.c.astype(np.float64) + lam[mJ])
    g0, grad0, x0, ax0 = orc.dual_grad(shifted, lam[:mJ], gamma)
    np.testing.assert_allclose(x, x0, rtol=0, atol=1e-12)
    np.testing.assert_allclose(grad[:mJ], grad0, rtol=0, atol=1e-9)
    assert abs(grad[mJ] - (x.sum() - inst.global_cap)) <= 1e-9 * max(1.0, x.sum())
    assert abs(ax[mJ] - x.sum()) <= 1e-9 * max(1.0, x.sum())
    # g = c.x + gamma/2 |x|^2 + lam.(Ax - b) + lam_g (sum x - M)
    #   = [(c + lam_g).x + gamma/2 |x|^2 + lam.(Ax - b)] - lam_g M
    assert abs(g - (g0 - lam[mJ] * inst.global_cap)) <= 1e-9 * max(1.0, abs(g))


@pytest.mark.parametrize("jacobi", [True, False])
@pytest.mark.parametrize("kw", [
    dict(seed=34, n_users=40, n_items=6, max_degree=4),
    dict(seed=35, n_users=40, n_items=5, max_degree=4, n_families=2, a_ones=False),
])
def test_step_bound_covers_the_largest_eigenvalue(orc, wl, kw, jacobi):
    inst = _with_cap(wl.random_small(**kw), 0.5)
    D, L = orc.scaling(inst, jacobi=jacobi)
    A = np.vstack([dense_A(inst), np.ones((1, inst.nnz))])
    As = D[:, None] * A
    ev = np.linalg.eigvalsh(As @ As.T).max()
    assert D.size == inst.n_rows
    if jacobi:
        assert abs(D[-1] - 1.0 / np.sqrt(inst.nnz)) <= 1e-15
    assert L >= ev * (1 - 1e-12)
    # the bound is not loose by more than the off-diagonal norm it adds
    print(f"lambda_max {ev:.6f}, bound {L:.6f}")
    assert L <= 3.0 * ev


def test_one_family_jacobi_bound_is_two(orc, wl):
    """m = 1, a = 1, Jacobi: the item blocks are 1, d_g = 1 and ||c||_2 = 1, so the
    bound is 2, which is also the exact largest eigenvalue (1 + ||c||)."""
    inst = _with_cap(wl.random_small(36, 50, 6, 4), 0.5)
    _, L = orc.scaling(inst, jacobi=True)
    A = np.vstack([dense_A(inst), np.ones((1, inst.nnz))])
    D, _ = orc.scaling(inst, jacobi=True)
    ev = np.linalg.eigvalsh((D[:, None] * A) @ (D[:, None] * A).T).max()
    assert abs(L - 2.0) <= 1e-12 and abs(ev - 2.0) <= 1e-9


def _qp_with_cap(inst, gamma):
    """The regularized primal with the global-count row by SLSQP: the item rows and
    the cap appended to A, b as one more inequality row."""
    A = np.vstack([dense_A(inst), np.ones((1, inst.nnz))])
    b = np.concatenate([inst.b.reshape(-1), [inst.global_cap]])
    flat = dataclasses.replace(inst, n_families=1, n_items=A.shape[0], global_cap=None,
                               b=b[None, :], a=None)
    # qp_solve builds A from the instance's families; hand it the stacked rows instead
    import tests.test_oracle_solve as tos
    orig = tos.dense_A
    tos.dense_A = lambda _inst: A
    try:
        return qp_solve(flat, gamma)
    finally:
        tos.dense_A = orig


@pytest.mark.parametrize("kw", [
    dict(seed=37, n_users=20, n_items=5, max_degree=4, b_scale=0.6),
    dict(seed=38, n_users=18, n_items=4, max_degree=4, n_families=2, a_ones=False, proj="box", b_scale=0.6),
])
def test_converged_solve_matches_qp_with_cap(orc, wl, kw):
    inst = _with_cap(wl.random_small(**kw), 0.35)
    gamma = 0.1
    lam, st, _, _ = orc.solve(inst, [gamma], [-1], tol=1e-13, max_iters=400_000, check_every=50, jacobi=True)
    assert st["status"] == 0
    g, grad, x, _ = orc.dual_grad(inst, lam, gamma)
    xq, pq = _qp_with_cap(inst, gamma)
    np.testing.assert_allclose(x, xq, atol=2e-6)
    assert abs(g - pq) <= 1e-7 * max(1.0, abs(pq))
    # the cap binds: positive dual, count at the cap
    assert lam[-1] > 1e-6
    assert abs(x.sum() - inst.global_cap) <= 1e-5 * inst.global_cap
    assert np.all(lam >= 0) and grad.max() <= 1e-6 and np.abs(lam * grad).max() <= 1e-6


def test_certificate_repair_is_feasible_and_weakly_dual(orc, wl):
    """At points where the count exceeds the cap, the certificate's repaired primal
    value bounds the dual value from above (weak duality), and repairing x by the
    factor it uses gives a feasible point."""
    inst = _with_cap(wl.random_small(39, 400, 10, 6, b_scale=0.5), 0.25)
    gamma = 0.05
    mJ = inst.n_families * inst.n_items
    rng = np.random.default_rng(3)
    repaired = 0
    for trial in range(5):
        lam = np.concatenate([rng.uniform(0, 0.2, mJ), [rng.uniform(0, 0.05)]])
        c = orc.certificate(inst, lam, gamma)
        g, grad, x, ax = orc.dual_grad(inst, lam, gamma)
        assert c["dual_obj"] <= c["primal_obj"] + 1e-9 * abs(c["primal_obj"])
        assert c["max_slack"] >= grad[-1] - 1e-12
        # the repair: item factors min(1, b/Ax) times rho = min(1, M / sum x)
        rho = min(1.0, inst.global_cap / x.sum()) if x.sum() > 0 else 1.0
        repaired += rho < 1.0
        r = np.minimum(1.0, np.where(ax[:mJ] > inst.b.reshape(-1), inst.b.reshape(-1) / ax[:mJ], 1.0)) * rho
        xt = r[inst.item_idx] * x
        assert xt.sum() <= inst.global_cap * (1 + 1e-12)
        ax_t = np.bincount(inst.item_idx, weights=xt, minlength=inst.n_items)
        assert np.all(ax_t <= inst.b.reshape(-1) * (1 + 1e-12) + 1e-12)
        p = float(inst.c.astype(np.float64) @ xt + 0.5 * gamma * xt @ xt)
        assert abs(p - c["primal_obj"]) <= 1e-9 * max(1.0, abs(p))
    assert repaired >= 3  # the cap was exceeded, so the global factor did its part
