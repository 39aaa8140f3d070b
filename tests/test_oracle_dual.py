"""Pins for the oracle's ObjectiveFunction (eqs. 2-4) and Jacobi scaling (Appendix C).

Independent references: a dense A built straight from Definition 1, central
finite differences of g (Danskin's theorem, eq. 4), concavity and the
smoothness bound L = ||A||^2/gamma (Appendix C), the inner minimum of the
Lagrangian against random feasible points, and eigenvalues of A'A'^T from
numpy.
"""
import numpy as np
import pytest

from tests.test_oracle_projection import brute_simplex


def dense_A(inst):
    """(m*J) x nnz matrix of Definition 1: row (k, j) holds a_kij at column e = (i, j)."""
    m, J, nnz = inst.n_families, inst.n_items, inst.nnz
    A = np.zeros((m * J, nnz))
    a = inst.a_dense().astype(np.float64)
    for k in range(m):
        A[k * J + inst.item_idx, np.arange(nnz)] = a[k]
    return A


def lagrangian(inst, A, x, lam, gamma):
    c = inst.c.astype(np.float64)
    return c @ x + 0.5 * gamma * x @ x + lam @ (A @ x - inst.b.reshape(-1))


CASES = [
    dict(seed=11, n_users=40, n_items=6, max_degree=5, n_families=1, proj="simplex_le"),
    dict(seed=12, n_users=40, n_items=6, max_degree=5, n_families=2, proj="simplex_le", a_ones=False),
    dict(seed=13, n_users=30, n_items=5, max_degree=4, n_families=2, proj="box"),
    dict(seed=14, n_users=30, n_items=7, max_degree=6, n_families=1, proj="simplex_eq"),
]


@pytest.fixture(params=range(len(CASES)))
def small(request, wl):
    kw = dict(CASES[request.param])
    return wl.random_small(**kw)


def test_primal_recovery_is_eq3(orc, small):
    """x*(lam) = Pi_C(-(A^T lam + c)/gamma), with Pi_C by support enumeration."""
    inst = small
    A = dense_A(inst)
    rng = np.random.default_rng(1)
    lam = rng.uniform(0, 0.5, size=A.shape[0])
    gamma = 0.3
    _, _, x, _ = orc.dual_grad(inst, lam, gamma)
    w = -(A.T @ lam + inst.c.astype(np.float64)) / gamma
    for i in range(inst.n_users):
        s, e = inst.row_ptr[i], inst.row_ptr[i + 1]
        if inst.proj == "box":
            ref = np.clip(w[s:e], 0, inst.radius)
        else:
            ref = brute_simplex(w[s:e], inst.radius, inst.proj == "simplex_eq")
        np.testing.assert_allclose(x[s:e], ref, atol=1e-12)


def test_gradient_is_danskin(orc, small):
    """grad g matches central differences of g within the Lipschitz bound of each coordinate."""
    inst = small
    A = dense_A(inst)
    rng = np.random.default_rng(2)
    gamma = 0.2
    lam = rng.uniform(0.05, 0.6, size=A.shape[0])
    g0, grad, _, _ = orc.dual_grad(inst, lam, gamma)
    h = 1e-6
    Lr = (A ** 2).sum(axis=1) / gamma
    for r in range(A.shape[0]):
        e = np.zeros_like(lam)
        e[r] = h
        gp = orc.dual_grad(inst, lam + e, gamma, want_x=False)[0]
        gm = orc.dual_grad(inst, lam - e, gamma, want_x=False)[0]
        fd = (gp - gm) / (2 * h)
        assert abs(fd - grad[r]) <= Lr[r] * h + 1e-7 * (1 + abs(g0)), (r, fd, grad[r])


def test_grad_equals_Ax_minus_b(orc, small):
    inst = small
    A = dense_A(inst)
    lam = np.random.default_rng(3).uniform(0, 1, size=A.shape[0])
    _, grad, x, ax = orc.dual_grad(inst, lam, 0.5)
    np.testing.assert_allclose(ax, A @ x, atol=1e-12)
    np.testing.assert_allclose(grad, A @ x - inst.b.reshape(-1), atol=1e-12)


def test_dual_value_is_inner_minimum(orc, small):
    """g(lam) = L(x*, lam) <= L(x, lam) for feasible x (eq. 2)."""
    inst = small
    A = dense_A(inst)
    rng = np.random.default_rng(4)
    gamma = 0.25
    lam = rng.uniform(0, 0.8, size=A.shape[0])
    g, _, x, _ = orc.dual_grad(inst, lam, gamma)
    assert abs(g - lagrangian(inst, A, x, lam, gamma)) <= 1e-10 * (1 + abs(g))
    for _ in range(200):
        y = np.empty(inst.nnz)
        for i in range(inst.n_users):
            s, e = inst.row_ptr[i], inst.row_ptr[i + 1]
            if inst.proj == "box":
                y[s:e] = rng.uniform(0, inst.radius, size=e - s)
            else:
                w = rng.dirichlet(np.ones(e - s))
                y[s:e] = w * inst.radius * (1.0 if inst.proj == "simplex_eq" else rng.uniform())
        assert lagrangian(inst, A, y, lam, gamma) >= g - 1e-10 * (1 + abs(g))


def test_concave_and_smooth(orc, small):
    """Concavity and g(l') >= g(l) + grad^T(l'-l) - (L/2)||l'-l||^2 with L = ||A||^2/gamma."""
    inst = small
    A = dense_A(inst)
    gamma = 0.3
    L = np.linalg.eigvalsh(A @ A.T).max() / gamma
    rng = np.random.default_rng(5)
    for _ in range(30):
        l1 = rng.uniform(0, 1, size=A.shape[0])
        l2 = rng.uniform(0, 1, size=A.shape[0])
        g1, gr1, _, _ = orc.dual_grad(inst, l1, gamma, want_x=False)
        g2 = orc.dual_grad(inst, l2, gamma, want_x=False)[0]
        lin = g1 + gr1 @ (l2 - l1)
        assert g2 <= lin + 1e-9 * (1 + abs(g1))
        assert g2 >= lin - 0.5 * L * np.sum((l2 - l1) ** 2) - 1e-9 * (1 + abs(g1))


@pytest.mark.parametrize("jacobi", [False, True])
def test_scaling_against_dense(orc, small, jacobi):
    inst = small
    A = dense_A(inst)
    D, Lhat = orc.scaling(inst, jacobi)
    nrm = np.linalg.norm(A, axis=1)
    Dref = np.where(nrm > 0, 1.0 / np.where(nrm > 0, nrm, 1), 1.0) if jacobi else np.ones_like(nrm)
    np.testing.assert_allclose(D, Dref, rtol=1e-14)
    As = Dref[:, None] * A
    lmax = np.linalg.eigvalsh(As @ As.T).max()
    assert Lhat >= lmax * (1 - 1e-12)
    if inst.n_families == 1:
        assert Lhat == pytest.approx(lmax, rel=1e-12)
        if jacobi:
            assert Lhat == pytest.approx(1.0, rel=1e-14)


def test_row_scaling_preserves_feasible_set(orc, small):
    """{x : Ax <= b} = {x : DAx <= Db} for positive D (Appendix C)."""
    inst = small
    A = dense_A(inst)
    D, _ = orc.scaling(inst, True)
    b = inst.b.reshape(-1)
    rng = np.random.default_rng(6)
    for _ in range(200):
        x = rng.uniform(0, 1, size=inst.nnz) * rng.uniform(0, 0.6)
        assert np.all(A @ x <= b) == np.all((D[:, None] * A) @ x <= D * b)
