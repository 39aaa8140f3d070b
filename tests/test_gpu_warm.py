"""GPU tests of the recurring-solve entry points: dl_problem_update (new c and
b on the same eligibility pattern) and dl_solve_warm (the candidate start with
the largest dual value at the first gamma starts the solve; the cold start
stays a candidate)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_07777_amd as dl
    dl.load()
    return dl


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_update_equals_fresh_problem(dl, wl, storage):
    """Updating day 0 with day 1's c and b gives bitwise the gradient of a
    problem built from day 1 (a, the pattern, D and the step bound are shared)."""
    import torch
    d0 = wl.cadence_base(3, n_users=20000, n_items=300)
    d1 = wl.cadence_next(d0, 1)
    p = dl.Problem.from_instance(d0, storage=storage)
    p.update(c=d1.c, b=d1.b)
    q = dl.Problem.from_instance(d1, storage=storage)
    lam = torch.from_numpy(np.random.default_rng(0).uniform(0, 0.5, size=300)).cuda()
    for gamma in (1e-1, 1e-3):
        o1, g1, x1 = p.dual_grad(lam, gamma, want_x=True)
        o2, g2, x2 = q.dual_grad(lam, gamma, want_x=True)
        assert torch.equal(g1, g2) and o1 == o2 and torch.equal(x1, x2)


def test_update_b_only_and_rejects_nonfinite(dl, wl):
    import torch
    d0 = wl.cadence_base(4, n_users=5000, n_items=50)
    p = dl.Problem.from_instance(d0)
    lam = torch.full((50,), 0.1, dtype=torch.float64, device="cuda")
    _, g0, _ = p.dual_grad(lam, 1e-2)
    p.update(b=d0.b * 2)
    _, g1, _ = p.dual_grad(lam, 1e-2)
    # grad = A x - b and x does not depend on b: doubling b shifts grad by -b
    b = torch.from_numpy(d0.b.reshape(-1)).cuda()
    torch.testing.assert_close(g0 - g1, b, rtol=1e-12, atol=1e-9 * float(b.abs().max()))
    c_bad = d0.c.copy()
    c_bad[17] = np.nan
    with pytest.raises(RuntimeError):
        p.update(c=c_bad)
    b_bad = d0.b.copy()
    b_bad[0, 3] = np.inf
    with pytest.raises(RuntimeError):
        p.update(b=b_bad)


def test_solve_warm_picks_best_and_converges_faster(dl, wl):
    import torch
    d0 = wl.cadence_base(5, n_users=50000, n_items=400)
    d1 = wl.cadence_next(d0, 1)
    sched = dict(gammas=[1e-1, 1e-2, 1e-3], iters=[300, 300, -1], tol=1e-4, max_iters=20000, check_every=10)
    p0 = dl.Problem.from_instance(d0)
    lam0, st0 = p0.solve(**sched)
    assert st0["status"] == 0
    p1 = dl.Problem.from_instance(d1)
    lam_cold, st_cold = p1.solve(**sched)
    bad = torch.full_like(lam0, float("nan"))
    # final-stage schedule only, from yesterday's duals, the cold start, or a broken prediction
    warm = dict(gammas=[1e-3], iters=[-1], tol=1e-4, max_iters=20000, check_every=10)
    lam_w, st_w, chosen, duals = p1.solve_warm([None, lam0, bad], **warm)
    print(f"cold {st_cold['iters']} iters; warm pick {chosen} duals {duals}; warm {st_w['iters']} iters")
    assert chosen == 1 and duals[2] == -np.inf and duals[1] > duals[0]
    assert st_w["status"] == 0 and st_w["rel_gap"] <= 1e-4
    assert st_w["iters"] < st_cold["iters"]
    # the judged run equals a plain solve from the chosen start
    lam_p, st_p = p1.solve(lam0=lam0, **warm)
    assert st_p["iters"] == st_w["iters"] and torch.equal(lam_p, lam_w)
    # all candidates broken -> error, nothing solved
    with pytest.raises(RuntimeError):
        p1.solve_warm([bad], **warm)
