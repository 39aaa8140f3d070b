"""dl_solve_noalloc (the solve without device allocation) against dl_solve.

Both run the same kernels on the same problem, so lam, the iteration count and
the certificate must agree bitwise.  Two calls in a row, the second on a
smaller problem, check that the fixed state array left behind by the first
call does not leak into the second; the too-large and tuner cases are
rejected with clear errors.
"""
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


def _same(dl, prob, sched):
    import torch
    ref, st_ref = prob.solve(**sched)
    out = torch.full_like(ref, float("nan"))
    got, st = prob.solve(**sched, out=out, noalloc=True)
    assert got.data_ptr() == out.data_ptr()
    assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy())
    for k in ("iters", "status", "stage", "n_checks", "dual_obj", "primal_obj", "rel_gap", "max_slack",
              "lagr_gap", "gamma"):
        a, b = st[k], st_ref[k]
        assert a == b or (isinstance(a, float) and np.isnan(a) and np.isnan(b)), (k, a, b)
    return st


def test_noalloc_solve_matches_dl_solve_twice(dl, wl):
    import torch
    big = wl.two_family(seed=0)                       # 2 x 100 rows, box, stored a
    small = wl.tiny_plain(seed=3, binding=True, n_users=3000, n_items=40)
    sched = dict(gammas=[1e-1, 1e-2, 1e-3], iters=[300, 300, -1], tol=1e-4, max_iters=20000, check_every=10)
    st1 = _same(dl, dl.Problem.from_instance(big, jacobi=True), sched)
    lam0 = torch.linspace(0.0, 0.2, small.n_items, dtype=torch.float64)
    st2 = _same(dl, dl.Problem.from_instance(small, jacobi=False),
                dict(gammas=[1e-2], iters=[150], check_every=0, lam0=lam0))
    print(f"first call {st1['iters']} iterations gap {st1['rel_gap']:.2e}; second {st2['iters']} iterations")
    assert st1["status"] == 0 and st2["iters"] == 150


def test_noalloc_rejects_what_it_cannot_hold(dl, wl):
    import paper_2606_07777_amd as pkg
    prob = dl.Problem.from_instance(wl.tiny_plain(seed=0, binding=True), jacobi=True)
    with pytest.raises(pkg.DualipError) as e:
        prob.solve([1e-2], [10], check_every=0, autotune_rounds=1, noalloc=True)
    assert "autotune" in str(e.value)
    # 2 x 9,000 dual rows: a valid problem (the histogram in device memory) whose
    # rows exceed the fixed state array
    wide = dl.Problem.from_instance(wl.random_small(93, 2000, 9000, 8, n_families=2, a_ones=False), jacobi=True)
    assert wide.nrow == 18_000
    with pytest.raises(pkg.DualipError) as e:
        wide.solve([1e-2], [10], check_every=0, noalloc=True)
    assert e.value.status == -4 and "16384" in str(e.value)
