"""Error paths and degenerate inputs of the C ABI on the GPU.  Every invalid
input here is rejected by a host check or by the device validation pass,
whose reads stay inside the arrays the row pointers describe."""
import dataclasses

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


@pytest.fixture(scope="module")
def base(wl):
    return wl.random_small(90, 500, 40, 12, n_families=2, a_ones=False)


def _status(exc):
    return exc.value.args[0] if exc.value.args else None


def make(dl, inst, **kw):
    return dl.Problem.from_instance(inst, **kw)


def test_malformed_csr_is_rejected(dl, base):
    rp = base.row_ptr.copy()
    rp[3], rp[4] = rp[4], rp[3]              # not nondecreasing
    with pytest.raises(RuntimeError, match="nondecreasing"):
        make(dl, dataclasses.replace(base, row_ptr=rp))
    idx = base.item_idx.copy()
    idx[7] = base.n_items                     # item out of range
    with pytest.raises(RuntimeError):
        make(dl, dataclasses.replace(base, item_idx=idx))
    idx = base.item_idx.copy()
    s = int(base.row_ptr[np.argmax(np.diff(base.row_ptr) >= 2)])
    idx[s + 1] = idx[s]                       # repeated item inside a row
    with pytest.raises(RuntimeError):
        make(dl, dataclasses.replace(base, item_idx=idx))


def test_non_finite_data_is_rejected(dl, base):
    c = base.c.copy()
    c[11] = np.inf
    with pytest.raises(RuntimeError):
        make(dl, dataclasses.replace(base, c=c))
    a = base.a.copy()
    a[1, 5] = np.nan
    with pytest.raises(RuntimeError):
        make(dl, dataclasses.replace(base, a=a))
    b = base.b.copy()
    b[0, 2] = np.nan
    with pytest.raises(RuntimeError):
        make(dl, dataclasses.replace(base, b=b))


def test_unsupported_shapes_and_options(dl, base, wl):
    with pytest.raises(RuntimeError):
        make(dl, dataclasses.replace(base, eq_families=0b100))        # family 2 does not exist
    with pytest.raises(RuntimeError):
        make(dl, dataclasses.replace(base, proj="boxcut", upper=0.0))  # box-cut needs u > 0
    big = wl.random_small(91, 200, 16384, 5)                          # J beyond the 16-bit item offsets
    with pytest.raises(RuntimeError):
        make(dl, big)
    wide = wl.random_small(92, 200, 14000, 5, n_families=2, a_ones=False)  # duals + factors beyond LDS
    with pytest.raises(RuntimeError):
        make(dl, wide)


def test_batch_rejects_a_problem_twice(dl, base):
    """Members keep per-pass state (fixed-point scales, partial slots) in their problem, so
    one problem cannot be two members; mixed kernel variants are refused too."""
    import dataclasses as dc
    p = make(dl, base)
    with pytest.raises(RuntimeError, match="twice"):
        dl.Batch([p, p])
    one = make(dl, dc.replace(base, n_families=1, a=None, b=base.b[:1], eq_families=0))
    with pytest.raises(RuntimeError):
        dl.Batch([p, one])


def test_bad_call_arguments(dl, base):
    import torch
    p = make(dl, base)
    lam = torch.zeros(base.n_families * base.n_items, dtype=torch.float64)
    with pytest.raises(RuntimeError):
        p.dual_grad(lam, 0.0)
    with pytest.raises(RuntimeError):
        p.dual_grad(lam, float("nan"))
    with pytest.raises(RuntimeError):
        p.solve([1e-2, 1e-3], [-1, 10])                               # only the last stage may run to tol


def test_iteration_cap_returns_valid_state(dl, orc, base):
    p = make(dl, base)
    lam, st = p.solve([1e-3], [-1], tol=1e-14, max_iters=40, check_every=10)
    assert st["status"] == 1 and st["iters"] == 40                    # DL_NOT_CONVERGED, results valid
    lam = lam.cpu().numpy()
    assert np.all(np.isfinite(lam)) and np.all(lam >= 0)
    lo, _, _, _ = orc.solve(base, [1e-3], [40], jacobi=True, check_every=0)
    assert np.linalg.norm(lam - lo) <= 1e-5 * max(np.linalg.norm(lo), 1e-300)


def test_empty_rows_and_empty_instance(dl, orc, wl):
    import torch
    inst = wl.random_small(92, 3000, 60, 20)
    # drop every third user's row: users with no eligible item
    keep = np.ones(inst.n_users, dtype=bool)
    keep[::3] = False
    deg = np.diff(inst.row_ptr) * keep
    rp = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    mask = np.repeat(keep, np.diff(inst.row_ptr))
    sparse = dataclasses.replace(inst, row_ptr=rp, item_idx=inst.item_idx[mask], c=inst.c[mask])
    p = make(dl, sparse)
    lam = np.full(60, 0.05)
    g, grad, x = p.dual_grad(torch.from_numpy(lam), 1e-2, want_x=True)
    go, grad_o, x_o, _ = orc.dual_grad(sparse, lam.astype(np.float32).astype(np.float64), 1e-2)
    assert abs(g - go) <= 2e-6 * max(1.0, abs(go))
    np.testing.assert_allclose(grad.cpu().numpy(), grad_o, rtol=1e-5, atol=1e-4)
    # no users at all: A x = 0, so the gradient is -b and g(lam) = -lam.b
    empty = dataclasses.replace(inst, n_users=0, row_ptr=np.zeros(1, dtype=np.int64),
                                item_idx=np.zeros(0, dtype=np.int32), c=np.zeros(0, dtype=np.float32))
    pe = make(dl, empty)
    g, grad, _ = pe.dual_grad(torch.from_numpy(lam), 1e-2)
    np.testing.assert_allclose(grad.cpu().numpy(), -inst.b.reshape(-1))
    # the dual value is taken at the FP32 gather point fl32(lam)
    lam32 = lam.astype(np.float32).astype(np.float64)
    assert g == pytest.approx(-float(lam32 @ inst.b.reshape(-1)), rel=1e-12)
