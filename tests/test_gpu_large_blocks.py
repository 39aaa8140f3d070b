"""Coupling blocks beyond one on-chip histogram (m * J > 13,000, Definition 1):
the gradient pass keeps every dual row in LDS and runs once per window of
histogram rows, each launch keeping the fixed-point sums of its own rows.
Parity against the FP64 oracle as for the one-window path (same error bounds),
and the limits that are refused with DL_EUNSUPPORTED.
"""
import dataclasses

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24  # FP32 unit roundoff


@pytest.fixture(scope="module")
def dl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_07777_amd as dl
    dl.load()
    return dl


def _cases(wl):
    # two families at 10,000 items (20,000 rows): a lognormal budget family and a count
    # cap, box [0, 1] (the two-family precision workload's families at the production J)
    two = wl.two_family(seed=5, n_users=150_000, n_items=10_000)
    # one family at 14,000 items: rows beyond the on-chip histogram with a == 1
    one = wl.tiny_plain(seed=6, binding=True, n_users=150_000, n_items=14_000, mean_degree=12.0)
    return {"two_family_10k": (two, 2e-2), "one_family_14k": (one, 1e-2),
            "two_family_10k_global": (dataclasses.replace(two, global_cap=0.2 * two.nnz), 2e-2),
            "two_family_10k_bf16": (two, 2e-2),
            # three stored families of 5,000 items: the four-family kernel in two windows
            "three_family_5k": (wl.random_small(9, 40_000, 5000, 30, n_families=3, a_ones=False, proj="box"), 2e-2)}


def _lam_point(orc, inst, gamma, seed):
    lam, _, _, _ = orc.solve(inst, [gamma], [30], jacobi=True, check_every=0)
    rng = np.random.default_rng(seed)
    return np.maximum(0.0, lam * (1 + 0.1 * rng.normal(size=lam.size)) + 0.01 * rng.uniform(size=lam.size))


@pytest.mark.parametrize("name", ["two_family_10k", "one_family_14k", "two_family_10k_global",
                                  "two_family_10k_bf16", "three_family_5k"])
def test_large_block_dual_grad_matches_oracle(dl, orc, wl, name):
    """BF16 storage: the oracle runs on the instance with c and a rounded to BF16,
    which is the data the GPU computes with."""
    import torch
    inst, gamma = _cases(wl)[name]
    assert inst.n_families * inst.n_items > 13_000
    bf = name.endswith("_bf16")
    prob = dl.Problem.from_instance(inst, jacobi=True, storage="bf16" if bf else "f32")
    assert prob.info()["n_windows"] == 2
    if bf:
        inst = dataclasses.replace(inst, c=orc.bf16_round(inst.c), a=orc.bf16_round(inst.a))
    lam = _lam_point(orc, inst, gamma, 4)
    lam32 = lam.astype(np.float32).astype(np.float64)
    g, grad, x = prob.dual_grad(torch.from_numpy(lam), gamma, want_obj=True, want_x=True)
    grad, x = grad.cpu().numpy(), x.cpu().numpy()
    go, grad_o, x_o, _ = orc.dual_grad(inst, lam32, gamma)
    a = inst.a_dense().astype(np.float64)
    J, mJ = inst.n_items, inst.n_families * inst.n_items
    # v = -(c + sum_k a_k mu_k)/gamma is formed in FP32: its rounding error scales with the
    # terms' magnitudes (|c| + sum_k |a_k mu_k|)/gamma, which exceed |v| where they cancel
    t = np.abs(inst.c.astype(np.float64)) + (abs(lam32[mJ]) if inst.global_cap is not None else 0.0)
    for k in range(inst.n_families):
        t += np.abs(a[k] * lam32[k * J + inst.item_idx])
    tmax = np.maximum.reduceat(t / gamma, inst.row_ptr[:-1])
    xtol = 32 * U32 * np.maximum(np.repeat(tmax, inst.degrees()), 1.0)
    assert np.all(np.abs(x - x_o) <= xtol), float((np.abs(x - x_o) / xtol).max())
    qs = np.array(prob.info()["qscale"], dtype=np.float64)
    worst = 0.0
    for k in range(inst.n_families):
        bound = np.bincount(inst.item_idx, weights=np.abs(a[k]) * (xtol + 1.0 / qs[k]), minlength=J)
        err = np.abs(grad[k * J:(k + 1) * J] - grad_o[k * J:(k + 1) * J])
        worst = max(worst, float((err / (bound + 1e-12)).max()))
        assert np.all(err <= bound + 1e-12), k
    if inst.global_cap is not None:
        gb = float(np.sum(xtol + 2.0 ** -30))
        assert abs(grad[mJ] - grad_o[mJ]) <= gb
    print(f"{name}: rows {prob.nrow}, worst grad err/bound {worst:.3f}, dual {g:.9g} vs {go:.9g}")
    assert abs(g - go) <= 2e-6 * max(1.0, abs(go))


def test_large_block_trajectory_matches_oracle(dl, orc, wl):
    """gamma 0.1 -> 0.01 (100 iterations each, Jacobi) on the two-family 10k-item instance."""
    inst, _ = _cases(wl)["two_family_10k"]
    prob = dl.Problem.from_instance(inst, jacobi=True)
    sched = dict(gammas=[1e-1, 1e-2], iters=[100, 100])
    lam, _ = prob.solve(**sched, check_every=0)
    lo, _, _, _ = orc.solve(inst, sched["gammas"], sched["iters"], jacobi=True, check_every=0)
    lam = lam.cpu().numpy()
    rel = np.linalg.norm(lam - lo) / np.linalg.norm(lo)
    el = np.abs(lam - lo).max() / np.abs(lo).max()
    print(f"large block trajectory: rel {rel:.2e}, elementwise {el:.2e}")
    assert rel <= 1e-5 and el <= 1e-5


def test_large_block_limits(dl, wl):
    import paper_2606_07777_amd as pkg
    # 16,384 items: beyond the 16-bit item offsets
    big = wl.tiny_plain(seed=7, binding=True, n_users=2000, n_items=16_384)
    with pytest.raises(pkg.DualipError) as e:
        dl.Problem.from_instance(big)
    assert e.value.status == -4
    # three families of 11,000 items: rows plus repair factors beyond one workgroup's LDS
    three = wl.random_small(8, 3000, 11_000, 20, n_families=3, a_ones=False)
    with pytest.raises(pkg.DualipError) as e:
        dl.Problem.from_instance(three)
    assert e.value.status == -4
    # batch members keep their histogram on chip
    inst, _ = _cases(wl)["one_family_14k"]
    p = dl.Problem.from_instance(inst)
    with pytest.raises(pkg.DualipError) as e:
        dl.Batch([p])
    assert e.value.status == -4
