"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on
the same seeded inputs.

Tolerances follow from the arithmetic of the FP32 path.  The GPU forms
v = (c + sum_k a_k mu_k) * (-1/gamma) in FP32 (relative error <= 3 u, u = 2^-24)
and the threshold theta from FP32 sums over one row, so per element
|x_gpu - x_fp64| <= 32 u max_i|v| for the user's row (a generous multiple of the
few roundings involved).  Each a_k x is then rounded to a fixed-point grid of
step 1/qscale_k (<= 2^-30 for a <= 1, z = 1) and summed exactly in 64-bit
integers, so (A x)_j carries at most sum_i |a_ij| (32 u max|v| + 1/qscale)
error.  Both sides evaluate at the same point mu = fl32(lambda).
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


@pytest.fixture(scope="module")
def dl():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2606_07777_amd as dl
    dl.load()
    return dl


def _cases(wl):
    return {
        "tiny_plain_binding": (wl.tiny_plain(seed=0, binding=True), 1e-2),
        "all_buckets_long_rows": (wl.random_small(51, 3000, 3500, 3000, b_scale=0.2), 5e-2),
        "two_family_box": (wl.random_small(52, 5000, 300, 200, n_families=2, a_ones=False, proj="box"), 2e-2),
        "simplex_eq": (wl.random_small(53, 4000, 200, 150, proj="simplex_eq"), 1e-2),
        "explicit_a": (wl.random_small(54, 4000, 500, 300, a_ones=False), 1e-2),
        "production_small": (wl.production(n_users=100_000, n_items=10_000), 1e-2),
        "appendix_a": (wl.appendix_a(seed=3, n_users=20_000, n_items=300, nu=12.0), 1.0),
        "boxcut": (wl.random_small(55, 6000, 400, 300, proj="boxcut", radius=1.0, upper=0.3, b_scale=0.2), 1e-2),
        "boxcut_long_rows": (wl.random_small(56, 3000, 3500, 3000, proj="boxcut", radius=2.0, upper=0.25,
                                             b_scale=0.2), 5e-2),
        # the four-family kernel: three stored families, and four with family 0 at a == 1
        "three_family_box": (wl.random_small(58, 4000, 200, 100, n_families=3, a_ones=False, proj="box"), 2e-2),
        "four_family_simplex": (wl.random_small(59, 4000, 150, 80, n_families=4, a_ones=True, b_scale=0.02), 1e-2),
    }


CASE_NAMES = ["tiny_plain_binding", "all_buckets_long_rows", "two_family_box", "simplex_eq", "explicit_a",
              "production_small", "appendix_a", "boxcut", "boxcut_long_rows", "three_family_box",
              "four_family_simplex"]


@pytest.fixture(scope="module")
def cases(wl):
    return _cases(wl)


def _lam_point(orc, inst, gamma, seed):
    """A realistic dual point: 40 oracle iterations from 0, plus noise."""
    lam, _, _, _ = orc.solve(inst, [gamma], [40], jacobi=True, check_every=0)
    rng = np.random.default_rng(seed)
    return np.maximum(0.0, lam * (1 + 0.1 * rng.normal(size=lam.size)) + 0.01 * rng.uniform(size=lam.size))


def _lam_close(lg, lo, tol=1e-5, what=""):
    """lam from the GPU against the oracle's: relative l2 distance <= tol and every
    coordinate within tol * max|lam_oracle| (both norm-wise and element-wise)."""
    lg, lo = np.asarray(lg, dtype=np.float64), np.asarray(lo, dtype=np.float64)
    scale = max(np.abs(lo).max(), 1e-300)
    rel = np.linalg.norm(lg - lo) / max(np.linalg.norm(lo), 1e-300)
    el = np.abs(lg - lo).max() / scale
    print(f"{what}: |lam| {np.linalg.norm(lo):.3e} rel l2 {rel:.2e} max elementwise {el:.2e} (of max|lam|)")
    assert rel <= tol, (what, rel)
    assert el <= tol, (what, el)
    return rel


def _item_bound(inst, prob, lam32, gamma):
    """Per coupling row (k, j): the bound on |(A x)_gpu - (A x)_fp64| of the module
    docstring, sum_i |a_kij| (32 u max(1, max_row|v|) + 1/qscale_k)."""
    vmax_row, _ = _row_vmax(inst, lam32, gamma)
    xtol = 32 * U32 * np.maximum(np.repeat(vmax_row, inst.degrees()), 1.0)
    a = inst.a_dense().astype(np.float64)
    qs = np.array(prob.info()["qscale"], dtype=np.float64)
    return np.concatenate([np.bincount(inst.item_idx, weights=np.abs(a[k]) * (xtol + 1.0 / qs[k]),
                                       minlength=inst.n_items) for k in range(inst.n_families)])


def _cert_close(cg, co, inst, prob, lam32, gamma):
    """GPU certificate against the oracle's at the same FP32 point and gamma.
    Dual and primal values: relative 2e-6 (FP32 per-element terms summed in FP64,
    as for the dual value of a gradient pass) and 4e-6 (the repair factor is
    rounded to FP32 once more).  The relative gap is their difference over
    max(1, |g|).  Slack and Lagrangian gap follow from the per-row bound on A x."""
    g, P = co["dual_obj"], co["primal_obj"]
    tg, tp = 2e-6 * max(1.0, abs(g)), 4e-6 * max(1.0, abs(P))
    bnd = _item_bound(inst, prob, lam32, gamma)
    print(f"certificate: dual {cg['dual_obj']:.9g} vs {g:.9g}; primal {cg['primal_obj']:.9g} vs {P:.9g}; "
          f"gap {cg['rel_gap']:.4e} vs {co['rel_gap']:.4e}; slack {cg['max_slack']:.4e} vs {co['max_slack']:.4e}; "
          f"lagr {cg['lagr_gap']:.6g} vs {co['lagr_gap']:.6g}")
    assert abs(cg["dual_obj"] - g) <= tg
    assert abs(cg["primal_obj"] - P) <= tp
    if np.isnan(co["rel_gap"]):
        assert np.isnan(cg["rel_gap"])
    else:
        assert abs(cg["rel_gap"] - co["rel_gap"]) <= (tg + tp) / max(1.0, abs(g))
    assert abs(cg["max_slack"] - co["max_slack"]) <= bnd.max() + 1e-12
    assert abs(cg["lagr_gap"] - co["lagr_gap"]) <= float(np.abs(lam32) @ bnd) + 1e-12


def _row_vmax(inst, lam32, gamma):
    """max_e |v_e| per row, in FP64, for the error bounds."""
    a = inst.a_dense().astype(np.float64)
    s = np.zeros(inst.nnz)
    for k in range(inst.n_families):
        s += a[k] * lam32[k * inst.n_items + inst.item_idx]
    v = np.abs(inst.c.astype(np.float64) + s) / gamma
    assert np.all(np.diff(inst.row_ptr) > 0), "parity instances have no empty rows"
    return np.maximum.reduceat(v, inst.row_ptr[:-1]), v


@pytest.mark.parametrize("layout", ["bucketed", "wavefront"])
@pytest.mark.parametrize("name", CASE_NAMES)
def test_dual_grad_matches_oracle(dl, orc, cases, name, layout):
    import torch
    inst, gamma = cases[name]
    prob = dl.Problem.from_instance(inst, jacobi=True, layout=layout)
    if layout == "wavefront":
        assert all(g in (6, 7) for g in prob.info()["bucket_glog"][:prob.info()["n_buckets"]])
    lam = _lam_point(orc, inst, gamma, 1)
    lam32 = lam.astype(np.float32).astype(np.float64)
    g, grad, x = prob.dual_grad(torch.from_numpy(lam), gamma, want_obj=True, want_x=True)
    grad, x = grad.cpu().numpy(), x.cpu().numpy()
    go, grad_o, x_o, ax_o = orc.dual_grad(inst, lam32, gamma)
    deg = inst.degrees()
    vmax_row, _ = _row_vmax(inst, lam32, gamma)
    vmax_el = np.repeat(vmax_row, deg)
    xerr = np.abs(x - x_o)
    xtol = 32 * U32 * np.maximum(vmax_el, 1.0)
    assert np.all(xerr <= xtol), f"x err {xerr.max():.3e} (worst ratio {(xerr / xtol).max():.2f})"
    a = inst.a_dense().astype(np.float64)
    qs = np.array(prob.info()["qscale"], dtype=np.float64)
    for k in range(inst.n_families):
        J = inst.n_items
        bound = np.bincount(inst.item_idx, weights=np.abs(a[k]) * (xtol + 1.0 / qs[k]), minlength=J)
        err = np.abs(grad[k * J:(k + 1) * J] - grad_o[k * J:(k + 1) * J])
        assert np.all(err <= bound + 1e-12), f"family {k}: grad err {err.max():.3e}"
    # norm-wise sanity on top of the elementwise bounds above (rows of up to 3000
    # FP32 terms reach a few 1e-6)
    rel = np.linalg.norm(grad - grad_o) / max(np.linalg.norm(ax_o), 1e-30)
    assert rel <= 1e-5, rel
    assert abs(g - go) <= 2e-6 * max(1.0, abs(go)), (g, go)
    print(f"{name}: nnz {inst.nnz} x err {xerr.max():.2e} grad rel {rel:.2e} dual rel {abs(g - go) / abs(go):.2e}")


@pytest.mark.parametrize("name", ["tiny_plain_binding", "all_buckets_long_rows", "simplex_eq", "two_family_box",
                                  "boxcut", "boxcut_long_rows", "four_family_simplex"])
def test_project_matches_oracle(dl, orc, cases, name):
    import torch
    inst, _ = cases[name]
    prob = dl.Problem.from_instance(inst)
    rng = np.random.default_rng(7)
    v = (rng.normal(size=inst.nnz) * 3).astype(np.float32)
    x = prob.project(torch.from_numpy(v)).cpu().numpy()
    xo = orc.project_rows(inst, v.astype(np.float64))
    vmax = np.maximum.reduceat(np.abs(v.astype(np.float64)), inst.row_ptr[:-1])
    tol = 32 * U32 * np.maximum(np.repeat(vmax, inst.degrees()), 1.0)
    assert np.all(np.abs(x - xo) <= tol), np.abs(x - xo).max()


@pytest.mark.parametrize("name", ["tiny_plain_binding", "two_family_box", "boxcut", "all_buckets_long_rows",
                                  "three_family_box"])
def test_certificate_matches_oracle(dl, orc, cases, name):
    """The certificate (dual value, repaired primal value, relative gap, max slack,
    Lagrangian gap) at a fixed point lam, against the oracle's at the same FP32
    point: simplex <=, box with two stored families, box-cut."""
    import torch
    inst, gamma = cases[name]
    prob = dl.Problem.from_instance(inst, jacobi=True)
    lam32 = _lam_point(orc, inst, gamma, 5).astype(np.float32).astype(np.float64)
    s = prob.solver(torch.from_numpy(lam32))
    s.set_stage(gamma, 1.0, True)
    cg = s.certificate()
    co = orc.certificate(inst, lam32, gamma)
    assert cg["gamma"] == gamma
    _cert_close(cg, co, inst, prob, lam32, gamma)


def _ladder_instance(wl, proj, radius=1.0, upper=0.0, seed=0):
    """Users of every degree class the kernel distinguishes (one lane per user up
    to a wavefront loop over rows longer than 64 * KMAX), at and next to each
    class boundary, 70 users per degree so tasks come full and partial."""
    rng = np.random.default_rng(seed)
    J = 4000
    degs = [1, 2, 3, 4, 5, 7, 8, 9, 11, 12, 13, 16, 17, 23, 24, 25, 31, 47, 48, 49, 64, 95, 96, 97, 190, 191,
            192, 193, 383, 384, 385, 700, 767, 768, 769, 770, 1000, 1536, 3000, 4000]
    rows = [d for d in degs for _ in range(70)]
    rng.shuffle(rows)
    rp = np.zeros(len(rows) + 1, dtype=np.int64)
    rp[1:] = np.cumsum(rows)
    idx = np.concatenate([np.sort(rng.choice(J, d, replace=False)) for d in rows]).astype(np.int32)
    c = -rng.uniform(size=idx.size).astype(np.float32)
    b = np.full((1, J), 5.0)
    return wl.Instance(f"ladder_{proj}", len(rows), J, 1, rp, idx, c, None, b, proj, radius, {}, upper)


def _adversarial_v(inst, z, seed):
    """Per row, one of ten patterns (by row index): ties (constant rows, both
    fitting and not fitting), a positive part summing to z exactly, a leader
    exactly z above the second entry (the one-leader exit boundary), all entries
    <= 0, magnitudes spread over 1e-6 .. 1e6, many ties at the threshold, plain
    normal, a third entry exactly at the two leaders' threshold (the two-leader
    exit boundary, z = 1), and three leaders over a tail of ties just below
    their threshold (the Newton path, z = 1)."""
    rng = np.random.default_rng(seed)
    v = np.empty(inst.nnz, dtype=np.float32)
    for i in range(inst.n_users):
        s, e = int(inst.row_ptr[i]), int(inst.row_ptr[i + 1])
        d = e - s
        kind = i % 10
        if kind == 0:
            r = np.full(d, np.float32(2.0 * z / d + 0.125))        # constant, sum > z
        elif kind == 1:
            r = np.full(d, np.float32(0.5 * z / d))                # constant, fits
        elif kind == 2:
            r = -rng.uniform(0.1, 3.0, size=d)                     # positive part = z exactly
            r[0] = z * 0.5
            if d > 1:
                r[1] = z * 0.25
                if d > 2:
                    r[2] = z * 0.25
                else:
                    r[0] = z * 0.75
            else:
                r[0] = z
        elif kind == 3:
            r = rng.uniform(-1.0, 0.25, size=d)                     # leader exactly z above the second
            r[rng.integers(d)] = 0.25 + z if d > 1 else 0.25 + z
            if d > 1:
                j = int(np.argmax(r))
                k = (j + 1) % d
                r[k] = 0.25
        elif kind == 4:
            r = -rng.exponential(size=d)                           # all <= 0
            r[rng.integers(d)] = 0.0
        elif kind == 5:
            r = rng.choice([-1.0, 1.0], size=d) * 10.0 ** rng.uniform(-6, 6, size=d)
        elif kind == 6:
            r = np.full(d, 0.75)                                   # ties at the threshold plus a tail
            r[: max(1, d // 3)] = 1.5
        elif kind == 8:
            r = rng.uniform(-1.0, 0.2, size=d)                     # m3 = (m1 + m2 - z) / 2 exactly
            r[:3] = [1.0, 0.5, 0.25][:d]
            rng.shuffle(r)
        elif kind == 9:
            r = np.full(d, 0.40625)                                # ties just below (m1+m2+m3-z)/3
            r[:3] = [1.0, 0.75, 0.5][:d]
            rng.shuffle(r)
        else:
            r = rng.normal(size=d) * 2
        v[s:e] = r
    return v


@pytest.mark.parametrize("proj", ["simplex_le", "simplex_eq", "box", "boxcut"])
def test_project_adversarial_rows(dl, orc, wl, proj):
    """ProjectionMap on adversarial rows in every degree class and kind, against
    the oracle's sort-based (simplex), clamp (box) and breakpoint (box-cut)
    projections; per element within 32 u max(1, max_row |v|)."""
    import torch
    z = 1.0
    inst = _ladder_instance(wl, proj, radius=z, upper=0.3 if proj == "boxcut" else 0.0, seed=11)
    prob = dl.Problem.from_instance(inst)
    glogs = prob.info()["bucket_glog"][:prob.info()["n_buckets"]]
    assert set(glogs) == {0, 1, 2, 3, 4, 5, 6, 7}, glogs
    v = _adversarial_v(inst, z, 3)
    x = prob.project(torch.from_numpy(v)).cpu().numpy().astype(np.float64)
    xo = orc.project_rows(inst, v.astype(np.float64))
    vmax = np.maximum.reduceat(np.abs(v.astype(np.float64)), inst.row_ptr[:-1])
    tol = 32 * U32 * np.maximum(np.repeat(vmax, inst.degrees()), 1.0)
    err = np.abs(x - xo)
    kinds = np.repeat(np.arange(inst.n_users) % 10, inst.degrees())
    for kd in range(10):
        m = kinds == kd
        print(f"{proj} pattern {kd}: max err {err[m].max():.2e}, worst err/tol {(err[m] / tol[m]).max():.3f}")
    assert np.all(err <= tol), float((err / tol).max())
    # the sets' constraints hold on the GPU side as well, up to the row's summed
    # element tolerance (a row of d entries carries d roundings of theta)
    sums = np.add.reduceat(x, inst.row_ptr[:-1])
    row_tol = np.add.reduceat(tol, inst.row_ptr[:-1])
    assert np.all(x >= 0)
    if proj in ("simplex_le", "boxcut"):
        assert np.all(sums <= z + row_tol)
    if proj == "simplex_eq":
        assert np.all(np.abs(sums - z) <= row_tol)
    if proj in ("box", "boxcut"):
        assert np.all(x <= (z if proj == "box" else 0.3) * (1 + 1e-6))


def test_trajectory_tiny_plain_binding(dl, orc, cases):
    """200 iterations at gamma = 1e-2 with step 1/L from the row-norm bound, no Jacobi."""
    import torch
    inst, gamma = cases["tiny_plain_binding"]
    prob = dl.Problem.from_instance(inst, jacobi=False)
    s = prob.solver()
    s.set_stage(gamma, 1.0, True)
    lam_gpu = {}
    done = 0
    for k in (50, 100, 200):
        s.step(k - done)
        done = k
        lam_gpu[k] = s.lam().cpu().numpy()
    _, _, snaps, _ = orc.solve(inst, [gamma], [200], jacobi=False, check_every=0, snap_iters=[50, 100, 200])
    for i, k in enumerate((50, 100, 200)):
        _lam_close(lam_gpu[k], snaps[i], what=f"iteration {k}")


def test_trajectory_production_prefix(dl, orc, cases):
    """The production shape (Zipf items, lognormal degrees, Jacobi) over the start
    of its continuation schedule: lam after 50 iterations at gamma 0.1 and 50
    more at 0.01 within 1e-5 of the FP64 oracle."""
    inst, _ = cases["production_small"]
    prob = dl.Problem.from_instance(inst, jacobi=True)
    s = prob.solver()
    out = []
    for g in (1e-1, 1e-2):
        s.set_stage(g, 1.0, True)
        s.step(50)
        out.append(s.lam().cpu().numpy())
    _, _, snaps, _ = orc.solve(inst, [1e-1, 1e-2], [50, 50], jacobi=True, check_every=0, snap_iters=[50, 100])
    for k, (lg, lo) in enumerate(zip(out, snaps)):
        _lam_close(lg, lo, what=f"production prefix, iteration {50 * (k + 1)}")


def test_literal_capacities_stay_slack(dl, orc, wl):
    import torch
    inst = wl.tiny_plain(seed=0, binding=False)
    prob = dl.Problem.from_instance(inst, jacobi=False)
    lam, st = prob.solve([1e-2], [200], check_every=0)
    assert torch.all(lam == 0).item()
    _, _, x = prob.dual_grad(lam, 1e-2, want_obj=False, want_x=True)
    xo = orc.project_rows(inst, -inst.c.astype(np.float64) / 1e-2)
    assert np.abs(x.cpu().numpy() - xo).max() <= 32 * U32 * 100


def test_continuation_solve_matches_oracle(dl, orc, wl):
    inst = wl.tiny_plain(seed=1, binding=True, n_users=20_000, n_items=200)
    prob = dl.Problem.from_instance(inst, jacobi=True)
    sched = dict(gammas=[1e-1, 1e-2, 1e-3], iters=[300, 300, -1])
    lam, st = prob.solve(**sched, tol=1e-4, max_iters=20000, check_every=10)
    lo, so, _, _ = orc.solve(inst, sched["gammas"], sched["iters"], tol=1e-4, max_iters=20000, check_every=10,
                             jacobi=True)
    print(f"gpu iters {st['iters']} gap {st['rel_gap']:.2e}; oracle iters {so['iters']} gap {so['rel_gap']:.2e}")
    assert st["status"] == 0 and so["status"] == 0
    assert st["rel_gap"] <= 1e-4
    # the same trajectory crosses the tolerance at the same check point
    assert st["iters"] == so["iters"]
    _lam_close(lam.cpu().numpy(), lo, what="continuation solve")
    # the certificate of the final point: dual and primal values, gap, slack
    _cert_close(st, so, inst, prob, lo.astype(np.float32).astype(np.float64), 1e-3)


@pytest.mark.parametrize("name", ["two_family_box", "three_family_box", "four_family_simplex"])
def test_multi_family_trajectory(dl, orc, cases, name):
    """gamma 0.1 -> 0.01, 150 iterations each, Jacobi: the two-family kernel (two
    tasks' rows in flight per wavefront) and the four-family kernel against the oracle."""
    inst, _ = cases[name]
    prob = dl.Problem.from_instance(inst, jacobi=True)
    sched = dict(gammas=[1e-1, 1e-2], iters=[150, 150])
    lam, _ = prob.solve(**sched, check_every=0)
    lo, _, _, _ = orc.solve(inst, sched["gammas"], sched["iters"], jacobi=True, check_every=0)
    assert np.linalg.norm(lo) > 0
    _lam_close(lam.cpu().numpy(), lo, what=f"{name} trajectory")


@pytest.mark.parametrize("gamma", [10.0, 1e3])
def test_dual_objective_at_large_gamma(dl, orc, cases, gamma):
    """Regression: the objective terms of padding lanes (v = -inf) must not be
    formed; at gamma > 1 they overflowed to inf * 0 = NaN."""
    import torch
    for name in ("tiny_plain_binding", "appendix_a"):
        inst, _ = cases[name]
        prob = dl.Problem.from_instance(inst, jacobi=True)
        lam = _lam_point(orc, inst, gamma, 3)
        lam32 = lam.astype(np.float32).astype(np.float64)
        g, grad, _ = prob.dual_grad(torch.from_numpy(lam), gamma)
        go, grad_o, _, ax_o = orc.dual_grad(inst, lam32, gamma)
        assert np.isfinite(g), name
        assert abs(g - go) <= 2e-6 * max(1.0, abs(go)), (name, g, go)
        s = prob.solver(torch.from_numpy(lam))
        s.set_stage(gamma, 1.0, True)
        c = s.certificate()
        assert np.isfinite(c["dual_obj"]) and np.isfinite(c["primal_obj"]), (name, c)


def test_appendix_a_six_stage_schedule(dl, orc, wl):
    """The paper's six-stage schedule (gamma 1e3 ... 1e-2, Table 4) on the
    Appendix-A construction, shortened to 100 iterations per stage: lam after
    every stage against the FP64 oracle, from the same warm starts."""
    import torch
    inst = wl.appendix_a(seed=4, n_users=20_000, n_items=300, nu=12.0)
    gammas = [1e3, 1e2, 1e1, 1e0, 1e-1, 1e-2]
    prob = dl.Problem.from_instance(inst, jacobi=True)
    s = prob.solver()
    lam_o = None
    for g in gammas:
        s.set_stage(g, 1.0, True)
        s.step(100)
        lo, so, _, _ = orc.solve(inst, [g], [100], jacobi=True, check_every=0, lam0=lam_o)
        lg = s.lam().cpu().numpy()
        _lam_close(lg, lo, what=f"gamma {g:g}")
        # continue both from the oracle's point so stage errors do not compound
        lam_o = lo
        s = prob.solver(torch.from_numpy(lo))
    # certificate of the final point at the final gamma, against the oracle's at the
    # same FP32 point
    s.set_stage(gammas[-1], 1.0, True)
    cert = s.certificate()
    co = orc.certificate(inst, lam_o.astype(np.float32).astype(np.float64), gammas[-1])
    print(f"certificate after the schedule: gpu {cert}; oracle {co}")
    assert cert["gamma"] == gammas[-1]
    _cert_close(cert, co, inst, prob, lam_o.astype(np.float32).astype(np.float64), gammas[-1])


def test_boxcut_continuation_solve_matches_oracle(dl, orc, wl):
    inst = wl.random_small(57, 20_000, 200, 60, proj="boxcut", radius=1.0, upper=0.35, b_scale=0.02)
    prob = dl.Problem.from_instance(inst, jacobi=True)
    sched = dict(gammas=[1e-1, 1e-2], iters=[200, 200])
    lam, _ = prob.solve(**sched, check_every=0)
    lo, _, _, _ = orc.solve(inst, sched["gammas"], sched["iters"], jacobi=True, check_every=0)
    assert np.linalg.norm(lo) > 0
    _lam_close(lam.cpu().numpy(), lo, what="box-cut trajectory")
    s = prob.solver(lam)
    s.set_stage(1e-2, 1.0, True)
    c = s.certificate()
    assert np.isfinite(c["rel_gap"]) and c["rel_gap"] >= -1e-6


def test_equality_family_free_duals(dl, orc, wl):
    """Family 1 as equality rows (free duals) next to capacity rows: the GPU
    trajectory against the oracle, duals of both signs, NaN certified gap and
    |Ax - b| slack."""
    import dataclasses
    import torch
    base = wl.random_small(26, 20_000, 200, 30, n_families=2, a_ones=False, b_scale=0.2)
    inst = dataclasses.replace(base, eq_families=0b10)
    x0 = np.zeros(inst.nnz)
    deg = np.diff(inst.row_ptr)
    x0 = np.repeat(0.97 / np.maximum(deg, 1), deg)  # near-full targets: some rows under-demanded
    b = inst.b.copy()
    b[1] = np.bincount(inst.item_idx, weights=inst.a[1].astype(np.float64) * x0, minlength=inst.n_items)
    inst = dataclasses.replace(inst, b=b)
    prob = dl.Problem.from_instance(inst, jacobi=True)
    lam, st = prob.solve([1e-1, 1e-2], [200, 200], check_every=0)
    lo, so, _, _ = orc.solve(inst, [1e-1, 1e-2], [200, 200], jacobi=True, check_every=0)
    lam = lam.cpu().numpy()
    J = inst.n_items
    print(f"equality family: lam_eq min {lo[J:].min():.3e} max {lo[J:].max():.3e}")
    _lam_close(lam, lo, what="equality family")
    assert (lo[J:] < 0).any() and (lam[:J] >= 0).all()
    assert np.isnan(st["rel_gap"]) and np.isnan(so["rel_gap"])
    assert abs(st["max_slack"] - so["max_slack"]) <= 1e-4 * max(1.0, so["max_slack"])


def test_halving_continuation_matches_oracle(dl, orc, wl):
    """The decay of the continuation ablation (gamma 0.16 -> 0.01, halved every
    25 iterations, momentum reset, step scaled with gamma), no Jacobi and with
    Jacobi, against the FP64 oracle run with the same schedule."""
    inst = wl.appendix_a(seed=6, n_users=20_000, n_items=300, nu=10.0)
    sched = dict(gammas=[0.16, 0.08, 0.04, 0.02, 0.01], iters=[25, 25, 25, 25, 50])
    for jac in (True, False):
        prob = dl.Problem.from_instance(inst, jacobi=jac)
        lam, _ = prob.solve(**sched, check_every=0)
        lo, _, _, _ = orc.solve(inst, sched["gammas"], sched["iters"], jacobi=jac, check_every=0)
        _lam_close(lam.cpu().numpy(), lo, what=f"halving, jacobi {jac}")


@pytest.mark.parametrize("variant", ["two_family_bf16", "stored_a_f32", "boxcut_equality", "four_family"])
def test_batch_kernel_variants_match_solo(dl, wl, variant):
    """The batched kernels of the other variants (two-family kernel with BF16,
    one stored family, box-cut with an equality family, the four-family kernel):
    every member ends bitwise where its solo run ends."""
    import dataclasses
    if variant == "two_family_bf16":
        members = [wl.random_small(300 + k, 3000 + 700 * k, 120, 40, n_families=2, a_ones=False, proj="box")
                   for k in range(3)]
        kw = dict(storage="bf16")
    elif variant == "stored_a_f32":
        members = [wl.random_small(310 + k, 2500 + 900 * k, 150, 60, a_ones=False) for k in range(3)]
        kw = {}
    elif variant == "four_family":
        members = [wl.random_small(330 + k, 2500 + 600 * k, 90, 40, n_families=4, a_ones=True, proj="box")
                   for k in range(3)]
        kw = {}
    else:
        members = []
        for k in range(3):
            m = wl.random_small(320 + k, 3000 + 500 * k, 100, 30, n_families=2, proj="boxcut", radius=1.0,
                                upper=0.4, a_ones=False, b_scale=0.05)
            deg = np.diff(m.row_ptr)
            x0 = np.repeat(0.9 / np.maximum(deg, 1), deg)
            b = m.b.copy()
            b[1] = np.bincount(m.item_idx, weights=m.a[1].astype(np.float64) * x0, minlength=m.n_items)
            members.append(dataclasses.replace(m, b=b, eq_families=0b10))
        kw = {}
    sched = dict(gammas=[1e-1, 1e-2], iters=[60, 60], check_every=0)
    probs = [dl.Problem.from_instance(m, jacobi=True, **kw) for m in members]
    lam_b, st_b = dl.Batch(probs).solve(**sched)
    for k, p in enumerate(probs):
        lam_s, st_s = p.solve(**sched)
        assert st_b[k]["iters"] == st_s["iters"] == 120
        assert np.array_equal(lam_b[k].cpu().numpy(), lam_s.cpu().numpy()), (variant, k)


@pytest.mark.parametrize("name,jacobi", [("tiny_plain_binding", False), ("production_small", True)])
def test_bf16_trajectory_within_1e3_of_fp64(dl, orc, cases, name, jacobi):
    """BF16 storage against the FP64 oracle on the original (unrounded) data:
    lam after 200 iterations within 1e-3 relative.  Rounding the data alone moves
    lam by 6.7e-4 (tiny binding) and 1.2e-4 (production shape) on these inputs;
    the two-family instance with lognormal a is covered by the rounded-data
    comparison instead (its data distance is 1.3e-3)."""
    inst, gamma = cases[name]
    prob = dl.Problem.from_instance(inst, storage="bf16", jacobi=jacobi)
    s = prob.solver()
    s.set_stage(gamma, 1.0, True)
    s.step(200)
    lam = s.lam().cpu().numpy()
    lo, _, _, _ = orc.solve(inst, [gamma], [200], jacobi=jacobi, check_every=0)
    rel = np.linalg.norm(lam - lo) / np.linalg.norm(lo)
    print(f"{name}: BF16 lam vs FP64 oracle on the original data: {rel:.2e}")
    assert rel <= 1e-3


def test_checkpoint_resume_is_bitwise(dl, cases):
    """Export after 70 iterations, resume in a fresh solver on a fresh problem of
    the same data, continue; equals the uninterrupted run bitwise (also across a
    stage switch after the resume)."""
    inst, gamma = cases["production_small"]
    p1 = dl.Problem.from_instance(inst, jacobi=True)
    a = p1.solver()
    a.set_stage(1e-1, 1.0, True)
    a.step(70)
    state, meta = a.export_state()
    state = state.clone()
    a.step(30)
    a.set_stage(1e-2, 1.0, True)
    a.step(40)
    ref = a.lam().cpu().numpy()
    p2 = dl.Problem.from_instance(inst, jacobi=True)
    b = p2.solver()
    b.import_state(state, meta)
    b.step(30)
    b.set_stage(1e-2, 1.0, True)
    b.step(40)
    assert np.array_equal(b.lam().cpu().numpy(), ref)
    bad = dict(meta, m_times_j=meta["m_times_j"] + 1)
    with pytest.raises(RuntimeError):
        b.import_state(state, bad)


def test_bitwise_deterministic(dl, cases):
    inst, gamma = cases["production_small"]
    out = []
    for _ in range(2):
        prob = dl.Problem.from_instance(inst, jacobi=True)
        lam, _ = prob.solve([1e-1, 1e-2], [30, 30], check_every=0)
        out.append(lam.cpu().numpy())
    assert np.array_equal(out[0], out[1])


def test_split_equals_uninterrupted(dl, cases):
    inst, gamma = cases["tiny_plain_binding"]
    prob = dl.Problem.from_instance(inst, jacobi=True)
    a = prob.solver()
    a.set_stage(gamma)
    a.step(60)
    b = prob.solver()
    b.set_stage(gamma)
    b.step(25)
    b.step(35)
    assert np.array_equal(a.lam().cpu().numpy(), b.lam().cpu().numpy())


# ---------------------------------------------------------------------------
# BF16 storage of c and a: FP32 arithmetic on the rounded values
# ---------------------------------------------------------------------------
def _rounded(orc, inst):
    import workloads
    a = None if inst.a is None else orc.bf16_round(inst.a)
    return workloads.Instance(inst.name + "_bf16", inst.n_users, inst.n_items, inst.n_families, inst.row_ptr,
                              inst.item_idx, orc.bf16_round(inst.c), a, inst.b, inst.proj, inst.radius)


@pytest.mark.parametrize("name", ["two_family_box", "production_small", "explicit_a", "three_family_box"])
def test_bf16_dual_grad_matches_oracle_on_rounded_data(dl, orc, cases, name):
    """With BF16 storage the GPU computes exactly the FP32 path on the RNE-rounded c and a."""
    import torch
    inst, gamma = cases[name]
    rinst = _rounded(orc, inst)
    prob = dl.Problem.from_instance(inst, storage="bf16", jacobi=True)
    lam = _lam_point(orc, rinst, gamma, 3)
    lam32 = lam.astype(np.float32).astype(np.float64)
    g, grad, x = prob.dual_grad(torch.from_numpy(lam), gamma, want_obj=True, want_x=True)
    grad, x = grad.cpu().numpy(), x.cpu().numpy()
    go, grad_o, x_o, ax_o = orc.dual_grad(rinst, lam32, gamma)
    vmax_row, _ = _row_vmax(rinst, lam32, gamma)
    xtol = 32 * U32 * np.maximum(np.repeat(vmax_row, rinst.degrees()), 1.0)
    assert np.all(np.abs(x - x_o) <= xtol)
    a = rinst.a_dense().astype(np.float64)
    qs = np.array(prob.info()["qscale"], dtype=np.float64)
    J = inst.n_items
    for k in range(inst.n_families):
        bound = np.bincount(inst.item_idx, weights=np.abs(a[k]) * (xtol + 1.0 / qs[k]), minlength=J)
        assert np.all(np.abs(grad[k * J:(k + 1) * J] - grad_o[k * J:(k + 1) * J]) <= bound + 1e-12)
    assert abs(g - go) <= 2e-6 * max(1.0, abs(go))


def test_bf16_trajectory_two_family(dl, orc, cases):
    """Fixed gamma = 1e-2, 200 iterations, Jacobi on.  FP32 storage against the FP64 oracle
    <= 1e-5; BF16 storage against the oracle on the RNE-rounded data <= 1e-5.  Against the
    original data the BF16 run may differ only by what rounding the data moves the oracle's
    own trajectory (measured here: about 1.3e-3 on this instance), plus 1e-5."""
    inst, _ = cases["two_family_box"]
    gamma = 1e-2
    rinst = _rounded(orc, inst)
    out = {}
    for storage in ("f32", "bf16"):
        prob = dl.Problem.from_instance(inst, storage=storage, jacobi=True)
        lam, _ = prob.solve([gamma], [200], check_every=0)
        out[storage] = lam.cpu().numpy()
    lo, _, _, _ = orc.solve(inst, [gamma], [200], jacobi=True, check_every=0)
    lr, _, _, _ = orc.solve(rinst, [gamma], [200], jacobi=True, check_every=0)
    rel = lambda u, w: np.linalg.norm(u - w) / np.linalg.norm(w)
    data = rel(lr, lo)
    print(f"f32 vs fp64 {rel(out['f32'], lo):.2e}; bf16 vs fp64(rounded) {rel(out['bf16'], lr):.2e}; "
          f"bf16 vs fp64(original) {rel(out['bf16'], lo):.2e}; fp64(rounded) vs fp64(original) {data:.2e}")
    assert rel(out["f32"], lo) <= 1e-5
    assert rel(out["bf16"], lr) <= 1e-5
    assert rel(out["bf16"], lo) <= data + 1e-5


# ---------------------------------------------------------------------------
# Batched form: many uneven instances per launch
# ---------------------------------------------------------------------------
def test_batch_matches_solo_solves(dl, orc, wl):
    """Each member of a batch ends bitwise where its solo solve ends (integer partial
    sums make the gradient independent of how workgroups split the tasks), after
    the same number of iterations; one member is checked against the oracle."""
    members = [wl.batch_member(k, binding=True, scale=0.02) for k in range(6)]
    sched = dict(gammas=[1e-1, 1e-2, 1e-3], iters=[100, 100, -1], tol=1e-4, max_iters=3000, check_every=10)
    probs = [dl.Problem.from_instance(m, jacobi=True) for m in members]
    lam_b, st_b = dl.Batch(probs).solve(**sched)
    for k, (m, p) in enumerate(zip(members, probs)):
        lam_s, st_s = p.solve(**sched)
        print(f"member {k}: I={m.n_users} J={m.n_items} nnz={m.nnz} iters batch {st_b[k]['iters']} "
              f"solo {st_s['iters']} gap {st_b[k]['rel_gap']:.2e}")
        assert st_b[k]["iters"] == st_s["iters"]
        assert np.array_equal(lam_b[k].cpu().numpy(), lam_s.cpu().numpy())
        _same_certificate(st_b[k], st_s)
    lo, so, _, _ = orc.solve(members[0], sched["gammas"], sched["iters"], tol=1e-4, max_iters=3000,
                             check_every=10, jacobi=True)
    assert abs(st_b[0]["dual_obj"] - so["dual_obj"]) <= 2e-4 * abs(so["dual_obj"])


def _same_certificate(a, b):
    """The batch computes a member's certificate in batched launches over its own
    workgroup split; at the same lam it matches the solo certificate up to the order
    of the per-workgroup FP64 objective sums (the A x sums are integers: slack and
    Lagrangian gap agree exactly)."""
    for key in ("dual_obj", "primal_obj"):
        assert abs(a[key] - b[key]) <= 1e-12 * max(1.0, abs(b[key])), (key, a[key], b[key])
    assert abs(a["rel_gap"] - b["rel_gap"]) <= 1e-12 or (np.isnan(a["rel_gap"]) and np.isnan(b["rel_gap"]))
    assert a["max_slack"] == b["max_slack"] and a["lagr_gap"] == b["lagr_gap"]


def test_batch_certificates_with_global_and_equality_rows(dl, wl):
    """Check points of a batch whose members carry a global-count row, an equality
    family, or neither: iteration counts, lam and certificates as in the solo solves."""
    import dataclasses
    members = []
    for k in range(3):
        m = wl.random_small(340 + k, 3000 + 800 * k, 80, 30, n_families=2, a_ones=True, b_scale=0.1)
        if k == 0:
            m = dataclasses.replace(m, global_cap=0.3 * m.n_users)
        elif k == 1:
            deg = np.diff(m.row_ptr)
            x0 = np.repeat(0.9 / np.maximum(deg, 1), deg)
            b = m.b.copy()
            b[1] = np.bincount(m.item_idx, weights=m.a[1].astype(np.float64) * x0, minlength=m.n_items)
            m = dataclasses.replace(m, b=b, eq_families=0b10)
        members.append(m)
    sched = dict(gammas=[1e-1, 1e-2], iters=[60, -1], tol=1e-4, max_iters=1500, check_every=10)
    probs = [dl.Problem.from_instance(m, jacobi=True) for m in members]
    lam_b, st_b = dl.Batch(probs).solve(**sched)
    for k, p in enumerate(probs):
        lam_s, st_s = p.solve(**sched)
        print(f"member {k}: iters batch {st_b[k]['iters']} solo {st_s['iters']} gap {st_b[k]['rel_gap']:.3e} "
              f"status {st_b[k]['status']}")
        assert st_b[k]["iters"] == st_s["iters"] and st_b[k]["status"] == st_s["status"]
        assert np.array_equal(lam_b[k].cpu().numpy(), lam_s.cpu().numpy())
        _same_certificate(st_b[k], st_s)


def test_batch_leaves_its_problems_intact(dl, wl):
    """The batch deals a small member more workgroups than its own grid has slots
    (here about 190 against 12); the certificate's per-workgroup sums must then go to
    the batch's own storage.  After a batched solve with check points, every member's
    problem still computes bitwise what a freshly created copy computes."""
    import torch
    members = [wl.random_small(350 + k, 3000 + 800 * k, 80, 30, b_scale=0.1) for k in range(3)]
    sched = dict(gammas=[1e-1, 1e-2], iters=[40, -1], tol=1e-4, max_iters=600, check_every=10)
    probs = [dl.Problem.from_instance(m, jacobi=True) for m in members]
    assert all(p.info()["n_workgroups"] < 64 for p in probs)
    dl.Batch(probs).solve(**sched)
    rng = np.random.default_rng(5)
    for m, p in zip(members, probs):
        fresh = dl.Problem.from_instance(m, jacobi=True)
        lam = torch.from_numpy(np.abs(rng.normal(size=p.nrow)) * 0.05)
        g1, grad1, x1 = p.dual_grad(lam, 1e-2, want_x=True)
        g2, grad2, x2 = fresh.dual_grad(lam, 1e-2, want_x=True)
        assert np.array_equal(grad1.cpu().numpy(), grad2.cpu().numpy())
        assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy()) and g1 == g2
        l1, s1 = p.solve(**sched)
        l2, s2 = fresh.solve(**sched)
        assert np.array_equal(l1.cpu().numpy(), l2.cpu().numpy()) and s1["iters"] == s2["iters"]
        _same_certificate(s1, s2)


def test_tuned_batch_matches_solo(dl, wl):
    """The batch tuner re-deals workgroups between and inside members from the measured
    time of the solve's own iterations (from iteration 10); every member still ends
    bitwise where its solo solve ends, and the report describes the kept split.  A
    second solve on the same batch without tuning starts again from the cost model."""
    members = [wl.batch_member(k, binding=True, scale=0.02) for k in range(6, 12)]
    sched = dict(gammas=[1e-1, 1e-2, 1e-3], iters=[100, 100, -1], tol=1e-4, max_iters=3000, check_every=10)
    probs = [dl.Problem.from_instance(m, jacobi=True) for m in members]
    batch = dl.Batch(probs)
    lam_b, st_b = batch.solve(autotune=2, **sched)
    tr = batch.tune()
    print(f"batch tune: {tr}")
    assert tr["rounds"] == 2 and tr["n_workgroups"] >= len(members)
    assert tr["pass_ms_model"] > 0 and 0 < tr["pass_ms_tuned"] <= tr["pass_ms_model"]
    assert tr["imbalance_tuned"] >= 1.0 and tr["imbalance_model"] >= 1.0
    for k, (m, p) in enumerate(zip(members, probs)):
        lam_s, st_s = p.solve(**sched)
        print(f"member {k}: I={m.n_users} nnz={m.nnz} iters batch {st_b[k]['iters']} solo {st_s['iters']}")
        assert st_b[k]["iters"] == st_s["iters"]
        assert np.array_equal(lam_b[k].cpu().numpy(), lam_s.cpu().numpy())
    lam_u, st_u = batch.solve(autotune=0, **sched)
    assert batch.tune()["rounds"] == 0
    for k in range(len(members)):
        assert np.array_equal(lam_u[k].cpu().numpy(), lam_b[k].cpu().numpy())


# ---------------------------------------------------------------------------
# Global-count coupling row (Section 5): sum over all (i, j) of x_ij <= M
# ---------------------------------------------------------------------------
def _global_cases(wl):
    import dataclasses
    out = {}
    base = wl.tiny_plain(seed=2, binding=True, n_users=8000, n_items=80)
    out["simplex"] = (dataclasses.replace(base, global_cap=0.3 * base.n_users), 1e-2)
    b2 = wl.random_small(60, 6000, 200, 150, n_families=2, a_ones=False, proj="box", b_scale=0.4)
    out["box_stored_a"] = (dataclasses.replace(b2, global_cap=0.5 * b2.nnz * 0.2), 2e-2)
    b3 = wl.random_small(61, 3000, 3500, 3000, proj="boxcut", radius=2.0, upper=0.25, b_scale=0.3)
    out["boxcut_long_rows"] = (dataclasses.replace(b3, global_cap=0.4 * b3.n_users), 5e-2)
    return out


@pytest.mark.parametrize("name", ["simplex", "box_stored_a", "boxcut_long_rows"])
def test_global_count_dual_grad_matches_oracle(dl, orc, wl, name):
    import torch
    inst, gamma = _global_cases(wl)[name]
    prob = dl.Problem.from_instance(inst, jacobi=True)
    assert prob.nrow == inst.n_families * inst.n_items + 1
    lam = _lam_point(orc, inst, gamma, 2)
    lam32 = lam.astype(np.float32).astype(np.float64)
    assert lam32[-1] > 0, "the cap binds at this point"
    g, grad, x = prob.dual_grad(torch.from_numpy(lam), gamma, want_obj=True, want_x=True)
    grad, x = grad.cpu().numpy(), x.cpu().numpy()
    go, grad_o, x_o, ax_o = orc.dual_grad(inst, lam32, gamma)
    # v carries the global dual: max|v| per row from the oracle's x-independent formula
    a = inst.a_dense().astype(np.float64)
    s = np.full(inst.nnz, lam32[-1])
    for k in range(inst.n_families):
        s += a[k] * lam32[k * inst.n_items + inst.item_idx]
    vabs = np.abs(inst.c.astype(np.float64) + s) / gamma
    vmax_el = np.repeat(np.maximum.reduceat(vabs, inst.row_ptr[:-1]), inst.degrees())
    xtol = 32 * U32 * np.maximum(vmax_el, 1.0)
    assert np.all(np.abs(x - x_o) <= xtol), float((np.abs(x - x_o) / xtol).max())
    qs = np.array(prob.info()["qscale"], dtype=np.float64)
    J, mJ = inst.n_items, inst.n_families * inst.n_items
    for k in range(inst.n_families):
        bound = np.bincount(inst.item_idx, weights=np.abs(a[k]) * (xtol + 1.0 / qs[k]), minlength=J)
        assert np.all(np.abs(grad[k * J:(k + 1) * J] - grad_o[k * J:(k + 1) * J]) <= bound + 1e-12), k
    # the global entry: sum of all x on a grid no coarser than 2^(30 - ceil log2 radius)
    qg = 2.0 ** (30 - np.ceil(np.log2(inst.radius)))
    gb = float(np.sum(xtol + 1.0 / qg))
    print(f"{name}: global grad {grad[mJ]:.6f} vs {grad_o[mJ]:.6f} (bound {gb:.2e}); dual {g:.9g} vs {go:.9g}")
    assert abs(grad[mJ] - grad_o[mJ]) <= gb
    assert abs(g - go) <= 2e-6 * max(1.0, abs(go))


@pytest.mark.parametrize("name", ["simplex", "box_stored_a"])
def test_global_count_trajectory_and_certificate(dl, orc, wl, name):
    """Continuation gamma 0.1 -> 0.01 (150 iterations each, Jacobi, the Weyl step
    bound): lam, including the global dual, within 1e-5 of the oracle; then the
    certificate (with the global repair factor) at the final point."""
    import torch
    inst, _ = _global_cases(wl)[name]
    prob = dl.Problem.from_instance(inst, jacobi=True)
    D, L = orc.scaling(inst, jacobi=True)
    assert abs(prob.info()["lhat"] - L) <= 1e-9 * L
    sched = dict(gammas=[1e-1, 1e-2], iters=[150, 150])
    lam, _ = prob.solve(**sched, check_every=0)
    lo, _, _, _ = orc.solve(inst, sched["gammas"], sched["iters"], jacobi=True, check_every=0)
    assert lo[-1] > 0
    _lam_close(lam.cpu().numpy(), lo, what=f"global-count {name}")
    lam32 = lo.astype(np.float32).astype(np.float64)
    s = prob.solver(torch.from_numpy(lam32))
    s.set_stage(1e-2, 1.0, True)
    cg = s.certificate()
    co = orc.certificate(inst, lam32, 1e-2)
    g, P = co["dual_obj"], co["primal_obj"]
    print(f"certificate: gpu {cg}; oracle {co}")
    assert abs(cg["dual_obj"] - g) <= 2e-6 * max(1.0, abs(g))
    assert abs(cg["primal_obj"] - P) <= 4e-6 * max(1.0, abs(P))
    assert abs(cg["rel_gap"] - co["rel_gap"]) <= 6e-6 * max(1.0, abs(P)) / max(1.0, abs(g))
    assert cg["rel_gap"] >= -1e-6


def test_global_count_batch_member_matches_solo(dl, wl):
    import dataclasses
    members = []
    for k in range(3):
        m = wl.tiny_plain(seed=70 + k, binding=True, n_users=3000 + 1500 * k, n_items=60)
        members.append(dataclasses.replace(m, global_cap=0.35 * m.n_users) if k != 1 else m)
    sched = dict(gammas=[1e-1, 1e-2], iters=[80, 80], check_every=0)
    probs = [dl.Problem.from_instance(m, jacobi=True) for m in members]
    lam_b, _ = dl.Batch(probs).solve(**sched)
    for k, p in enumerate(probs):
        lam_s, _ = p.solve(**sched)
        assert lam_b[k].numel() == p.nrow
        assert np.array_equal(lam_b[k].cpu().numpy(), lam_s.cpu().numpy()), k
