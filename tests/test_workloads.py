"""The shared input generator: known-answer vectors, reproducibility, shapes."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_philox_known_answers(wl):
    # Known-answer vectors published with the Random123 library for Philox-4x32-10
    kat = [
        ([0, 0, 0, 0], [0, 0], [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]),
        ([0xffffffff] * 4, [0xffffffff] * 2, [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]),
        ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], [0xa4093822, 0x299f31d0],
         [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]),
    ]
    for ctr, key, out in kat:
        assert wl.philox4x32_10(ctr, key) == out


def test_thread_count_independent(wl):
    code = ("import workloads as w, hashlib; p = w.production(n_users=30000, n_items=2000); "
            "print(hashlib.sha1(p.row_ptr.tobytes() + p.item_idx.tobytes() + p.c.tobytes()).hexdigest())")
    outs = set()
    for t in ("1", "3", "8"):
        r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                           env=dict(os.environ, OMP_NUM_THREADS=t), check=True)
        outs.add(r.stdout.strip())
    assert len(outs) == 1


def test_tiny_plain_shape(wl):
    inst = wl.tiny_plain(seed=0)
    d = inst.degrees()
    assert inst.n_users == 10_000 and inst.n_items == 100
    assert d.min() >= 1 and d.max() <= 100
    assert abs(d.mean() - 10.0) < 0.15
    assert np.all(inst.c <= 0) and np.all(inst.c >= -1)
    assert np.allclose(inst.b, 0.5 * inst.nnz / 100)
    assert np.allclose(wl.tiny_plain(seed=0, binding=True).b, 50.0)
    for i in range(0, inst.n_users, 101):
        row = inst.item_idx[inst.row_ptr[i]:inst.row_ptr[i + 1]]
        assert np.all(np.diff(row) > 0) and row.min() >= 0 and row.max() < 100


def test_production_shape_small(wl):
    p = wl.production(n_users=50_000)
    d = p.degrees()
    # lognormal(4.2, 0.6): median e^4.2 = 66.7, mean e^(4.2+0.18) = 79.8
    assert abs(np.median(d) - 66.7) < 2.5
    assert abs(d.mean() - 79.8) < 2.0
    assert d.max() <= 2000
    w = p.meta["item_weight"]
    assert w.max() == 1.0 and np.all(p.c <= 0) and np.all(p.c >= -1)
    # c_ij = -U * w_j
    assert np.all(-p.c <= w[p.item_idx] * (1 + 1e-7))
    n = p.item_counts()
    np.testing.assert_allclose(p.b[0], 0.3 * n)
    # the most popular item by weight is the most frequently eligible one
    assert np.argmax(n) == np.argmax(w)


def test_two_family_and_batch(wl):
    f = wl.two_family()
    assert f.a.shape == (2, f.nnz) and np.all(f.a[1] == 1.0) and f.proj == "box"
    np.testing.assert_allclose(f.b[1], 0.3 * f.item_counts())
    m = wl.batch_member(0, scale=0.05)
    assert 100 <= m.n_items <= 5000 and m.degrees().max() <= m.n_items


def test_oracle_and_library_are_independent():
    """The oracle and the GPU package share no code and never import each other."""
    pkg = os.path.join(ROOT, "paper_2606_07777_amd")
    orc = os.path.join(ROOT, "oracle")
    for d, banned in ((pkg, r"\boracle\b"), (orc, r"paper_2606_07777_amd|dualip\.h|csrc")):
        if not os.path.isdir(d):
            continue
        for dp, _, fs in os.walk(d):
            for f in fs:
                if f.endswith((".py", ".c", ".h", ".hip", ".cpp")):
                    txt = open(os.path.join(dp, f), errors="ignore").read()
                    code = "\n".join(l for l in txt.splitlines()
                                     if l.strip().startswith(("import", "from", "#include")))
                    assert not re.search(banned, code), os.path.join(dp, f)


def test_appendix_a_construction(wl):
    """The Appendix-A recipe, checked against its own definition: per-item counts,
    a = s_j * value with one scale per item, the value cap, and capacities
    b = rho (greedy load + eps) with rho in [0.5, 1] and the greedy load
    recomputed here from the rows."""
    inst = wl.appendix_a(seed=7, n_users=20_000, n_items=300, nu=12.0, c_max=6.0, eps0=1e-3)
    assert inst.n_families == 1 and inst.a.shape == (1, inst.nnz)
    assert np.array_equal(inst.item_counts(), inst.meta["item_counts"])
    assert abs(inst.nnz / inst.n_users - 12.0) < 0.5
    for i in range(0, inst.n_users, 97):
        row = inst.item_idx[inst.row_ptr[i]:inst.row_ptr[i + 1]]
        assert np.all(np.diff(row) > 0)
    val = -inst.c.astype(np.float64)
    assert np.all(val > 0) and val.max() <= 6.0 and np.any(val == np.float32(6.0))
    ratio = inst.a[0].astype(np.float64) / val
    for j in range(0, 300, 7):
        r = ratio[inst.item_idx == j]
        if r.size:
            assert np.allclose(r, r[0], rtol=1e-6), j
    load = np.zeros(300)
    a = inst.a[0]
    for i in range(inst.n_users):
        s, e = inst.row_ptr[i], inst.row_ptr[i + 1]
        if e > s:
            k = s + int(np.argmax(a[s:e]))
            load[inst.item_idx[k]] += float(a[k])
    rho = inst.b[0] / (load + 1e-3)
    assert np.all(rho >= 0.5 - 1e-12) and np.all(rho <= 1.0 + 1e-12)
    assert rho.std() > 0.1  # drawn, not constant


def test_appendix_a_thread_count_independent(wl):
    code = ("import workloads as w, hashlib; p = w.appendix_a(seed=1, n_users=30000, n_items=500); "
            "print(hashlib.sha1(p.row_ptr.tobytes() + p.item_idx.tobytes() + p.c.tobytes() + p.a.tobytes()"
            " + p.b.tobytes()).hexdigest())")
    outs = set()
    for t in ("1", "4"):
        r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                           env=dict(os.environ, OMP_NUM_THREADS=t), check=True)
        outs.add(r.stdout.strip())
    assert len(outs) == 1
