"""Seeded synthetic matching-LP instances.

This package is the one source of inputs shared by the CPU oracle and the GPU
path.  It builds eligibility patterns and coefficient arrays only; it holds none
of the solver's arithmetic (no projection, no dual step, no scaling).

The instance families mirror the paper's matching workloads (Section 3.3 and
Definition 1: users x items, per-user simplex or box, one or more per-item
coupling families with diagonal blocks).  The paper's production data is not
public (Section 8), so every instance here is synthetic; the recipes are:

* ``tiny_plain``    10k users x 100 items, degree Poisson(10) clipped to [1,100],
                    uniform items, c = -U(0,1), a = 1, simplex sum <= 1.
* ``production``    10M users x 10k items, degree round(lognormal(4.2, 0.6))
                    clipped to [1,2000], Zipf(1.1) item popularity,
                    c = -U(0,1) * popularity weight, a = 1, b_j = 0.3 n_j.
* ``two_family``    tiny_plain pattern plus a per-item budget family
                    (a ~ lognormal(0,0.5), b = 0.2 sum_i a_ij) and a count cap
                    (a = 1, b = 0.3 n_j); box 0 <= x <= 1.
* ``batch_member``  users log-uniform in [5e4, 2e6], items log-uniform in
                    [100, 5000], degree round(lognormal(3.5, 0.8)) clipped to
                    [1, items], uniform items, c = -U(0,1), a = 1.
* ``cadence_day``   recurring daily instances: a base pattern with per-day
                    drift of c and b.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wlgen.c")
_LIB = os.path.join(_HERE, "libwlgen.so")

DEG_POISSON, DEG_LOGNORMAL, DEG_CONST = 0, 1, 2
ITEM_UNIFORM, ITEM_ZIPF = 0, 1
C_NEG_UNIFORM, C_NEG_UNIFORM_POP = 0, 1
A_ONES, A_LOGNORMAL = 0, 1


class _Params(ctypes.Structure):
    _fields_ = [
        ("n_users", ctypes.c_int64),
        ("n_items", ctypes.c_int32),
        ("pad0", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("deg_kind", ctypes.c_int32),
        ("deg_min", ctypes.c_int32),
        ("deg_max", ctypes.c_int32),
        ("item_kind", ctypes.c_int32),
        ("deg_p1", ctypes.c_double),
        ("deg_p2", ctypes.c_double),
        ("zipf_s", ctypes.c_double),
        ("c_kind", ctypes.c_int32),
        ("n_families", ctypes.c_int32),
        ("a_kind", ctypes.c_int32 * 4),
        ("a_p1", ctypes.c_double * 4),
        ("a_p2", ctypes.c_double * 4),
    ]


class _AppxParams(ctypes.Structure):
    _fields_ = [
        ("n_users", ctypes.c_int64),
        ("n_items", ctypes.c_int32),
        ("pad0", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("nu", ctypes.c_double),
        ("breadth_sigma", ctypes.c_double),
        ("value_sigma", ctypes.c_double),
        ("resp_sigma", ctypes.c_double),
        ("noise_sigma", ctypes.c_double),
        ("c_max", ctypes.c_double),
        ("scale_sigma", ctypes.c_double),
        ("eps0", ctypes.c_double),
    ]


def build(force: bool = False) -> str:
    """Compiles the generator into a shared library next to its source."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.wl_degrees.argtypes = [ctypes.POINTER(_Params), ctypes.c_void_p]
        lib.wl_degrees.restype = ctypes.c_int
        lib.wl_fill.argtypes = [ctypes.POINTER(_Params)] + [ctypes.c_void_p] * 5
        lib.wl_fill.restype = ctypes.c_int
        lib.wl_draw.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int64, ctypes.c_int64,
                                ctypes.c_int, ctypes.c_void_p]
        lib.wl_draw.restype = ctypes.c_int
        lib.wl_appx_counts.argtypes = [ctypes.POINTER(_AppxParams), ctypes.c_void_p]
        lib.wl_appx_counts.restype = ctypes.c_int64
        lib.wl_appx_fill.argtypes = [ctypes.POINTER(_AppxParams)] + [ctypes.c_void_p] * 6
        lib.wl_appx_fill.restype = ctypes.c_int
        lib.wl_philox4x32_10.argtypes = [ctypes.c_void_p] * 3
        lib.wl_philox4x32_10.restype = None
        _lib = lib
    return _lib


def philox4x32_10(ctr, key) -> List[int]:
    """The raw block function, for known-answer tests."""
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().wl_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return [int(x) for x in out]


def draw(seed: int, stream: int, first: int, n: int, normal: bool = False) -> np.ndarray:
    """n counter-based draws (U[0,1) or N(0,1)) for entities first..first+n-1."""
    out = np.empty(n, dtype=np.float64)
    rc = _load().wl_draw(seed, stream, first, n, 1 if normal else 0, out.ctypes.data)
    assert rc == 0
    return out


@dataclass
class Instance:
    """A ridge-regularized matching LP (paper eq. 1 with Definition 1's A).

    Arrays are user-major CSR: row i holds user i's eligible items.
    ``a`` is family-major (m x nnz) or None when every family has a_ij = 1.
    ``b`` is (m x J).  ``proj`` is the per-user simple set: 'simplex_le'
    (sum x <= radius, x >= 0), 'simplex_eq' (sum x = radius, x >= 0) or 'box'
    (0 <= x <= radius).
    """
    name: str
    n_users: int
    n_items: int
    n_families: int
    row_ptr: np.ndarray
    item_idx: np.ndarray
    c: np.ndarray
    a: Optional[np.ndarray]
    b: np.ndarray
    proj: str = "simplex_le"
    radius: float = 1.0
    meta: dict = field(default_factory=dict)
    upper: float = 0.0   # u of the box-cut set {0 <= x <= u, sum x <= radius}
    eq_families: int = 0  # bit k: family k holds equality rows A_k x = b_k
    global_cap: Optional[float] = None  # M of a global-count row sum_(i,j) x_ij <= M (None: no such row)

    @property
    def n_rows(self) -> int:
        """Dual coordinates: m*J item rows, plus the global-count row when present."""
        return self.n_families * self.n_items + (self.global_cap is not None)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    def item_counts(self) -> np.ndarray:
        return np.bincount(self.item_idx, minlength=self.n_items).astype(np.int64)

    def a_dense(self) -> np.ndarray:
        """Family-major coefficients with the ones materialised."""
        if self.a is None:
            return np.ones((self.n_families, self.nnz), dtype=np.float32)
        return self.a

    def user_slice(self, first: int, count: int) -> "Instance":
        """The sub-instance of users [first, first+count) with b unchanged."""
        s, e = int(self.row_ptr[first]), int(self.row_ptr[first + count])
        rp = (self.row_ptr[first:first + count + 1] - s).astype(np.int64)
        a = None if self.a is None else np.ascontiguousarray(self.a[:, s:e])
        return Instance(self.name + f"[{first}:{first + count}]", count, self.n_items, self.n_families,
                        rp, self.item_idx[s:e].copy(), self.c[s:e].copy(), a, self.b.copy(),
                        self.proj, self.radius, dict(self.meta), self.upper, self.eq_families, self.global_cap)


def _generate(n_users, n_items, seed, deg_kind, deg_p1, deg_p2, deg_min, deg_max, item_kind,
              zipf_s, c_kind, fam_kinds=(A_ONES,), fam_p=((0.0, 0.0),)):
    p = _Params()
    p.n_users, p.n_items, p.seed = int(n_users), int(n_items), int(seed)
    p.deg_kind, p.deg_p1, p.deg_p2 = deg_kind, float(deg_p1), float(deg_p2)
    p.deg_min, p.deg_max = int(deg_min), int(deg_max)
    p.item_kind, p.zipf_s, p.c_kind = item_kind, float(zipf_s), c_kind
    p.n_families = len(fam_kinds)
    for k, (kind, (p1, p2)) in enumerate(zip(fam_kinds, fam_p)):
        p.a_kind[k], p.a_p1[k], p.a_p2[k] = kind, p1, p2
    lib = _load()
    rp = np.empty(int(n_users) + 1, dtype=np.int64)
    assert lib.wl_degrees(ctypes.byref(p), rp.ctypes.data) == 0
    nnz = int(rp[-1])
    idx = np.empty(nnz, dtype=np.int32)
    c = np.empty(nnz, dtype=np.float32)
    n_ln = sum(1 for k in fam_kinds if k == A_LOGNORMAL)
    a_ln = np.empty((max(n_ln, 1), nnz), dtype=np.float32)
    w = np.empty(int(n_items), dtype=np.float64)
    rc = lib.wl_fill(ctypes.byref(p), rp.ctypes.data, idx.ctypes.data, c.ctypes.data,
                     a_ln.ctypes.data, w.ctypes.data)
    assert rc == 0, f"wl_fill failed ({rc})"
    return rp, idx, c, (a_ln if n_ln else None), w


def tiny_plain(seed: int = 0, binding: bool = False, n_users: int = 10_000, n_items: int = 100,
               mean_degree: float = 10.0) -> Instance:
    """Plain one-family matching LP at small size.

    b is 0.5 * nnz / J as stated for this workload (every capacity slack), or
    with ``binding`` 0.5 * I / J, which makes most capacities bind.
    """
    rp, idx, c, _, _ = _generate(n_users, n_items, seed, DEG_POISSON, mean_degree, 0.0, 1, n_items,
                                 ITEM_UNIFORM, 0.0, C_NEG_UNIFORM)
    J = n_items
    level = 0.5 * n_users / J if binding else 0.5 * rp[-1] / J
    b = np.full((1, J), float(level), dtype=np.float64)
    return Instance("tiny_plain" + ("_binding" if binding else ""), n_users, J, 1, rp, idx, c, None,
                    b, "simplex_le", 1.0, {"seed": seed, "binding": binding})


def production(seed: int = 2, n_users: int = 10_000_000, n_items: int = 10_000,
               deg_mu: float = 4.2, deg_sigma: float = 0.6, deg_max: int = 2000,
               zipf_s: float = 1.1, b_frac: float = 0.3) -> Instance:
    """Production-shape plain instance (10M users x 10k items by default)."""
    rp, idx, c, _, w = _generate(n_users, n_items, seed, DEG_LOGNORMAL, deg_mu, deg_sigma, 1, deg_max,
                                 ITEM_ZIPF, zipf_s, C_NEG_UNIFORM_POP)
    n = np.bincount(idx, minlength=n_items).astype(np.float64)
    b = (b_frac * n)[None, :]
    return Instance("production", n_users, n_items, 1, rp, idx, c, None, b, "simplex_le", 1.0,
                    {"seed": seed, "item_weight": w})


def two_family(seed: int = 0, n_users: int = 10_000, n_items: int = 100, box: float = 1.0) -> Instance:
    """tiny_plain pattern with a budget family and a count-cap family, box set."""
    rp, idx, c, a_ln, _ = _generate(n_users, n_items, seed, DEG_POISSON, 10.0, 0.0, 1, n_items,
                                    ITEM_UNIFORM, 0.0, C_NEG_UNIFORM,
                                    fam_kinds=(A_LOGNORMAL, A_ONES), fam_p=((0.0, 0.5), (0.0, 0.0)))
    nnz = int(rp[-1])
    a = np.empty((2, nnz), dtype=np.float32)
    a[0] = a_ln[0]
    a[1] = 1.0
    b = np.empty((2, n_items), dtype=np.float64)
    b[0] = 0.2 * np.bincount(idx, weights=a[0].astype(np.float64), minlength=n_items)
    b[1] = 0.3 * np.bincount(idx, minlength=n_items)
    return Instance("two_family", n_users, n_items, 2, rp, idx, c, a, b, "box", box, {"seed": seed})


def batch_member(k: int, binding: bool = True, scale: float = 1.0) -> Instance:
    """Member k (0..63) of the uneven batch; ``scale`` shrinks the user count."""
    seed = 4000 + k
    u = draw(seed, 99, 0, 2)
    I = int(round(math.exp(math.log(5e4) + u[0] * (math.log(2e6) - math.log(5e4))) * scale))
    J = int(round(math.exp(math.log(100) + u[1] * (math.log(5000) - math.log(100)))))
    I = max(I, 1)
    rp, idx, c, _, _ = _generate(I, J, seed, DEG_LOGNORMAL, 3.5, 0.8, 1, J, ITEM_UNIFORM, 0.0,
                                 C_NEG_UNIFORM)
    level = 0.5 * I / J if binding else 0.5 * rp[-1] / J
    b = np.full((1, J), float(level), dtype=np.float64)
    return Instance(f"batch_member{k}", I, J, 1, rp, idx, c, None, b, "simplex_le", 1.0,
                    {"seed": seed, "binding": binding})


def appendix_a(seed: int = 0, n_users: int = 100_000, n_items: int = 1000, nu: float = 20.0,
               breadth_sigma: float = 1.0, value_sigma: float = 0.5, resp_sigma: float = 0.5,
               noise_sigma: float = 0.25, c_max: float = 10.0, scale_sigma: float = 1.0,
               eps0: float = 1e-3) -> Instance:
    """The paper's Appendix-A construction (resource-major, greedy-load capacities).

    Users are the paper's requests, items its resources.  The solver minimises,
    so c = -value; a = s_j * value; per-user simplex sum x <= 1.  The
    distribution parameters (which the paper does not publish) are arguments.
    """
    p = _AppxParams()
    p.n_users, p.n_items, p.seed = int(n_users), int(n_items), int(seed)
    p.nu, p.breadth_sigma, p.value_sigma, p.resp_sigma = float(nu), float(breadth_sigma), float(value_sigma), \
        float(resp_sigma)
    p.noise_sigma, p.c_max, p.scale_sigma, p.eps0 = float(noise_sigma), float(c_max), float(scale_sigma), float(eps0)
    lib = _load()
    K = np.empty(int(n_items), dtype=np.int64)
    nnz = lib.wl_appx_counts(ctypes.byref(p), K.ctypes.data)
    assert nnz >= 0, f"wl_appx_counts failed ({nnz})"
    rp = np.empty(int(n_users) + 1, dtype=np.int64)
    idx = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float32)
    a = np.empty((1, nnz), dtype=np.float32)
    b = np.empty((1, int(n_items)), dtype=np.float64)
    rc = lib.wl_appx_fill(ctypes.byref(p), K.ctypes.data, rp.ctypes.data, idx.ctypes.data, val.ctypes.data,
                          a.ctypes.data, b.ctypes.data)
    assert rc == 0, f"wl_appx_fill failed ({rc})"
    return Instance("appendix_a", int(n_users), int(n_items), 1, rp, idx, -val, a, b, "simplex_le", 1.0,
                    {"seed": seed, "nu": nu, "item_counts": K})


def cadence_base(chain: int, n_users: int = 1_000_000, n_items: int = 5000) -> Instance:
    """Day 0 of a recurring chain: tiny_plain distributions, binding b."""
    inst = tiny_plain(seed=chain, binding=True, n_users=n_users, n_items=n_items)
    inst.name = f"cadence{chain}_day0"
    inst.meta.update({"chain": chain, "day": 0})
    return inst


def cadence_next(prev: Instance, day: int) -> Instance:
    """Next day of a chain: c <- min(0, c + 0.05|c| N(0,1)), b <- b (1 + U(-0.05, 0.05)).

    The eligibility pattern is unchanged.
    """
    chain = int(prev.meta.get("chain", 0))
    seed = 5_000_000 + chain
    z = draw(seed, 200 + day, 0, prev.nnz, normal=True)
    c = np.minimum(0.0, prev.c.astype(np.float64) + 0.05 * np.abs(prev.c) * z).astype(np.float32)
    u = draw(seed, 400 + day, 0, prev.b.size)
    b = prev.b * (1.0 + (u.reshape(prev.b.shape) - 0.5) * 0.1)
    meta = dict(prev.meta)
    meta["day"] = day
    return Instance(f"cadence{chain}_day{day}", prev.n_users, prev.n_items, prev.n_families,
                    prev.row_ptr, prev.item_idx, c, prev.a, b, prev.proj, prev.radius, meta)


def random_small(seed: int, n_users: int, n_items: int, max_degree: int, n_families: int = 1,
                 proj: str = "simplex_le", radius: float = 1.0, a_ones: bool = True,
                 b_scale: float = 0.3, upper: float = 0.0) -> Instance:
    """Small random instance for property tests (any projection kind, m families;
    ``upper`` is the cap u of the box-cut set)."""
    rp, idx, c, a_ln, _ = _generate(n_users, n_items, seed, DEG_LOGNORMAL, math.log(max(2, max_degree) / 2),
                                    0.7, 1, max_degree, ITEM_UNIFORM, 0.0, C_NEG_UNIFORM,
                                    fam_kinds=tuple(A_ONES if (a_ones and k == 0) else A_LOGNORMAL
                                                    for k in range(n_families)),
                                    fam_p=tuple((0.0, 0.5) for _ in range(n_families)))
    nnz = int(rp[-1])
    if a_ones and n_families == 1:
        a = None
        sums = np.bincount(idx, minlength=n_items)[None, :].astype(np.float64)
    else:
        a = np.empty((n_families, nnz), dtype=np.float32)
        r = 0
        for k in range(n_families):
            if a_ones and k == 0:
                a[k] = 1.0
            else:
                a[k] = a_ln[r]
                r += 1
        sums = np.stack([np.bincount(idx, weights=a[k].astype(np.float64), minlength=n_items)
                         for k in range(n_families)])
    b = b_scale * sums * radius
    return Instance(f"random_small{seed}", n_users, n_items, n_families, rp, idx, c, a, b, proj, radius,
                    {"seed": seed}, upper)
