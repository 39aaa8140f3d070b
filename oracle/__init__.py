"""FP64 CPU oracle for ridge-regularized matching-LP dual ascent.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports, links or
calls anything here, and nothing here imports the GPU package.

The arithmetic lives in ``dualip_oracle.c`` (plain C, FP64, OpenMP over users
with a fixed chunked merge order).  This module is argument marshalling plus
a few tiny pure-Python helpers used by the pins.

Every function states the passage of the paper it follows:
  eq. 2  dual function g(lam)                       -> dual_grad
  eq. 3  primal recovery x*(lam) = Pi_C(-(A^T lam + c)/gamma)
  eq. 4  gradient A x*(lam) - b (Danskin)
  Section 4.3  sort-based simplex projection (Duchi et al.) -> project_simplex
  Appendix C   Jacobi row scaling, step proportional to gamma -> scaling
  Section 4.4 / Section 6  accelerated projected ascent with continuation -> solve
  Table 4      primal / dual / gap / slack               -> certificate
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dualip_oracle.c")
_LIB = os.path.join(_HERE, "libdualip_oracle.so")

PROJ = {"simplex_le": 0, "simplex_eq": 1, "box": 2, "boxcut": 3}


class _Inst(ctypes.Structure):
    _fields_ = [
        ("n_users", ctypes.c_int64),
        ("n_items", ctypes.c_int32),
        ("n_families", ctypes.c_int32),
        ("row_ptr", ctypes.c_void_p),
        ("item_idx", ctypes.c_void_p),
        ("c", ctypes.c_void_p),
        ("a", ctypes.c_void_p),
        ("b", ctypes.c_void_p),
        ("proj", ctypes.c_int32),
        ("eq_mask", ctypes.c_int32),
        ("radius", ctypes.c_double),
        ("upper", ctypes.c_double),
        ("global_count", ctypes.c_int32),
        ("global_cap", ctypes.c_double),
    ]


class _Stats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int64),
        ("gamma", ctypes.c_double),
        ("dual_obj", ctypes.c_double),
        ("primal_obj", ctypes.c_double),
        ("rel_gap", ctypes.c_double),
        ("max_slack", ctypes.c_double),
        ("lagr_gap", ctypes.c_double),
        ("status", ctypes.c_int32),
        ("stage", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class _Opts(ctypes.Structure):
    _fields_ = [
        ("n_stages", ctypes.c_int32),
        ("jacobi", ctypes.c_int32),
        ("gammas", ctypes.c_void_p),
        ("iters", ctypes.c_void_p),
        ("tol", ctypes.c_double),
        ("max_iters", ctypes.c_int64),
        ("check_every", ctypes.c_int32),
        ("reset_momentum", ctypes.c_int32),
        ("step_scale", ctypes.c_double),
        ("n_snap", ctypes.c_int64),
        ("snap_iters", ctypes.c_void_p),
        ("snap_lambda", ctypes.c_void_p),
        ("trace_dual", ctypes.c_void_p),
    ]


def build(force: bool = False) -> str:
    """Compiles the oracle (gcc, FP64, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        vp = ctypes.c_void_p
        lib.orc_project_simplex.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_int, vp]
        lib.orc_project_simplex.restype = None
        lib.orc_project_box.argtypes = [vp, ctypes.c_int64, ctypes.c_double, vp]
        lib.orc_project_box.restype = None
        lib.orc_project_boxcut.argtypes = [vp, ctypes.c_int64, ctypes.c_double, ctypes.c_double, vp]
        lib.orc_project_boxcut.restype = None
        lib.orc_project_rows.argtypes = [vp, vp, vp]
        lib.orc_dual_grad_ex.argtypes = [vp, vp, ctypes.c_double, vp, vp, vp, vp, vp, vp]
        lib.orc_primal.argtypes = [vp, vp, ctypes.c_double, vp, vp]
        lib.orc_scaling.argtypes = [vp, ctypes.c_int, vp, vp]
        lib.orc_certificate.argtypes = [vp, vp, ctypes.c_double, vp]
        lib.orc_solve.argtypes = [vp, vp, vp, vp, vp]
        for f in ("orc_project_rows", "orc_dual_grad_ex", "orc_primal", "orc_scaling",
                  "orc_certificate", "orc_solve"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class _Bound:
    """Keeps the instance arrays alive (and contiguous) for a C call."""

    def __init__(self, inst):
        self.rp = np.ascontiguousarray(inst.row_ptr, dtype=np.int64)
        self.idx = np.ascontiguousarray(inst.item_idx, dtype=np.int32)
        self.c = np.ascontiguousarray(inst.c, dtype=np.float32)
        self.a = None if inst.a is None else np.ascontiguousarray(inst.a, dtype=np.float32)
        self.b = np.ascontiguousarray(inst.b, dtype=np.float64).reshape(-1)
        cap = getattr(inst, "global_cap", None)
        self.s = _Inst(int(inst.n_users), int(inst.n_items), int(inst.n_families), self.rp.ctypes.data,
                       self.idx.ctypes.data, self.c.ctypes.data, _p(self.a), self.b.ctypes.data,
                       PROJ[inst.proj], int(getattr(inst, "eq_families", 0) or 0), float(inst.radius),
                       float(getattr(inst, "upper", 0.0) or 0.0), int(cap is not None),
                       float(cap) if cap is not None else 0.0)
        # dual coordinates: m*J item rows, then the global-count row when present
        self.mJ = int(inst.n_families) * int(inst.n_items) + (cap is not None)  # all dual rows
        self.nnz = int(self.rp[-1])

    @property
    def ref(self):
        return ctypes.byref(self.s)


# -------------------------------------------------------------------------- #
# ProjectionMap                                                               #
# -------------------------------------------------------------------------- #
def project_simplex(v, z: float = 1.0, eq: bool = False) -> np.ndarray:
    """Pi onto {x >= 0, sum x <= z} (or = z): sort-based method of Duchi et al. (Section 4.3)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    x = np.empty_like(v)
    _load().orc_project_simplex(v.ctypes.data, v.size, float(z), int(eq), x.ctypes.data)
    return x


def project_box(v, u: float = 1.0) -> np.ndarray:
    """Pi onto [0, u]^d (the box variant of the per-user set, Section 3.3)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    x = np.empty_like(v)
    _load().orc_project_box(v.ctypes.data, v.size, float(u), x.ctypes.data)
    return x


def project_boxcut(v, u: float = 1.0, z: float = 1.0) -> np.ndarray:
    """Pi onto {0 <= x <= u, sum x <= z} (box-cut primitive of Table 1)."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    x = np.empty_like(v)
    _load().orc_project_boxcut(v.ctypes.data, v.size, float(u), float(z), x.ctypes.data)
    return x


def project_rows(inst, v) -> np.ndarray:
    """Blockwise Pi_C over every user's row (Table 1, ProjectionMap)."""
    bd = _Bound(inst)
    v = np.ascontiguousarray(v, dtype=np.float64)
    x = np.empty_like(v)
    assert _load().orc_project_rows(bd.ref, v.ctypes.data, x.ctypes.data) == 0
    return x


# -------------------------------------------------------------------------- #
# ObjectiveFunction                                                           #
# -------------------------------------------------------------------------- #
def dual_grad(inst, lam, gamma: float, want_x: bool = True):
    """(g(lam), grad g(lam), x*(lam), A x*(lam)) per eqs. 2-4, FP64.

    lam has shape (m*J,) in the problem's own units.
    """
    bd = _Bound(inst)
    lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(-1)
    assert lam.size == bd.mJ
    grad = np.empty(bd.mJ)
    ax = np.empty(bd.mJ)
    g = ctypes.c_double()
    x = np.empty(bd.nnz) if want_x else None
    rc = _load().orc_dual_grad_ex(bd.ref, lam.ctypes.data, float(gamma), ax.ctypes.data, grad.ctypes.data,
                                  ctypes.addressof(g), _p(x), None, None)
    assert rc == 0
    return g.value, grad, x, ax


def primal(inst, x, gamma: float):
    """(c^T x + (gamma/2)||x||^2, A x) for a given primal point (eq. 1)."""
    bd = _Bound(inst)
    x = np.ascontiguousarray(x, dtype=np.float64)
    ax = np.empty(bd.mJ)
    p = ctypes.c_double()
    _load().orc_primal(bd.ref, x.ctypes.data, float(gamma), ctypes.addressof(p), ax.ctypes.data)
    return p.value, ax


def scaling(inst, jacobi: bool = True):
    """(D, Lhat): Jacobi row scaling and the bound Lhat >= ||DA||_2^2 (Appendix C)."""
    bd = _Bound(inst)
    D = np.empty(bd.mJ)
    L = ctypes.c_double()
    _load().orc_scaling(bd.ref, int(jacobi), D.ctypes.data, ctypes.addressof(L))
    return D, L.value


def certificate(inst, lam, gamma: float) -> dict:
    """Dual value, repaired-primal value, relative gap and max slack at lam (Table 4 metrics)."""
    bd = _Bound(inst)
    lam = np.ascontiguousarray(lam, dtype=np.float64).reshape(-1)
    st = _Stats()
    _load().orc_certificate(bd.ref, lam.ctypes.data, float(gamma), ctypes.byref(st))
    return st.as_dict()


def solve(inst, gammas: Sequence[float], iters: Sequence[int], tol: float = 1e-4,
          max_iters: int = 20000, check_every: int = 10, jacobi: bool = True,
          reset_momentum: bool = True, step_scale: float = 1.0, lam0=None,
          snap_iters: Sequence[int] = (), trace: bool = False):
    """Accelerated projected dual ascent with gamma continuation (Sections 4.4, 6).

    Returns (lam, stats, snapshots[len(snap_iters), m*J], trace_or_None).
    """
    bd = _Bound(inst)
    g = np.ascontiguousarray(gammas, dtype=np.float64)
    it = np.ascontiguousarray(iters, dtype=np.int64)
    snaps = np.ascontiguousarray(sorted(snap_iters), dtype=np.int64)
    snap_lam = np.zeros((max(len(snaps), 1), bd.mJ))
    tr = np.full(max_iters, np.nan) if trace else None
    o = _Opts(len(g), int(jacobi), g.ctypes.data, it.ctypes.data, float(tol), int(max_iters),
              int(check_every), int(reset_momentum), float(step_scale), len(snaps),
              snaps.ctypes.data if len(snaps) else None, snap_lam.ctypes.data, _p(tr))
    lam_out = np.empty(bd.mJ)
    l0 = None if lam0 is None else np.ascontiguousarray(lam0, dtype=np.float64).reshape(-1)
    st = _Stats()
    rc = _load().orc_solve(bd.ref, ctypes.byref(o), _p(l0), lam_out.ctypes.data, ctypes.byref(st))
    assert rc == 0
    return lam_out, st.as_dict(), snap_lam[:len(snaps)], tr


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even of FP32 values to BF16 (8 significant bits, FP32's
    exponent range), returned as FP32.

    Written from the definition of the format rather than its bit layout: a
    finite x is a multiple of the quantum q = 2^(max(e, -126) - 7), with e the
    exponent of its leading bit (-126 is the smallest normal exponent, below it
    the quantum stays 2^-133); x / q is exact in FP64, rounded to the nearest
    integer with ties to even, and scaled back.  A result of magnitude 2^128 or
    more is outside the format and becomes +-inf; NaN and +-inf pass through.
    """
    with np.errstate(invalid="ignore", over="ignore"):  # NaN payloads and overflow to inf
        x32 = np.ascontiguousarray(x, dtype=np.float32)
        xd = x32.astype(np.float64)
        out = xd.copy()
        fin = np.isfinite(xd) & (xd != 0.0)
        _, E = np.frexp(xd[fin])                      # |x| = f 2^E with f in [0.5, 1)
        q = np.ldexp(1.0, np.maximum(E - 1, -126) - 7)
        r = np.rint(xd[fin] / q) * q                  # rint: nearest, ties to even
        r = np.where(np.abs(r) >= 2.0 ** 128, np.copysign(np.inf, r), r)
        out[fin] = r
        return out.astype(np.float32)
