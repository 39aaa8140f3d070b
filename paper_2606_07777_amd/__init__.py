"""Python binding of libdualip (gfx950 ridge-regularized matching-LP dual ascent).

Argument marshalling only: every step of the computation runs in the HIP
library declared in include/dualip.h.  PyTorch supplies device memory and the
stream.  The binding raises if the built library is missing; there is no CPU
fallback.

Function names follow the C ABI (dl_problem_create, dl_dual_grad, dl_project,
dl_solve, dl_solver_*); the classes Problem and Solver wrap them for tensors.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("DUALIP_LIB", os.path.join(HERE, "libdualip.so"))

DL_OK, DL_NOT_CONVERGED = 0, 1
STATUS = {0: "DL_OK", 1: "DL_NOT_CONVERGED", -1: "DL_EINVAL", -2: "DL_ENOMEM", -3: "DL_EHIP",
          -4: "DL_EUNSUPPORTED", -5: "DL_DIVERGED", -6: "DL_NUMERIC"}
PROJ = {"simplex_le": 0, "simplex_eq": 1, "box": 2, "boxcut": 3}
STORAGE = {"f32": 0, "bf16": 1}
LAYOUT = {"bucketed": 0, "wavefront": 1}


class DualipError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class dl_problem_desc(ctypes.Structure):
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
        ("storage", ctypes.c_int32),
        ("radius", ctypes.c_double),
        ("upper", ctypes.c_double),
        ("jacobi", ctypes.c_int32),
        ("wg_per_cu", ctypes.c_int32),
        ("layout", ctypes.c_int32),
        ("eq_families", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
        ("global_cap", ctypes.c_double),
        ("global_count", ctypes.c_int32),
    ]


class dl_solver_meta(ctypes.Structure):
    _fields_ = [
        ("gamma", ctypes.c_double),
        ("eta", ctypes.c_double),
        ("tk", ctypes.c_double),
        ("iters", ctypes.c_int64),
        ("m_times_j", ctypes.c_int64),
    ]


class dl_problem_info(ctypes.Structure):
    _fields_ = [
        ("n_users", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("n_items", ctypes.c_int32),
        ("n_families", ctypes.c_int32),
        ("n_stored_families", ctypes.c_int32),
        ("n_workgroups", ctypes.c_int32),
        ("n_tasks", ctypes.c_int64),
        ("lhat", ctypes.c_double),
        ("bytes_per_pass", ctypes.c_double),
        ("device_bytes", ctypes.c_double),
        ("max_degree", ctypes.c_int32),
        ("n_buckets", ctypes.c_int32),
        ("bucket_glog", ctypes.c_int32 * 8),
        ("bucket_users", ctypes.c_int64 * 8),
        ("qscale", ctypes.c_float * 4),
        ("n_rows", ctypes.c_int64),
        ("n_windows", ctypes.c_int32),
    ]


class dl_solve_opts(ctypes.Structure):
    _fields_ = [
        ("n_stages", ctypes.c_int32),
        ("check_every", ctypes.c_int32),
        ("gammas", ctypes.c_void_p),
        ("iters", ctypes.c_void_p),
        ("tol", ctypes.c_double),
        ("max_iters", ctypes.c_int64),
        ("reset_momentum", ctypes.c_int32),
        ("autotune_rounds", ctypes.c_int32),
        ("step_scale", ctypes.c_double),
    ]


class dl_solve_stats(ctypes.Structure):
    _fields_ = [
        ("iters", ctypes.c_int64),
        ("stage", ctypes.c_int32),
        ("status", ctypes.c_int32),
        ("gamma", ctypes.c_double),
        ("dual_obj", ctypes.c_double),
        ("primal_obj", ctypes.c_double),
        ("rel_gap", ctypes.c_double),
        ("max_slack", ctypes.c_double),
        ("lagr_gap", ctypes.c_double),
        ("n_checks", ctypes.c_int64),
        ("wall_ms", ctypes.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class dl_tune_result(ctypes.Structure):
    _fields_ = [
        ("n_workgroups", ctypes.c_int32),
        ("rounds", ctypes.c_int32),
        ("pass_ms_model", ctypes.c_double),
        ("pass_ms_tuned", ctypes.c_double),
        ("imbalance_model", ctypes.c_double),
        ("imbalance_tuned", ctypes.c_double),
    ]


class dl_mlp_desc(ctypes.Structure):
    _fields_ = [
        ("n_in", ctypes.c_int32),
        ("hidden", ctypes.c_int32),
        ("max_batch", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
    ]


class dl_timing(ctypes.Structure):
    _fields_ = [
        ("n_grad", ctypes.c_int64),
        ("grad_ms_total", ctypes.c_double),
        ("n_update", ctypes.c_int64),
        ("update_ms_total", ctypes.c_double),
    ]


# Every symbol include/dualip.h declares, with its ctypes signature.
_VP, _I32, _I64, _D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
SIGNATURES = {
    "dl_problem_create": ([ctypes.POINTER(dl_problem_desc), ctypes.POINTER(_VP)], _I32),
    "dl_problem_destroy": ([_VP], None),
    "dl_problem_get_info": ([_VP, ctypes.POINTER(dl_problem_info)], _I32),
    "dl_dual_grad": ([_VP, _VP, _D, _VP, _VP, _VP], _I32),
    "dl_project": ([_VP, _VP, _VP], _I32),
    "dl_solve": ([_VP, ctypes.POINTER(dl_solve_opts), _VP, _VP, ctypes.POINTER(dl_solve_stats)], _I32),
    "dl_read_bandwidth": ([_I64, _I32, _VP, ctypes.POINTER(_D)], _I32),
    "dl_solve_noalloc": ([_VP, ctypes.POINTER(dl_solve_opts), _VP, _VP, ctypes.POINTER(dl_solve_stats)], _I32),
    "dl_solver_create": ([_VP, _VP, ctypes.POINTER(_VP)], _I32),
    "dl_solver_destroy": ([_VP], None),
    "dl_solver_set_stage": ([_VP, _D, _D, _I32], _I32),
    "dl_solver_step": ([_VP, _I64], _I32),
    "dl_solver_get_lambda": ([_VP, _VP], _I32),
    "dl_solver_certificate": ([_VP, ctypes.POINTER(dl_solve_stats)], _I32),
    "dl_solver_enable_timing": ([_VP, _I32], _I32),
    "dl_solver_get_timing": ([_VP, ctypes.POINTER(dl_timing)], _I32),
    "dl_solver_autotune": ([_VP, _I32, ctypes.POINTER(dl_tune_result)], _I32),
    "dl_batch_create": ([_I32, ctypes.POINTER(_VP), ctypes.POINTER(_VP)], _I32),
    "dl_batch_destroy": ([_VP], None),
    "dl_batch_solve": ([_VP, ctypes.POINTER(dl_solve_opts), ctypes.POINTER(_VP), ctypes.POINTER(_VP),
                        ctypes.POINTER(dl_solve_stats)], _I32),
    "dl_batch_get_tune": ([_VP, ctypes.POINTER(dl_tune_result)], _I32),
    "dl_item_features": ([_VP, _VP, _VP, _VP, _VP], _I32),
    "dl_solver_export": ([_VP, _VP, ctypes.POINTER(dl_solver_meta)], _I32),
    "dl_solver_import": ([_VP, _VP, ctypes.POINTER(dl_solver_meta)], _I32),
    "dl_mlp_set_input_norm": ([_VP, _VP, _VP], _I32),
    "dl_mlp_predict_duals": ([_VP, _VP, _I64, _VP, ctypes.c_double, _VP], _I32),
    "dl_problem_update": ([_VP, _VP, _VP], _I32),
    "dl_solve_warm": ([_VP, ctypes.POINTER(dl_solve_opts), _I32, ctypes.POINTER(_VP), _VP,
                       ctypes.POINTER(dl_solve_stats), ctypes.POINTER(_I32), _VP], _I32),
    "dl_mlp_create": ([ctypes.POINTER(dl_mlp_desc), ctypes.POINTER(_VP)], _I32),
    "dl_mlp_destroy": ([_VP], None),
    "dl_mlp_num_params": ([_VP], _I64),
    "dl_mlp_set_params": ([_VP, _VP], _I32),
    "dl_mlp_get_params": ([_VP, _VP], _I32),
    "dl_mlp_forward": ([_VP, _VP, _I64, _VP], _I32),
    "dl_mlp_gradients": ([_VP, _VP, _VP, _I64, _VP, _VP], _I32),
    "dl_mlp_train_step": ([_VP, _VP, _VP, _I64, ctypes.c_float, ctypes.c_float, ctypes.POINTER(_D)], _I32),
    "dl_last_error": ([], ctypes.c_char_p),
}

_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads the built library (raises if it is missing: no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"libdualip.so is not built ({path}); run paper_2606_07777_amd/build.py")
        lib = ctypes.CDLL(path)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _check(status: int, allow=(DL_OK,)) -> int:
    if status not in allow and status < 0:
        raise DualipError(status, load().dl_last_error().decode())
    return status


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


def _stream(torch, stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Problem:
    """A created dl_problem on the current device.

    row_ptr (int64), item_idx (int32), c (float32) and a (float32, m x nnz, or
    None) may be torch tensors on the device or numpy arrays (copied there);
    b is host data (m x J).
    """

    def __init__(self, n_users, n_items, n_families, row_ptr, item_idx, c, a, b, proj="simplex_le",
                 radius=1.0, storage="f32", jacobi=True, wg_per_cu=0, stream=None, layout="bucketed", upper=0.0,
                 eq_families=0, global_cap=None):
        import torch
        self.torch = torch
        dev = torch.device("cuda", torch.cuda.current_device())

        def dev_t(x, dt):
            if x is None:
                return None
            if isinstance(x, torch.Tensor):
                return x.to(device=dev, dtype=dt).contiguous()
            return torch.from_numpy(np.ascontiguousarray(x)).to(device=dev, dtype=dt)

        self.m, self.J, self.I = int(n_families), int(n_items), int(n_users)
        self._rp = dev_t(row_ptr, torch.int64)
        self._idx = dev_t(item_idx, torch.int32)
        self._c = dev_t(c, torch.float32)
        self._a = dev_t(a, torch.float32)
        bh = np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(-1))
        self.stream = _stream(torch, stream)
        desc = dl_problem_desc(self.I, self.J, self.m, _ptr(self._rp), _ptr(self._idx), _ptr(self._c),
                               _ptr(self._a), bh.ctypes.data, PROJ[proj], STORAGE[storage], float(radius),
                               float(upper), int(jacobi), int(wg_per_cu), LAYOUT[layout], int(eq_families),
                               self.stream, float(global_cap) if global_cap is not None else 0.0,
                               int(global_cap is not None))
        h = ctypes.c_void_p()
        _check(load().dl_problem_create(ctypes.byref(desc), ctypes.byref(h)))
        self.handle = h
        # the library copied what it needs
        self._rp = self._idx = self._c = self._a = None
        info = self.info()
        self.nnz = info["nnz"]
        self.nrow = info["n_rows"]  # dual coordinates: m*J, plus the global-count row

    @classmethod
    def from_instance(cls, inst, storage="f32", jacobi=True, wg_per_cu=0, stream=None, layout="bucketed"):
        """From any object with the attributes of a CSR matching instance."""
        return cls(inst.n_users, inst.n_items, inst.n_families, inst.row_ptr, inst.item_idx, inst.c, inst.a,
                   inst.b, inst.proj, inst.radius, storage, jacobi, wg_per_cu, stream, layout,
                   float(getattr(inst, "upper", 0.0) or 0.0), int(getattr(inst, "eq_families", 0) or 0),
                   getattr(inst, "global_cap", None))

    def close(self):
        if getattr(self, "handle", None):
            load().dl_problem_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        o = dl_problem_info()
        _check(load().dl_problem_get_info(self.handle, ctypes.byref(o)))
        d = {f: getattr(o, f) for f, _ in o._fields_}
        nb = d["n_buckets"]
        d["bucket_glog"] = list(o.bucket_glog)[:nb]
        d["bucket_users"] = list(o.bucket_users)[:nb]
        d["qscale"] = list(o.qscale)[:self.m]
        return d

    def _check_rows(self, t, what):
        """Device dual vectors must hold n_rows entries (the library reads that many)."""
        if t is not None and t.numel() != self.nrow:
            raise ValueError(f"{what} has {t.numel()} entries, expected n_rows = {self.nrow}")

    def _empty(self, n, dt):
        return self.torch.empty(n, dtype=dt, device="cuda")

    def dual_grad(self, lam, gamma: float, want_obj=True, want_x=False):
        """dl_dual_grad: (g(lam) or None, grad tensor [n_rows] f64, x tensor [nnz] f32 or None)."""
        torch = self.torch
        lam = lam.to(device="cuda", dtype=torch.float64).contiguous()
        self._check_rows(lam, "lam")
        grad = self._empty(self.nrow, torch.float64)
        x = self._empty(self.nnz, torch.float32) if want_x else None
        g = ctypes.c_double()
        _check(load().dl_dual_grad(self.handle, _ptr(lam), float(gamma), _ptr(grad),
                                   ctypes.addressof(g) if want_obj else None, _ptr(x)))
        torch.cuda.current_stream().synchronize()
        return (g.value if want_obj else None), grad, x

    def project(self, v):
        """dl_project: x = Pi_C(v) row by row (caller order)."""
        torch = self.torch
        v = v.to(device="cuda", dtype=torch.float32).contiguous()
        x = self._empty(self.nnz, torch.float32)
        _check(load().dl_project(self.handle, _ptr(v), _ptr(x)))
        return x

    def solve(self, gammas: Sequence[float], iters: Sequence[int], tol=1e-4, max_iters=20000, check_every=10,
              reset_momentum=True, step_scale=1.0, lam0=None, autotune_rounds=0, out=None, noalloc=False):
        """dl_solve over the schedule; returns (lam tensor f64 [m*J], stats dict).

        noalloc=True calls dl_solve_noalloc (no device allocation inside the call);
        out may then be a preallocated float64 tensor of m*J entries."""
        torch = self.torch
        g = np.ascontiguousarray(gammas, dtype=np.float64)
        it = np.ascontiguousarray(iters, dtype=np.int64)
        o = dl_solve_opts(len(g), int(check_every), g.ctypes.data, it.ctypes.data, float(tol), int(max_iters),
                          int(reset_momentum), int(autotune_rounds), float(step_scale))
        l0 = None if lam0 is None else lam0.to(device="cuda", dtype=torch.float64).contiguous()
        self._check_rows(l0, "lam0")
        if out is None:
            out = self._empty(self.nrow, torch.float64)
        elif out.dtype != torch.float64 or out.numel() != self.nrow or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 tensor of m*J entries")
        st = dl_solve_stats()
        fn = load().dl_solve_noalloc if noalloc else load().dl_solve
        _check(fn(self.handle, ctypes.byref(o), _ptr(l0), _ptr(out), ctypes.byref(st)),
               allow=(DL_OK, DL_NOT_CONVERGED))
        return out, st.as_dict()

    def solver(self, lam0=None) -> "Solver":
        return Solver(self, lam0)

    def update(self, c=None, b=None):
        """dl_problem_update: new c (caller CSR order) and / or b on the same pattern."""
        torch = self.torch
        ct = None if c is None else (c.to(device="cuda", dtype=torch.float32).contiguous()
                                     if isinstance(c, torch.Tensor) else
                                     torch.from_numpy(np.ascontiguousarray(c, dtype=np.float32)).cuda())
        bh = None if b is None else np.ascontiguousarray(np.asarray(b, dtype=np.float64).reshape(-1))
        if ct is not None and ct.numel() != self.nnz:
            raise ValueError(f"c has {ct.numel()} entries, the problem has {self.nnz} nonzeros")
        if bh is not None and bh.size != self.m * self.J:
            raise ValueError(f"b has {bh.size} entries, expected {self.m * self.J}")
        _check(load().dl_problem_update(self.handle, _ptr(ct), None if bh is None else bh.ctypes.data))

    def solve_warm(self, candidates, gammas, iters, tol=1e-4, max_iters=20000, check_every=10,
                   reset_momentum=True, step_scale=1.0, autotune_rounds=0):
        """dl_solve_warm: returns (lam, stats, chosen index, candidate dual values)."""
        torch = self.torch
        g = np.ascontiguousarray(gammas, dtype=np.float64)
        it = np.ascontiguousarray(iters, dtype=np.int64)
        o = dl_solve_opts(len(g), int(check_every), g.ctypes.data, it.ctypes.data, float(tol), int(max_iters),
                          int(reset_momentum), int(autotune_rounds), float(step_scale))
        ts = [None if c is None else c.to(device="cuda", dtype=torch.float64).contiguous() for c in candidates]
        for t in ts:
            if t is not None and t.numel() != self.nrow:
                raise ValueError(f"a candidate has {t.numel()} entries, expected {self.nrow}")
        arr = (ctypes.c_void_p * len(ts))(*[_ptr(t) for t in ts])
        out = self._empty(self.nrow, torch.float64)
        st = dl_solve_stats()
        chosen = ctypes.c_int32(-1)
        duals = np.zeros(len(ts))
        _check(load().dl_solve_warm(self.handle, ctypes.byref(o), len(ts), arr, _ptr(out), ctypes.byref(st),
                                    ctypes.byref(chosen), duals.ctypes.data), allow=(DL_OK, DL_NOT_CONVERGED))
        return out, st.as_dict(), chosen.value, duals

    def item_features(self, lam_prev, g_prev, b_prev):
        """dl_item_features: [J, 16] FP32 features (family 0) on the device."""
        torch = self.torch
        lp = lam_prev.to(device="cuda", dtype=torch.float64).contiguous()
        gp = g_prev.to(device="cuda", dtype=torch.float64).contiguous()
        bp = np.ascontiguousarray(np.asarray(b_prev, dtype=np.float64).reshape(-1))
        out = self._empty(self.J * 16, torch.float32)
        _check(load().dl_item_features(self.handle, _ptr(lp), _ptr(gp), bp.ctypes.data, _ptr(out)))
        return out.view(self.J, 16)


class Solver:
    """Stepwise Maximizer (dl_solver_*)."""

    def __init__(self, prob: Problem, lam0=None):
        self.prob = prob
        torch = prob.torch
        self._l0 = None if lam0 is None else lam0.to(device="cuda", dtype=torch.float64).contiguous()
        prob._check_rows(self._l0, "lam0")
        h = ctypes.c_void_p()
        _check(load().dl_solver_create(prob.handle, _ptr(self._l0), ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            load().dl_solver_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stage(self, gamma: float, step_scale: float = 1.0, reset: bool = True):
        _check(load().dl_solver_set_stage(self.handle, float(gamma), float(step_scale), int(reset)))

    def step(self, n: int):
        _check(load().dl_solver_step(self.handle, int(n)))

    def lam(self):
        out = self.prob._empty(self.prob.nrow, self.prob.torch.float64)
        _check(load().dl_solver_get_lambda(self.handle, _ptr(out)))
        return out

    def export_state(self):
        """(state tensor on the device, meta dict): a checkpoint of the dual state."""
        torch = self.prob.torch
        state = self.prob._empty(2 * self.prob.nrow, torch.float64)
        meta = dl_solver_meta()
        _check(load().dl_solver_export(self.handle, _ptr(state), ctypes.byref(meta)))
        return state, {f: getattr(meta, f) for f, _ in meta._fields_}

    def import_state(self, state, meta: dict):
        """Loads a checkpoint from export_state (same problem data)."""
        torch = self.prob.torch
        state = state.to(device="cuda", dtype=torch.float64).contiguous()
        if state.numel() != 2 * self.prob.nrow:
            raise ValueError("state size does not match the problem")
        m = dl_solver_meta(**meta)
        _check(load().dl_solver_import(self.handle, _ptr(state), ctypes.byref(m)))

    def certificate(self) -> dict:
        st = dl_solve_stats()
        _check(load().dl_solver_certificate(self.handle, ctypes.byref(st)))
        return st.as_dict()

    def autotune(self, rounds: int = 10) -> dict:
        """dl_solver_autotune: balance the workgroup split from measured times."""
        r = dl_tune_result()
        _check(load().dl_solver_autotune(self.handle, int(rounds), ctypes.byref(r)))
        return {f: getattr(r, f) for f, _ in r._fields_}

    def enable_timing(self, on: bool = True):
        _check(load().dl_solver_enable_timing(self.handle, int(on)))

    def timing(self) -> dict:
        t = dl_timing()
        _check(load().dl_solver_get_timing(self.handle, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in t._fields_}


class Batch:
    """dl_batch_*: several problems solved in lockstep, one launch per iteration phase."""

    def __init__(self, probs):
        self.probs = list(probs)
        arr = (ctypes.c_void_p * len(self.probs))(*[p.handle.value for p in self.probs])
        h = ctypes.c_void_p()
        _check(load().dl_batch_create(len(self.probs), arr, ctypes.byref(h)))
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            load().dl_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, gammas, iters, tol=1e-4, max_iters=20000, check_every=10, reset_momentum=True,
              step_scale=1.0, lam0=None, autotune=2):
        """Returns ([lam tensor per member], [stats dict per member]).  autotune > 0
        (the default) re-deals the workgroups from the measured time of the solve's own
        iterations, that many rounds per grid (see tune()); 0 keeps the cost-model split."""
        torch = self.probs[0].torch
        n = len(self.probs)
        g = np.ascontiguousarray(gammas, dtype=np.float64)
        it = np.ascontiguousarray(iters, dtype=np.int64)
        o = dl_solve_opts(len(g), int(check_every), g.ctypes.data, it.ctypes.data, float(tol), int(max_iters),
                          int(reset_momentum), int(autotune), float(step_scale))
        outs = [p._empty(p.nrow, torch.float64) for p in self.probs]
        out_arr = (ctypes.c_void_p * n)(*[_ptr(t) for t in outs])
        l0 = None
        if lam0 is not None:
            l0t = [t.to(device="cuda", dtype=torch.float64).contiguous() for t in lam0]
            for p, t in zip(self.probs, l0t):
                p._check_rows(t, "lam0")
            l0 = (ctypes.c_void_p * n)(*[_ptr(t) for t in l0t])
        stats = (dl_solve_stats * n)()
        _check(load().dl_batch_solve(self.handle, ctypes.byref(o), l0, out_arr, stats),
               allow=(DL_OK, DL_NOT_CONVERGED))
        return outs, [s.as_dict() for s in stats]

    def tune(self):
        """dl_batch_get_tune: the last solve's workgroup tuning as a dict."""
        r = dl_tune_result()
        _check(load().dl_batch_get_tune(self.handle, ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in dl_tune_result._fields_}


def read_bandwidth(nbytes: int, reps: int = 10, stream=None) -> float:
    """dl_read_bandwidth: sustained HBM read GB/s over a library-allocated buffer of nbytes."""
    import torch
    g = ctypes.c_double()
    _check(load().dl_read_bandwidth(int(nbytes), int(reps), _stream(torch, stream), ctypes.byref(g)))
    return g.value


class MLP:
    """dl_mlp_*: the warm-start network (16 -> H -> H -> 1) on BF16 matrix cores."""

    def __init__(self, hidden: int = 256, max_batch: int = 16384, stream=None):
        import torch
        self.torch = torch
        self.hidden, self.max_batch = int(hidden), int(max_batch)
        d = dl_mlp_desc(16, self.hidden, self.max_batch, _stream(torch, stream))
        h = ctypes.c_void_p()
        _check(load().dl_mlp_create(ctypes.byref(d), ctypes.byref(h)))
        self.handle = h
        self.n_params = int(load().dl_mlp_num_params(h))

    def close(self):
        if getattr(self, "handle", None):
            load().dl_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        a = np.ascontiguousarray(flat, dtype=np.float32)
        assert a.size == self.n_params
        _check(load().dl_mlp_set_params(self.handle, a.ctypes.data))

    def get_params(self):
        a = np.empty(self.n_params, dtype=np.float32)
        _check(load().dl_mlp_get_params(self.handle, a.ctypes.data))
        return a

    def set_input_norm(self, shift, scale):
        sh = np.ascontiguousarray(shift, dtype=np.float32).reshape(16)
        sc = np.ascontiguousarray(scale, dtype=np.float32).reshape(16)
        _check(load().dl_mlp_set_input_norm(self.handle, sh.ctypes.data, sc.ctypes.data))

    def predict_duals(self, X, lam_prev, s: float):
        """max(0, lam_prev + s * MLP(X)) in FP64 on the device."""
        torch = self.torch
        X = X.to(device="cuda", dtype=torch.float32).contiguous()
        lp = lam_prev.to(device="cuda", dtype=torch.float64).contiguous()
        if lp.numel() != X.shape[0]:
            raise ValueError("lam_prev must have one entry per row of X")
        out = torch.empty(X.shape[0], dtype=torch.float64, device="cuda")
        _check(load().dl_mlp_predict_duals(self.handle, _ptr(X), X.shape[0], _ptr(lp), float(s), _ptr(out)))
        return out

    def forward(self, X):
        torch = self.torch
        X = X.to(device="cuda", dtype=torch.float32).contiguous()
        y = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        _check(load().dl_mlp_forward(self.handle, _ptr(X), X.shape[0], _ptr(y)))
        return y

    def gradients(self, X, dy):
        torch = self.torch
        X = X.to(device="cuda", dtype=torch.float32).contiguous()
        dy = dy.to(device="cuda", dtype=torch.float32).contiguous()
        y = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(load().dl_mlp_gradients(self.handle, _ptr(X), _ptr(dy), X.shape[0], _ptr(y), _ptr(g)))
        return y, g

    def train_step(self, X, target, lr: float, wd: float = 0.0, want_loss: bool = True):
        """One AdamW step; returns the loss before it (synchronising) or None."""
        torch = self.torch
        X = X.to(device="cuda", dtype=torch.float32).contiguous()
        t = target.to(device="cuda", dtype=torch.float32).contiguous()
        if X.shape[0] > self.max_batch or t.numel() != X.shape[0]:
            raise ValueError("batch larger than max_batch or target of the wrong length")
        loss = ctypes.c_double()
        _check(load().dl_mlp_train_step(self.handle, _ptr(X), _ptr(t), X.shape[0], float(lr), float(wd),
                                        ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None
