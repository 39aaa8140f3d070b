"""Learned warm start for recurring solves on slowly drifting inputs.

Not part of the paper's method.  The paper's matching problems are re-solved
on a cadence (Section 1) and each gamma stage is warm-started from the previous
stage's duals (Section 6).  Here a small network predicts how each item's dual
moves from one day to the next, and the prediction competes with yesterday's
duals and the cold start on the dual objective before the solve starts; the
cold start stays the judge's fallback.

Day d, with every arithmetic step in the library's kernels:
  1. g   = grad g_gamma(lam_prev) on today's instance          (gradient pass)
  2. F   = per-item features of today's instance, lam_prev, g   (item pass)
  3. lam = max(0, lam_prev + s * MLP(F))                        (MFMA GEMMs)
  4. dl_solve_warm over {lam, lam_prev, 0} at the final gamma.
Python here only moves buffers and drives the training loop.
"""
from __future__ import annotations

import time

import numpy as np

from . import MLP

# Feature columns whose values move with the instance size (log n and the
# extremes of c over an item's users) are switched off by a zero input scale,
# so a network trained on small days applies to large ones.
SIZE_DEPENDENT_COLUMNS = (1, 4, 5)
USED_COLUMNS = 12


def he_init(seed: int, hidden: int) -> np.ndarray:
    """Flat FP32 parameters: He-normal W1 (used input rows), W2, w3; zero biases."""
    rng = np.random.default_rng(seed)
    W1 = np.zeros((16, hidden))
    W1[:USED_COLUMNS] = rng.normal(size=(USED_COLUMNS, hidden)) * np.sqrt(2.0 / USED_COLUMNS)
    W2 = rng.normal(size=(hidden, hidden)) * np.sqrt(2.0 / hidden)
    w3 = rng.normal(size=hidden) * np.sqrt(1.0 / hidden)
    parts = [W1.reshape(-1), np.zeros(hidden), W2.reshape(-1), np.zeros(hidden), w3, np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


class WarmStart:
    """The warm-start network with its input normalisation and target scale."""

    def __init__(self, hidden: int = 256, max_batch: int = 1 << 16, seed: int = 0, gamma: float = 1e-3):
        import torch
        self.torch = torch
        self.hidden, self.max_batch, self.gamma = int(hidden), int(max_batch), float(gamma)
        self.net = MLP(hidden=self.hidden, max_batch=self.max_batch)
        self.net.set_params(he_init(seed, self.hidden))
        self.shift = np.zeros(16, dtype=np.float32)
        self.scale = np.ones(16, dtype=np.float32)
        self.s = 1.0

    # ---------------------------------------------------------------- inference
    def features(self, prob, lam_prev, b_prev):
        """(F [J, 16] device, gradient at lam_prev) for today's problem."""
        _, g, _ = prob.dual_grad(lam_prev, self.gamma, want_obj=False)
        return prob.item_features(lam_prev, g, b_prev), g

    def predict(self, prob, lam_prev, b_prev):
        """Predicted duals for today's problem (device FP64, length J)."""
        if prob.m != 1:
            raise ValueError("the warm-start network covers one constraint family")
        F, _ = self.features(prob, lam_prev, b_prev)
        lam_prev = lam_prev.to(device="cuda", dtype=self.torch.float64).contiguous()
        out = []
        for r0 in range(0, F.shape[0], self.max_batch):
            r1 = min(F.shape[0], r0 + self.max_batch)
            out.append(self.net.predict_duals(F[r0:r1], lam_prev[r0:r1], self.s))
        return out[0] if len(out) == 1 else self.torch.cat(out)

    def solve(self, prob, lam_prev, b_prev, gammas=None, iters=None, tol=1e-4, max_iters=20000, check_every=10):
        """Judged warm solve; returns (lam, stats, info) where info has the chosen
        candidate ('learned', 'previous' or 'cold'), the candidates' dual values
        and the seconds spent predicting (inside stats['wall_s'])."""
        torch = self.torch
        gammas = [self.gamma] if gammas is None else gammas
        iters = [-1] * len(gammas) if iters is None else iters
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam_l = self.predict(prob, lam_prev, b_prev)
        torch.cuda.synchronize()
        t_pred = time.perf_counter() - t0
        lam, st, chosen, duals = prob.solve_warm([lam_l, lam_prev, None], gammas, iters, tol=tol,
                                                 max_iters=max_iters, check_every=check_every)
        torch.cuda.synchronize()
        st["wall_s"] = time.perf_counter() - t0
        names = ("learned", "previous", "cold")
        return lam, st, {"chosen": names[chosen], "duals": dict(zip(names, map(float, duals))),
                         "predict_s": t_pred}

    # ----------------------------------------------------------------- training
    def fit(self, X: np.ndarray, dlam: np.ndarray, epochs: int = 20, batch: int = 8192, lr: float = 1e-3,
            wd: float = 1e-4, seed: int = 0, log=None):
        """Trains on feature rows X [N, 16] (FP32) and dual moves dlam [N]
        (today's optimum minus lam_prev).  Sets the input normalisation from X
        and the target scale s from dlam; returns the per-epoch mean losses."""
        torch = self.torch
        X = np.ascontiguousarray(X, dtype=np.float32)
        dlam = np.asarray(dlam, dtype=np.float64).reshape(-1)
        n = X.shape[0]
        if n == 0 or dlam.size != n:
            raise ValueError("need matching, non-empty X and dlam")
        mean = X.astype(np.float64).mean(axis=0)
        std = X.astype(np.float64).std(axis=0)
        shift = np.where(std > 0, mean, 0.0)
        scale = np.where(std > 1e-12, 1.0 / np.maximum(std, 1e-12), 0.0)
        scale[list(SIZE_DEPENDENT_COLUMNS)] = 0.0
        scale[USED_COLUMNS:] = 0.0
        self.shift, self.scale = shift.astype(np.float32), scale.astype(np.float32)
        self.net.set_input_norm(self.shift, self.scale)
        self.s = float(max(np.std(dlam), 1e-12))
        Xd = torch.from_numpy(X).cuda()
        Td = torch.from_numpy((dlam / self.s).astype(np.float32)).cuda()
        gen = torch.Generator(device="cuda")
        gen.manual_seed(seed)
        batch = min(batch, self.max_batch)
        steps_per_epoch = max(1, n // batch)
        total = epochs * steps_per_epoch
        history = []
        step = 0
        for ep in range(epochs):
            perm = torch.randperm(n, device="cuda", generator=gen)
            losses = []
            for k in range(steps_per_epoch):
                sel = perm[k * batch:(k + 1) * batch]
                # cosine decay to 1% of lr
                lr_k = lr * (0.01 + 0.99 * 0.5 * (1.0 + np.cos(np.pi * step / max(total, 1))))
                want = (k == steps_per_epoch - 1) or (k % 50 == 0)
                lo = self.net.train_step(Xd.index_select(0, sel), Td.index_select(0, sel), lr_k, wd, want_loss=want)
                if lo is not None:
                    losses.append(lo)
                step += 1
            history.append(float(np.mean(losses)))
            if log:
                log(f"epoch {ep + 1}/{epochs}: loss {history[-1]:.4f} (target variance 0.5)")
        return history

    # -------------------------------------------------------------- persistence
    def save(self, path: str):
        np.savez(path, params=self.net.get_params(), shift=self.shift, scale=self.scale, s=np.float64(self.s),
                 hidden=np.int64(self.hidden), gamma=np.float64(self.gamma))

    @classmethod
    def load(cls, path: str, max_batch: int = 1 << 16) -> "WarmStart":
        z = np.load(path, allow_pickle=False)
        w = cls(hidden=int(z["hidden"]), max_batch=max_batch, gamma=float(z["gamma"]))
        w.net.set_params(z["params"])
        w.shift, w.scale, w.s = z["shift"].astype(np.float32), z["scale"].astype(np.float32), float(z["s"])
        w.net.set_input_norm(w.shift, w.scale)
        return w
