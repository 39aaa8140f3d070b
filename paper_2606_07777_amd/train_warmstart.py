"""Trains the warm-start network on synthetic daily chains and stores it.

Each chain is a day-0 matching instance (uniform items, Poisson(10) degrees,
c = -U(0,1), a = 1, binding b = 0.5 I/J, user simplex <= 1) followed by days
on the same eligibility pattern whose costs and capacities drift:
c <- min(0, c + 0.05 |c| N(0,1)), b <- b (1 + U(-0.05, 0.05)).  Day 0 is solved
cold over the continuation schedule; each later day is solved from the
previous day's duals at the final gamma to a 1e-4 certified gap.  Every day
contributes one row per item: its features (taken at the previous day's duals
on the new day's instance) and the move of its dual.  Chains are split 90/10
into training and validation.

    python -m paper_2606_07777_amd.train_warmstart --chains 100 --days 20 \\
        --users 1000000 --items 5000 --out paper_2606_07777_amd/weights/warmstart.npz
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COLD = dict(gammas=[1e-1, 1e-2, 1e-3], iters=[300, 300, -1], tol=1e-4, max_iters=20000, check_every=10)
FINAL = dict(gammas=[1e-3], iters=[-1], tol=1e-4, max_iters=20000, check_every=10)
CHAIN_SEED0 = 5000


def log(msg):
    print(f"[warmstart] {msg}", flush=True)


def collect_chain(chain: int, days: int, n_users: int, n_items: int, ws, pool):
    """[(features [J,16] f32, dual move [J] f64, warm iterations)] for days 1..days."""
    import torch

    import paper_2606_07777_amd as dl
    import workloads as wl
    inst = wl.cadence_base(chain, n_users=n_users, n_items=n_items)
    nxt = pool.submit(wl.cadence_next, inst, 1)
    prob = dl.Problem.from_instance(inst)
    lam, st = prob.solve(**COLD)
    rows = []
    for d in range(1, days + 1):
        today = nxt.result()
        if d < days:
            nxt = pool.submit(wl.cadence_next, today, d + 1)
        prob.update(c=today.c, b=today.b)
        F, _ = ws.features(prob, lam, inst.b)
        lam_new, st = prob.solve(lam0=lam, **FINAL)
        if st["status"] != 0:
            log(f"chain {chain} day {d}: status {st['status']} gap {st['rel_gap']:.2e}")
        rows.append((F.cpu().numpy(), (lam_new - lam).cpu().numpy(), st["iters"]))
        inst, lam = today, lam_new
    del prob
    torch.cuda.synchronize()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--chains", type=int, default=100)
    ap.add_argument("--days", type=int, default=20)
    ap.add_argument("--users", type=int, default=1_000_000)
    ap.add_argument("--items", type=int, default=5000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--hidden", type=int, default=256)
    ap.add_argument("--max-seconds", type=float, default=0.0,
                    help="stop collecting new chains after this many seconds (0 = no limit)")
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2606_07777_amd", "weights", "warmstart.npz"))
    args = ap.parse_args()

    import torch

    from paper_2606_07777_amd.learned import WarmStart
    torch.cuda.set_device(0)
    ws = WarmStart(hidden=args.hidden)
    t0 = time.time()
    chains, iters = [], []
    with ThreadPoolExecutor(max_workers=1) as pool:
        for k in range(args.chains):
            rows = collect_chain(CHAIN_SEED0 + k, args.days, args.users, args.items, ws, pool)
            chains.append(rows)
            iters.extend(r[2] for r in rows)
            el = time.time() - t0
            log(f"chain {k + 1}/{args.chains} collected ({el:.0f}s); "
                f"previous-day solves: mean {np.mean(iters):.0f} iterations")
            if args.max_seconds and el * (k + 2) / (k + 1) > args.max_seconds and k + 1 < args.chains:
                log(f"time budget reached: {k + 1} chains collected")
                break
    collect_s = time.time() - t0
    # the last 10% of the chains validate
    n_val = max(1, len(chains) // 10)
    train = [r for rows in chains[:len(chains) - n_val] for r in rows]
    val = [r for rows in chains[len(chains) - n_val:] for r in rows]
    Xtr = np.concatenate([r[0] for r in train])
    Ttr = np.concatenate([r[1] for r in train])
    Xva = np.concatenate([r[0] for r in val])
    Tva = np.concatenate([r[1] for r in val])
    log(f"{Xtr.shape[0]} training rows, {Xva.shape[0]} validation rows; std of the dual move {Ttr.std():.3e}")
    hist = ws.fit(Xtr, Ttr, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    # validation: mean squared error of the predicted move against doing nothing
    pred = []
    Xv = torch.from_numpy(Xva).cuda()
    for r0 in range(0, Xv.shape[0], ws.max_batch):
        pred.append(ws.net.forward(Xv[r0:r0 + ws.max_batch]).double().cpu().numpy() * ws.s)
    pred = np.concatenate(pred)
    mse_model = float(np.mean((pred - Tva) ** 2))
    mse_zero = float(np.mean(Tva ** 2))
    log(f"validation: mse {mse_model:.3e} vs {mse_zero:.3e} for the previous day's duals "
        f"(explained {1 - mse_model / mse_zero:.1%})")
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    ws.save(args.out)
    print(json.dumps({"rows_train": int(Xtr.shape[0]), "rows_val": int(Xva.shape[0]), "final_loss": hist[-1],
                      "val_mse": mse_model, "val_mse_previous": mse_zero, "collect_s": collect_s,
                      "train_s": time.time() - t0 - collect_s, "chains": len(chains), "days": args.days,
                      "users": args.users, "items": args.items,
                      "out": os.path.relpath(args.out, ROOT)}), flush=True)


if __name__ == "__main__":
    main()
