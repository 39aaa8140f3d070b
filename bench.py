"""Benchmark of the dual-ascent hot path on one MI355X.

A step is one accelerated dual iteration: the gradient pass over every nonzero
(gather lam, closed-form primal, per-user projection, per-item reduction) plus
the fused item-space update.  The workload is the production-shape instance:
10M users x 10k items, degree round(lognormal(4.2, 0.6)) clipped to [1,2000],
Zipf(1.1) item popularity, c = -U(0,1) * popularity weight, a = 1, b = 0.3 n_j,
user simplex sum <= 1.  Inputs are generated on the host and copied to HBM
before any timing.

Prints one JSON line (the metric is nnz*iterations per second over the timed
steps) with the roofline of the dominant kernel and a CPU-oracle baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_instance(args):
    import workloads
    t = time.time()
    if args.workload == "production":
        inst = workloads.production(n_users=args.users, n_items=args.items)
        desc = (f"production {args.users} users x {args.items} items, degree lognormal(4.2,0.6) clipped "
                f"[1,2000], Zipf(1.1) items, a=1, b=0.3 n_j, simplex<=1")
    elif args.workload == "appendix_a":
        inst = workloads.appendix_a(seed=0, n_users=args.users, n_items=args.items, nu=args.nu)
        desc = (f"appendix-A construction {args.users} users x {args.items} items, nu={args.nu}, lognormal "
                f"breadth/value/scale, a = s_j c_ij stored, greedy-load b, simplex<=1")
    elif args.workload == "two_family":
        inst = workloads.two_family(seed=0, n_users=args.users, n_items=args.items)
        desc = (f"two coupling families {args.users} users x {args.items} items (budget a ~ lognormal(0,0.5), "
                f"b = 0.2 sum a; count cap a = 1, b = 0.3 n_j), degree Poisson(10), uniform items, box [0,1]")
    else:
        inst = workloads.tiny_plain(seed=0, binding=True)
        desc = "tiny_plain 10k users x 100 items, binding capacities"
    log(f"generated {desc}: nnz {inst.nnz} in {time.time() - t:.1f}s")
    return inst, desc


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha1()
    for f in ("dl_grad.hip", "dl_grad_kernels.h", "dl_grad_variant.hip", "dl_common.h"):
        h.update(open(os.path.join(ROOT, "paper_2606_07777_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(args):
    """HBM bytes per gradient pass from the committed rocprofv3 counter summary of this
    storage form, when it was taken on the current kernel source and the production
    workload; otherwise None."""
    name = "grad_pass_production_traffic.json" if args.storage == "f32" else "grad_pass_production_bf16_traffic.json"
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path) or args.workload != "production" or args.layout != "bucketed":
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha1") != kernel_source_hash():
        return None
    return rec.get("traffic_bytes_per_pass")


def host_cpu():
    """Model name, logical CPUs and physical cores of this host (from /proc/cpuinfo)."""
    model, cores = "unknown", set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model == "unknown":
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None:
            cores.add((phys, core))
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(), "physical_cores": len(cores) or None}


def oracle_rate(sample, budget_s: float):
    """(nnz*iter/s, iterations, seconds) of the FP64 oracle on sample within about budget_s."""
    import oracle
    # marginal cost of an iteration: one call of 1 iteration and one of 3
    t = time.time()
    oracle.solve(sample, [1e-2], [1], jacobi=True, check_every=0)
    t1 = time.time() - t
    t = time.time()
    oracle.solve(sample, [1e-2], [3], jacobi=True, check_every=0)
    per = max((time.time() - t - t1) / 2, 1e-3)
    iters = max(1, min(300, int(budget_s / per)))
    t = time.time()
    oracle.solve(sample, [1e-2], [iters], jacobi=True, check_every=0)
    el = time.time() - t
    return sample.nnz * iters / el, iters, el


def cpu_rate_child(path: str, budget_s: float):
    """Child process of cpu_baseline: the oracle on a saved sample with the
    thread count its environment sets (prints one JSON line)."""
    import numpy as np
    import workloads
    z = np.load(path)
    sample = workloads.Instance("sample", int(z["n_users"]), int(z["n_items"]), 1, z["row_ptr"], z["item_idx"],
                                z["c"], None, z["b"], "simplex_le", 1.0)
    rate, iters, el = oracle_rate(sample, budget_s)
    print(json.dumps({"rate": rate, "iters": iters, "seconds": el}), flush=True)


def cpu_baseline(inst, budget_s: float):
    """The FP64 oracle on a bounded sample of the same instance (its first S
    users), with every host thread and, in a child process, with one thread."""
    import subprocess
    import tempfile

    import numpy as np
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    S = min(inst.n_users, 500_000)
    sample = inst.user_slice(0, S)
    # b scaled with the sample so the capacities keep binding
    sample.b = inst.b * (S / inst.n_users)
    rate, iters, el = oracle_rate(sample, budget_s)
    out = {"value": rate, "unit": "nnz*iter/s", "cores": threads, "kind": "oracle",
           "sample": f"first {S} users ({sample.nnz} nnz) of the same instance, b scaled by {S}/{inst.n_users}, "
                     f"{iters} FP64 iterations in {el:.1f}s", "host": host_cpu()}
    # one thread: the same sample in a child process with OMP_NUM_THREADS=1
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "sample.npz")
        np.savez(path, n_users=S, n_items=inst.n_items, row_ptr=sample.row_ptr, item_idx=sample.item_idx,
                 c=sample.c, b=sample.b)
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-rate-child", path,
                            "--cpu-budget", str(budget_s)], env=env, capture_output=True, text=True,
                           timeout=max(120.0, 8 * budget_s))
        if r.returncode == 0:
            one = json.loads(r.stdout.strip().splitlines()[-1])
            out["one_thread"] = {"value": one["rate"], "iters": one["iters"], "seconds": one["seconds"]}
        else:
            out["one_thread"] = {"error": r.stderr[-400:]}
    return out


def six_stage(prob, iters):
    """The six-stage schedule gamma = 1e3, 1e2, 10, 1, 0.1, 0.01 (the paper's
    solution-quality runs), each stage warm-started with momentum reset; the
    certificate (primal, dual, relative gap, max slack) after every stage."""
    import torch
    s = prob.solver()
    rows = []
    t0 = time.perf_counter()
    for g in (1e3, 1e2, 1e1, 1e0, 1e-1, 1e-2):
        s.set_stage(g, 1.0, True)
        s.step(iters)
        c = s.certificate()
        torch.cuda.synchronize()
        rows.append({"gamma": g, "iters": iters, "primal": c["primal_obj"], "dual": c["dual_obj"],
                     "rel_gap": c["rel_gap"], "max_slack": c["max_slack"], "elapsed_s": time.perf_counter() - t0})
        log(f"six-stage gamma {g:g}: primal {c['primal_obj']:.6e} dual {c['dual_obj']:.6e} "
            f"gap {c['rel_gap']:.3e} slack {c['max_slack']:.3e}")
    return rows


def ablation(args):
    """The paper's two algorithmic ablations on its Appendix-A construction
    (users = sources, items = destinations): |L - L_hat| of the dual value at
    gamma = 0.01 every 10 iterations for (1) Jacobi row scaling on vs off at
    fixed gamma = 0.01, and (2) gamma decayed 0.16 -> 0.01 (halved every 25
    iterations, step scaled with gamma, momentum reset) vs fixed gamma = 0.01,
    both with Jacobi.  L_hat is the dual value at gamma = 0.01 after a long
    continuation solve.  Prints its own JSON line."""
    import numpy as np
    import torch

    import paper_2606_07777_amd as dl
    import workloads
    t = time.time()
    inst = workloads.appendix_a(seed=1, n_users=args.users, n_items=args.items, nu=args.nu)
    log(f"appendix-A instance {args.users} x {args.items}, nnz {inst.nnz} in {time.time() - t:.1f}s")
    torch.cuda.set_device(0)
    g_final = 1e-2
    n_it = args.ablation_iters
    probs = {True: dl.Problem.from_instance(inst, jacobi=True), False: dl.Problem.from_instance(inst, jacobi=False)}
    del inst
    pj = probs[True]
    # reference: long continuation solve, then the dual value at gamma = 0.01
    lam_ref, st = pj.solve([0.16, 0.08, 0.04, 0.02, 0.01], [200, 200, 200, 200, args.ablation_ref_iters],
                           check_every=0)
    L_hat = pj.dual_grad(lam_ref, g_final, want_obj=True)[0]
    log(f"L_hat = {L_hat:.10e} after {st['iters']} iterations")

    def curve(prob, schedule):
        s = prob.solver()
        out = []
        it = 0
        for gamma, k in schedule:
            s.set_stage(gamma, 1.0, True)
            done = 0
            while done < k:
                step = min(10 - it % 10, k - done)
                s.step(step)
                done += step
                it += step
                if it % 10 == 0:
                    L = prob.dual_grad(s.lam(), g_final, want_obj=True)[0]
                    out.append([it, abs(L - L_hat)])
        return out

    fixed = [(g_final, n_it)]
    decay = [(0.16, 25), (0.08, 25), (0.04, 25), (0.02, 25), (g_final, n_it - 100)]
    res = {"metric": "|L - L_hat| of the dual value at gamma = 0.01 every 10 iterations", "L_hat": L_hat,
           "jacobi_on": curve(probs[True], fixed), "jacobi_off": curve(probs[False], fixed),
           "continuation": curve(probs[True], decay), "fixed_gamma": None,
           "config": {"workload": f"appendix-A construction {args.users} x {args.items}, nu={args.nu}",
                      "iterations": n_it}}
    res["fixed_gamma"] = res["jacobi_on"]
    for k in ("jacobi_on", "jacobi_off", "continuation"):
        c = res[k]
        log(f"{k}: " + ", ".join(f"{i}:{v:.3e}" for i, v in c[::max(1, len(c) // 8)]))
    print(json.dumps(res), flush=True)


def learned_eval(args, log=log):
    """Time to a 1e-4 certified gap on drifting days: cold start over the
    continuation schedule, the previous day's duals at the final gamma, and the
    judged learned start ({learned, previous, cold} at the final gamma).  Times
    include the learned path's gradient pass, feature pass and network."""
    import numpy as np
    import torch

    import paper_2606_07777_amd as dl
    import workloads as wl
    from paper_2606_07777_amd.learned import WarmStart
    cold = dict(gammas=[1e-1, 1e-2, 1e-3], iters=[300, 300, -1], tol=1e-4, max_iters=20000, check_every=10)
    final = dict(gammas=[1e-3], iters=[-1], tol=1e-4, max_iters=20000, check_every=10)
    ws = WarmStart.load(args.learned)
    days = []

    def timed(fn):
        torch.cuda.synchronize()
        t = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t

    for ch in range(args.eval_chains):
        chain = 6000 + ch
        inst = wl.cadence_base(chain, n_users=args.eval_users, n_items=args.eval_items)
        prob = dl.Problem.from_instance(inst)
        (lam, st), t = timed(lambda: prob.solve(**cold))
        log(f"eval chain {chain} day 0: cold {st['iters']} iterations, {t:.2f}s, gap {st['rel_gap']:.1e}")
        for d in range(1, args.eval_days + 1):
            today = wl.cadence_next(inst, d)
            prob.update(c=today.c, b=today.b)
            (lc, sc), tc = timed(lambda: prob.solve(**cold))
            (lp, sp), tp = timed(lambda: prob.solve(lam0=lam, **final))
            (ll, sl, info), tl = timed(lambda: ws.solve(prob, lam, inst.b, **final))
            rec = {"chain": chain, "day": d,
                   "cold": {"s": tc, "iters": sc["iters"], "gap": sc["rel_gap"], "status": sc["status"]},
                   "previous": {"s": tp, "iters": sp["iters"], "gap": sp["rel_gap"], "status": sp["status"]},
                   "learned": {"s": tl, "iters": sl["iters"], "gap": sl["rel_gap"], "status": sl["status"],
                               "chosen": info["chosen"], "predict_s": info["predict_s"]}}
            days.append(rec)
            log(f"eval chain {chain} day {d}: cold {sc['iters']} it {tc:.2f}s | previous {sp['iters']} it "
                f"{tp:.2f}s | learned ({info['chosen']}) {sl['iters']} it {tl:.2f}s")
            inst, lam = today, ll
        del prob
    def mean(k, f):
        return float(np.mean([r[k][f] for r in days]))
    return {"workload": f"drifting days of a {args.eval_users} x {args.eval_items} matching instance "
                        f"(Poisson(10) degrees, c=-U(0,1), binding b=0.5 I/J; c, b drift 5%/day)",
            "chains": args.eval_chains, "days_per_chain": args.eval_days, "weights": os.path.relpath(args.learned, ROOT),
            "mean_s": {k: mean(k, "s") for k in ("cold", "previous", "learned")},
            "mean_iters": {k: mean(k, "iters") for k in ("cold", "previous", "learned")},
            "speedup_learned_vs_cold": mean("cold", "s") / max(mean("learned", "s"), 1e-12),
            "speedup_learned_vs_previous": mean("previous", "s") / max(mean("learned", "s"), 1e-12),
            "days": days}


def member_rates(members, probs, gamma=1e-1, warm=30):
    """Solo gradient-pass time of every batch member (HIP events around 30 passes,
    after `warm` untimed iterations at gamma 0.1 and, when gamma differs, 5 more at
    gamma) against one batched iteration.  Prints its own JSON line."""
    import torch

    import paper_2606_07777_amd as dl
    rows = []
    for m, p in zip(members, probs):
        s = p.solver()
        s.set_stage(1e-1)
        s.step(warm)
        if gamma != 1e-1:
            s.set_stage(gamma)
            s.step(5)
        s.enable_timing(True)
        s.step(30)
        t = s.timing()
        ms = t["grad_ms_total"] / t["n_grad"]
        rows.append({"users": m.n_users, "items": m.n_items, "nnz": m.nnz, "pass_ms": ms,
                     "bytes_per_pass": p.info()["bytes_per_pass"],
                     "GBps": p.info()["bytes_per_pass"] / (ms * 1e-3) / 1e9})
        del s
    batch = dl.Batch(probs)
    _, _ = batch.solve(gammas=[1e-1], iters=[60], check_every=0, autotune=2)
    torch.cuda.synchronize()
    tr = batch.tune()
    nnz = sum(r["nnz"] for r in rows)
    solo_ms = sum(r["pass_ms"] for r in rows)
    for r in rows:
        log(f"member I={r['users']} J={r['items']} nnz={r['nnz']}: {r['pass_ms']:.4f} ms, {r['GBps']:.0f} GB/s")
    out = {"metric": "gradient-pass time of the uneven batch members, solo vs one batched iteration", "unit": "ms",
           "solo_sum_ms": solo_ms, "batched_iteration_ms": tr["pass_ms_tuned"],
           "solo_GBps_min": min(r["GBps"] for r in rows), "solo_GBps_max": max(r["GBps"] for r in rows),
           "batched_GBps": sum(r["bytes_per_pass"] for r in rows) / (tr["pass_ms_tuned"] * 1e-3) / 1e9,
           "members": rows,
           "config": {"workload": f"uneven batch of {len(members)}", "gamma": gamma, "warm_iterations": warm}}
    print(json.dumps(out), flush=True)


def batch_bench(args):
    """The uneven batch: 64 instances (users log-uniform in [5e4, 2e6], items
    log-uniform in [100, 5000], degree round(lognormal(3.5, 0.8)), uniform items,
    c = -U(0,1), a = 1, binding b = 0.5 I/J, simplex <= 1) solved to a 1e-4 gap
    (gamma 1e-1, 1e-2 for 300 iterations each, then 1e-3): as one batch (one
    launch per iteration phase for all live members) with the batch tuner (the
    default), again with the cost-model workgroup split, and as 64 sequential
    solo solves.  Prints its own JSON line."""
    import numpy as np
    import torch

    import paper_2606_07777_amd as dl
    import workloads as wl
    t = time.time()
    members = [wl.batch_member(k, binding=True, scale=args.batch_scale) for k in range(args.batch_n)]
    nnz = [m.nnz for m in members]
    log(f"generated {len(members)} members, {sum(nnz)} nnz, {sum(m.n_users for m in members)} users "
        f"in {time.time() - t:.1f}s")
    torch.cuda.set_device(0)
    probs = [dl.Problem.from_instance(m, jacobi=True) for m in members]
    if args.member_rates:
        return member_rates(members, probs, args.rates_gamma, args.rates_warmup)
    sched = dict(gammas=[1e-1, 1e-2, 1e-3], iters=[300, 300, -1], tol=1e-4, max_iters=20000, check_every=10)
    batch = dl.Batch(probs)
    # untimed warm-up (first launches of every kernel)
    batch.solve(gammas=[1e-1, 1e-3], iters=[60, 10], check_every=10, autotune=1)
    torch.cuda.synchronize()
    # the batched solve as shipped: the tuner times the solve's own iterations
    t0 = time.perf_counter()
    lam_b, st_b = batch.solve(autotune=args.batch_tune, **sched)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    tune = batch.tune() if args.batch_tune > 0 else None
    log(f"batch (tuner rounds {args.batch_tune}): {t_batch:.2f}s, "
        f"iterations {min(s['iters'] for s in st_b)}..{max(s['iters'] for s in st_b)}; tuner {tune}")
    # the same with the cost-model split throughout
    t0 = time.perf_counter()
    _, st_t = batch.solve(autotune=0, **sched)
    torch.cuda.synchronize()
    t_model = time.perf_counter() - t0
    log(f"batch, cost-model split: {t_model:.2f}s")
    if tune is not None:
        # the tuner's own cost: 60 iterations with and without it
        short = dict(gammas=[1e-1], iters=[60], check_every=0)
        t0 = time.perf_counter()
        batch.solve(autotune=0, **short)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        t0 = time.perf_counter()
        batch.solve(autotune=args.batch_tune, **short)
        torch.cuda.synchronize()
        tune["overhead_s"] = time.perf_counter() - t0 - t_plain
        log(f"tuner overhead {tune['overhead_s']:.3f}s")
    if args.no_batch_solo:
        out = {"metric": "time to a 1e-4 gap for every member of the uneven batch", "unit": "s",
               "batch_s": t_batch, "batch_cost_model_s": t_model, "batch_tuner": tune,
               "batch_nnz_iter_per_s": sum(n * s["iters"] for n, s in zip(nnz, st_b)) / t_batch,
               "members": len(members), "nnz": int(sum(nnz)),
               "converged": int(sum(s["status"] == 0 for s in st_b)),
               "config": {"workload": f"uneven batch of {len(members)} (users scale {args.batch_scale})"}}
        print(json.dumps(out), flush=True)
        return
    t0 = time.perf_counter()
    st_s = []
    for p in probs:
        st_s.append(p.solve(**sched)[1])
    torch.cuda.synchronize()
    t_solo = time.perf_counter() - t0
    log(f"solo: {t_solo:.2f}s")
    # the solo solves again with each problem's own workgroup tuner (it keeps the
    # tuned split on the problem, so this runs after the untuned solves)
    t0 = time.perf_counter()
    st_st = []
    for p in probs:
        st_st.append(p.solve(autotune_rounds=2, **sched)[1])
    torch.cuda.synchronize()
    t_solo_tuned = time.perf_counter() - t0
    log(f"solo, tuned: {t_solo_tuned:.2f}s")
    work_b = sum(n * s["iters"] for n, s in zip(nnz, st_b))
    work_s = sum(n * s["iters"] for n, s in zip(nnz, st_s))
    same = all(a["iters"] == b["iters"] == c["iters"] == d["iters"] for a, b, c, d in zip(st_b, st_s, st_t, st_st))
    for k, (a, b, c, d) in enumerate(zip(st_b, st_s, st_t, st_st)):
        if not a["iters"] == b["iters"] == c["iters"] == d["iters"]:
            log(f"member {k}: iterations batch {a['iters']} (gap {a['rel_gap']:.9e}), solo {b['iters']} "
                f"(gap {b['rel_gap']:.9e}), batch cost-model {c['iters']} (gap {c['rel_gap']:.9e}), "
                f"solo tuned {d['iters']} (gap {d['rel_gap']:.9e})")
    out = {"metric": "time to a 1e-4 gap for every member of the uneven batch", "unit": "s",
           "batch_s": t_batch, "batch_cost_model_s": t_model, "batch_tuner": tune,
           "solo_sequential_s": t_solo, "speedup": t_solo / t_batch,
           "solo_sequential_tuned_s": t_solo_tuned, "speedup_vs_tuned_solo": t_solo_tuned / t_batch,
           "batch_nnz_iter_per_s": work_b / t_batch, "solo_nnz_iter_per_s": work_s / t_solo,
           "same_iterations_as_solo": same, "members": len(members), "nnz": int(sum(nnz)),
           "converged": int(sum(s["status"] == 0 for s in st_b)),
           "max_rel_gap": float(max(s["rel_gap"] for s in st_b)),
           "config": {"workload": f"uneven batch of {len(members)} (users scale {args.batch_scale})"}}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--workload", default="production",
                    choices=["production", "tiny", "batch", "appendix_a", "ablation", "two_family"])
    ap.add_argument("--ablation-iters", type=int, default=500)
    ap.add_argument("--ablation-ref-iters", type=int, default=4000)
    ap.add_argument("--nu", type=float, default=80.0, help="mean nonzeros per user of the appendix-A workload")
    ap.add_argument("--six-stage", type=int, default=0,
                    help="also run the six-stage gamma schedule 1e3..1e-2 with this many iterations per stage")
    ap.add_argument("--batch-n", type=int, default=64)
    ap.add_argument("--batch-scale", type=float, default=1.0)
    ap.add_argument("--member-rates", action="store_true",
                    help="with --workload batch: per-member solo pass rates against one batched pass")
    ap.add_argument("--no-batch-solo", action="store_true",
                    help="batch workload: time the batched solves only (no sequential solo solves)")
    ap.add_argument("--rates-gamma", type=float, default=1e-1, help="--member-rates: gamma of the timed passes")
    ap.add_argument("--rates-warmup", type=int, default=30, help="--member-rates: untimed iterations at gamma 0.1 first")
    ap.add_argument("--timed-gamma", type=float, default=1e-2,
                    help="gamma of the timed steps (after --warmup iterations at 0.1; 5 more at this gamma if it differs)")
    ap.add_argument("--batch-tune", type=int, default=2,
                    help="balancing rounds of the batch tuner (0: cost-model split only)")
    ap.add_argument("--users", type=int, default=10_000_000)
    ap.add_argument("--items", type=int, default=10_000)
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16"])
    ap.add_argument("--layout", default="bucketed", choices=["bucketed", "wavefront"],
                    help="user-to-lane mapping; wavefront = one wavefront per user (baseline layout)")
    ap.add_argument("--wg-per-cu", type=int, default=8, help="largest workgroups-per-CU grid the tuner may pick")
    ap.add_argument("--tune-rounds", type=int, default=10, help="workgroup-split balancing rounds (0 = off)")
    ap.add_argument("--copy-ref-mb", type=int, default=0,
                    help="run a device copy of this size first (reference kernel for counter scaling)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--cpu-rate-child", default=None, help=argparse.SUPPRESS)
    ap.add_argument("--solve", action="store_true", help="also time a cold solve to a 1e-4 certified gap")
    ap.add_argument("--learned", default=os.path.join(ROOT, "paper_2606_07777_amd", "weights", "warmstart.npz"),
                    help="warm-start network for the time-to-gap comparison ('' = skip)")
    ap.add_argument("--eval-users", type=int, default=10_000_000)
    ap.add_argument("--eval-items", type=int, default=10_000)
    ap.add_argument("--eval-chains", type=int, default=4)
    ap.add_argument("--eval-days", type=int, default=5)
    args = ap.parse_args()

    if args.cpu_rate_child:
        return cpu_rate_child(args.cpu_rate_child, args.cpu_budget)
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; multi-GPU runs are not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    if args.workload == "batch":
        return batch_bench(args)
    if args.workload == "ablation":
        return ablation(args)

    import numpy as np
    import torch

    import paper_2606_07777_amd as dl

    inst, desc = make_instance(args)
    torch.cuda.set_device(0)
    if args.copy_ref_mb:
        n = args.copy_ref_mb * 1024 * 1024 // 4
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log(f"reference copy: {args.copy_ref_mb} MiB read, {args.copy_ref_mb} MiB written")
    t = time.time()
    prob = dl.Problem.from_instance(inst, storage=args.storage, jacobi=True, wg_per_cu=args.wg_per_cu,
                                    layout=args.layout)
    torch.cuda.synchronize()
    info = prob.info()
    log(f"problem created in {time.time() - t:.1f}s: {info['n_workgroups']} workgroups, {info['n_tasks']} tasks, "
        f"buckets {list(zip(info['bucket_glog'], info['bucket_users']))}")

    s = prob.solver()
    # warm-up: the first continuation stage, so the timed steps see a realistic active set
    s.set_stage(1e-1, 1.0, True)
    s.step(args.warmup)
    if args.timed_gamma != 1e-1:
        s.set_stage(args.timed_gamma, 1.0, True)
        s.step(5)
    tune = None
    if args.tune_rounds > 0:
        tune = s.autotune(args.tune_rounds)
        log(f"workgroup split tuned: {tune}")
    torch.cuda.synchronize()
    log("warm-up done")

    s.enable_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(args.steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tm = s.timing()
    s.enable_timing(False)
    ms_step = el * 1e3 / args.steps
    grad_ms = tm["grad_ms_total"] / max(tm["n_grad"], 1)
    upd_ms = tm["update_ms_total"] / max(tm["n_update"], 1)
    bytes_pass = info["bytes_per_pass"]
    achieved = bytes_pass / (grad_ms * 1e-3) / 1e9
    value = inst.nnz * args.steps / el
    cert = s.certificate()
    log(f"{args.steps} steps: {ms_step:.3f} ms/step, grad pass {grad_ms:.3f} ms ({achieved:.0f} GB/s), "
        f"update {upd_ms:.3f} ms; gap at gamma={args.timed_gamma:g} after warm-up: {cert['rel_gap']:.3e}")
    # the practical read ceiling: a streaming read of as many bytes as one pass reads
    ceiling = dl.read_bandwidth(int(bytes_pass), reps=20)
    torch.cuda.empty_cache()
    log(f"streaming read of {bytes_pass / 1e9:.2f} GB: {ceiling:.0f} GB/s (pass at {achieved / ceiling:.1%} of it)")

    out = {
        "metric": "nnz*iter/s of the dual-gradient pass plus fused update at 10M users x 10k items",
        "value": value,
        "unit": "nnz*iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.storage == "f32" else "bf16-storage/f32",
        "data": "synthetic",
        "config": {"workload": desc, "n_users": inst.n_users, "n_items": inst.n_items, "nnz": inst.nnz,
                   "storage": args.storage, "layout": args.layout, "gamma_timed": args.timed_gamma,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": measured_traffic(args),
                     "kernel": "grad_pass", "kernel_ms": grad_ms, "bytes_per_pass": bytes_pass,
                     "ceiling": {"GBps": ceiling, "frac": achieved / ceiling,
                                 "kernel": "dl_read_bandwidth: 16-byte nontemporal streaming reads of "
                                           "bytes_per_pass bytes"}},
        "update_ms": upd_ms,
        "schedule": tune,
    }
    del s
    if args.solve:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lam, st = prob.solve([1e-1, 1e-2, 1e-3], [300, 300, -1], tol=1e-4, max_iters=20000, check_every=10)
        torch.cuda.synchronize()
        out["cold_solve_production"] = {"cold_s": time.perf_counter() - t0, "iters": st["iters"], "rel_gap": st["rel_gap"],
                              "status": st["status"], "schedule": "gamma 1e-1,1e-2 (300 each) then 1e-3 to 1e-4 gap"}
        log(f"cold solve: {out['cold_solve_production']}")
    if args.six_stage:
        out["six_stage"] = six_stage(prob, args.six_stage)
    if args.learned and os.path.exists(args.learned) and args.workload == "production":
        del prob
        torch.cuda.empty_cache()
        out["time_to_gap"] = learned_eval(args)
    if not args.no_cpu_baseline:
        log("cpu baseline ...")
        out["cpu_baseline"] = cpu_baseline(inst, args.cpu_budget)
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
