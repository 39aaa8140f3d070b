"""Trajectory parity at the full production shape: 10M users x 10k items
(degree lognormal(4.2, 0.6) clipped to [1, 2000], Zipf(1.1) item popularity,
about 0.8B nonzeros), the instance the benchmark times.

The GPU solver and the FP64 oracle (on the host's cores) run the start of the
continuation schedule from lam = 0: 20 iterations at gamma = 0.1, then the
stage switch (momentum reset) and 10 at gamma = 0.01, Jacobi on.  lam after
each stage must agree to 1e-5, norm-wise and element-wise.  The oracle takes
about 2 s per iteration here on 16 cores, so this is the slowest GPU test.
"""
import os
import time

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


def test_production_full_shape_prefix(dl, orc, wl):
    t = time.time()
    inst = wl.production()
    print(f"production instance: {inst.n_users} users, {inst.n_items} items, nnz {inst.nnz} "
          f"({time.time() - t:.1f}s)", flush=True)
    assert inst.n_users == 10_000_000 and inst.n_items == 10_000 and inst.nnz > 7.9e8
    prob = dl.Problem.from_instance(inst, jacobi=True)
    s = prob.solver()
    out = []
    for g, n in ((1e-1, 20), (1e-2, 10)):
        s.set_stage(g, 1.0, True)
        s.step(n)
        out.append(s.lam().cpu().numpy())
    prob.close()
    t = time.time()
    _, _, snaps, _ = orc.solve(inst, [1e-1, 1e-2], [20, 10], jacobi=True, check_every=0, snap_iters=[20, 30])
    host_s = time.time() - t
    threads = os.environ.get("OMP_NUM_THREADS", str(os.cpu_count()))
    print(f"oracle: 30 FP64 iterations in {host_s:.1f}s on {threads} threads "
          f"({inst.nnz * 30 / host_s:.3e} nnz*iter/s)", flush=True)
    for k, (lg, lo) in enumerate(zip(out, snaps)):
        rel = np.linalg.norm(lg - lo) / np.linalg.norm(lo)
        el = np.abs(lg - lo).max() / np.abs(lo).max()
        print(f"after {(20, 30)[k]} iterations: |lam| {np.linalg.norm(lo):.4e}, rel l2 {rel:.2e}, "
              f"max elementwise {el:.2e}", flush=True)
        assert np.linalg.norm(lo) > 0
        assert rel <= 1e-5 and el <= 1e-5
