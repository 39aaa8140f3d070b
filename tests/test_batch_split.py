"""Host logic of the batched launch: the split of one instance's tasks into
workgroup ranges of equal estimated time (paper_2606_07777_amd/csrc/dl_split.h).

The header is plain C++; it is compiled with g++ into a small driver that reads
cases on stdin.  Each result is checked against properties that define the
split, computed here from explicit per-task weights (a task's cost-model weight,
scaled inside each measured range so that the range sums to its measured time).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER_DIR = os.path.join(ROOT, "paper_2606_07777_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include "dl_split.h"
int main() {
  long long T, K; int w;
  while (std::scanf("%lld %d %lld", &T, &w, &K) == 3) {
    std::vector<double> cm((size_t)T + 1, 0.0);
    for (long long t = 0; t < T; ++t) { double c; std::scanf("%lf", &c); cm[(size_t)t + 1] = cm[(size_t)t] + c; }
    dl_inst_profile pr;
    if (K > 0) {
      pr.b.resize((size_t)K + 1); pr.ticks.resize((size_t)K);
      for (long long k = 0; k <= K; ++k) { long long v; std::scanf("%lld", &v); pr.b[(size_t)k] = v; }
      for (long long k = 0; k < K; ++k) std::scanf("%lf", &pr.ticks[(size_t)k]);
    }
    std::vector<int64_t> b = dl_split_tasks(w, pr, cm);
    for (size_t q = 0; q < b.size(); ++q) std::printf("%lld ", (long long)b[q]);
    std::printf("\n");
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("split")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", HEADER_DIR, str(src), "-o", str(exe)], check=True)
    return str(exe)


def run(driver, cases):
    lines = []
    for cost, w, b, ticks in cases:
        lines.append(f"{len(cost)} {w} {len(ticks)}")
        lines.append(" ".join(repr(float(c)) for c in cost))
        if len(ticks):
            lines.append(" ".join(str(int(v)) for v in b))
            lines.append(" ".join(repr(float(v)) for v in ticks))
    out = subprocess.run([driver], input="\n".join(lines) + "\n", capture_output=True, text=True, check=True).stdout
    return [np.array([int(v) for v in ln.split()], dtype=np.int64) for ln in out.strip().splitlines()]


def task_weights(cost, b, ticks):
    """Explicit per-task weights: model weight, scaled per measured range."""
    wt = np.asarray(cost, dtype=np.float64).copy()
    for k in range(len(ticks)):
        lo, hi = b[k], b[k + 1]
        mass = wt[lo:hi].sum()
        if mass > 0:
            wt[lo:hi] *= max(ticks[k], 1.0) / mass
    return wt


def random_case(rng):
    T = int(rng.integers(0, 3000))
    cost = rng.integers(64, 700, size=T).astype(np.float64)
    w = int(rng.integers(1, 80))
    b, ticks = [], []
    if T > 0 and rng.random() < 0.7:
        K = int(rng.integers(1, 25))
        cuts = np.sort(rng.integers(0, T + 1, size=K - 1))
        b = [0] + [int(c) for c in cuts] + [T]
        ticks = [float(v) for v in rng.integers(0, 200000, size=K)]
    return cost, w, b, ticks


def check_split(bounds, cost, w, b, ticks):
    T = len(cost)
    assert len(bounds) == w + 1 and bounds[0] == 0 and bounds[-1] == T
    assert np.all(np.diff(bounds) >= 0)
    wt = task_weights(cost, b, ticks)
    run_before = np.concatenate([[0.0], np.cumsum(wt)])  # weight of tasks [0, t)
    tot = run_before[-1]
    eps = 1e-9 * max(tot, 1.0)
    for q in range(1, w):
        target = tot * q / w
        t = bounds[q]
        # every task before the boundary (after the previous one) has its midpoint below the target
        if t > bounds[q - 1]:
            assert run_before[t - 1] + 0.5 * wt[t - 1] < target + eps
        # the task at the boundary has its midpoint at or past it
        if t < T:
            assert run_before[t] + 0.5 * wt[t] >= target - eps
    # equal time: every range is within one task of the ideal share
    big = wt.max() if T else 0.0
    for q in range(w):
        share = run_before[bounds[q + 1]] - run_before[bounds[q]]
        assert share <= tot / w + big + eps


def test_split_properties_on_random_profiles(driver):
    rng = np.random.default_rng(20261202)
    cases = [random_case(rng) for _ in range(400)]
    for res, (cost, w, b, ticks) in zip(run(driver, cases), cases):
        check_split(res, cost, w, b, ticks)


def test_profile_proportional_to_the_model_changes_nothing(driver):
    """Measured times that are exactly twice the model weights give the
    cost-model split (powers of two keep the arithmetic exact)."""
    rng = np.random.default_rng(7)
    cases, plain = [], []
    for _ in range(100):
        T = int(rng.integers(1, 2000))
        cost = rng.integers(64, 700, size=T).astype(np.float64)
        w = int(rng.integers(1, 64))
        K = int(rng.integers(1, 12))
        b = [0] + sorted(int(c) for c in rng.integers(0, T + 1, size=K - 1)) + [T]
        ticks = [2.0 * cost[b[k]:b[k + 1]].sum() for k in range(K)]
        # an empty range measures one tick (the floor) but holds no tasks
        cases.append((cost, w, b, ticks))
        plain.append((cost, w, [], []))
    for r1, r2 in zip(run(driver, cases), run(driver, plain)):
        assert np.array_equal(r1, r2)


def test_split_follows_measured_time(driver):
    """Uniform model weights, but the second half measured 3x slower: the
    boundaries move so that each range holds a quarter of the measured time."""
    cost = np.full(1000, 100.0)
    b = [0, 500, 1000]
    ticks = [50000.0, 150000.0]  # 100 and 300 ticks per task
    (res,) = run(driver, [(cost, 4, b, ticks)])
    # total 200000 ticks; quarters end at 50000 (task 500), 100000, 150000
    assert res.tolist() == [0, 500, 667, 833, 1000]
    check_split(res, cost, 4, b, ticks)


def test_degenerate_inputs(driver):
    out = run(driver, [(np.zeros(0), 3, [], []), (np.array([5.0]), 4, [], []),
                       (np.array([1.0, 1.0, 1.0]), 1, [], [])])
    assert out[0].tolist() == [0, 0, 0, 0]
    assert out[1][0] == 0 and out[1][-1] == 1 and np.all(np.diff(out[1]) >= 0)
    assert out[2].tolist() == [0, 3]
