// Host-only helper of the batched launch: cutting one instance's tasks into
// workgroup ranges of equal estimated time.  Plain C++ (no HIP), so the rule
// can be compiled and checked on its own.
#pragma once

#include <stdint.h>

#include <algorithm>
#include <vector>

// Measured cost of one instance's pass: workgroup ranges [b[k], b[k+1]) and
// the clock ticks each took.  Empty = not measured.
struct dl_inst_profile {
  std::vector<int64_t> b;  // K + 1 nondecreasing task indices, b[0] = 0, b[K] = T
  std::vector<double> ticks;  // K
};

// Task boundaries (w + 1 entries, 0 .. T) of w workgroups with equal estimated
// time.  A task weighs its cost-model weight; inside each measured range the
// weights are scaled so that the range adds up to its measured time (at least
// one tick).  `cm` holds the prefix sums of the model weights (T + 1 entries).
// Boundary q falls before the first task whose weight midpoint reaches q/w of
// the total, found by binary search on the nondecreasing weighted prefix sum.
inline std::vector<int64_t> dl_split_tasks(int w, const dl_inst_profile& pr, const std::vector<double>& cm) {
  const int64_t T = (int64_t)cm.size() - 1;
  const size_t K = pr.ticks.size();
  // per measured range: ticks per unit of model weight, and the weighted sum before it
  std::vector<double> f(K), before(K + 1, 0.0);
  for (size_t k = 0; k < K; ++k) {
    const double mc = cm[(size_t)pr.b[k + 1]] - cm[(size_t)pr.b[k]];
    f[k] = mc > 0.0 ? std::max(pr.ticks[k], 1.0) / mc : 0.0;
    before[k + 1] = before[k] + f[k] * mc;
  }
  // weighted prefix sum over tasks [0, t)
  auto W = [&](int64_t t) -> double {
    if (K == 0) return cm[(size_t)t];
    // the range holding task t: the last k with b[k] <= t
    const size_t k = (size_t)(std::upper_bound(pr.b.begin(), pr.b.end() - 1, t) - pr.b.begin()) - 1;
    if (k >= K) return before[K];
    return before[k] + f[k] * (cm[(size_t)t] - cm[(size_t)pr.b[k]]);
  };
  const double tot = W(T);
  std::vector<int64_t> bounds((size_t)w + 1, 0);
  int64_t lo = 0;
  for (int q = 1; q < w; ++q) {
    const double target = tot * (double)q / (double)w;
    // smallest t in [lo, T) with 0.5 (W(t) + W(t + 1)) >= target, else T
    int64_t a = lo, b = T;
    while (a < b) {
      const int64_t mid = a + (b - a) / 2;
      if (0.5 * (W(mid) + W(mid + 1)) < target)
        a = mid + 1;
      else
        b = mid;
    }
    bounds[(size_t)q] = a;
    lo = a;
  }
  bounds[(size_t)w] = T;
  return bounds;
}
