// Host check of the range-table inverse used by the charged step: the node
// it finds (largest j <= jhi with R_j <= r, node 0 if none) must be the one
// a one-by-one walk down from jhi finds, for every walk length, for r on a
// node, below the table and anywhere inside it, for tables with runs of
// equal values, in FP64 and FP32.  Prints "<type>: <cases> cases,
// <mismatches> mismatches" per type; exit status 1 on any mismatch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "ems_step.hpp"

using namespace ems;

template <class R>
static int walk_one_by_one(int nodes, const R* Rt, R r, int jhi) {
  int lo = jhi > nodes - 1 ? nodes - 1 : jhi;
  while (lo > 0 && Rt[lo] > r) --lo;
  return lo > nodes - 2 ? nodes - 2 : lo;
}

template <class R>
static long check(const char* name) {
  const int nodes = 201;
  std::mt19937_64 g(7);
  std::uniform_real_distribution<double> u01(0.0, 1.0);
  long bad = 0, n = 0;
  for (int trial = 0; trial < 120; ++trial) {
    // non-decreasing tables, growing by 1-40% a node; every third has
    // repeated values
    std::vector<R> Rt(nodes);
    double acc = std::exp(-15.0 * u01(g));
    for (int j = 0; j < nodes; ++j) {
      if (!(trial % 3 == 0 && j % 7 == 3)) acc += acc * (0.01 + 0.39 * u01(g));
      Rt[j] = (R)acc;
    }
    StepEnv<R> e{};
    e.nodes = nodes;
    e.lnemin = (R)std::log(1e-3);
    e.dlog = (R)((std::log(1e8) - std::log(1e-3)) / (nodes - 1));
    const double l0 = std::log((double)Rt[0]), l1 = std::log((double)Rt[nodes - 1]);
    for (int jhi = 0; jhi <= nodes; ++jhi) {
      for (int q = 0; q < 200; ++q) {
        R r;
        if (q % 4 == 0) r = Rt[(size_t)(u01(g) * nodes) % nodes];
        else if (q % 4 == 1) r = (R)((double)Rt[0] * 1.5 * u01(g));
        else r = (R)std::exp(l0 - 1.0 + (l1 - l0 + 1.0) * u01(g));
        const int j = walk_one_by_one<R>(nodes, Rt.data(), r, jhi);
        const R want = std::exp(e.lnemin + (R)j * e.dlog + e.dlog * (r - Rt[j]) / (Rt[j + 1] - Rt[j]));
        const R got = inverse_range<R>(e, Rt.data(), r, jhi);
        ++n;
        if (!(got == want) && !(std::isnan((double)got) && std::isnan((double)want))) {
          if (bad < 5) std::printf("%s mismatch: table %d, jhi %d, r %.17g, node %d\n", name, trial, jhi, (double)r, j);
          ++bad;
        }
      }
    }
  }
  std::printf("%s: %ld cases, %ld mismatches\n", name, n, bad);
  return bad;
}

int main() {
  const long bad = check<double>("double") + check<float>("float");
  return bad != 0 ? 1 : 0;
}
