// ems_geometry.cpp -- host construction of the box geometry's BVH.
#include "ems_geometry.hpp"

#include <math.h>

#include <algorithm>

namespace ems {

namespace {

// single-precision bound below (above) x with a relative margin, so that
// node tests done with reciprocals stay conservative
float widen_down(double x) {
  const double m = x - 1e-6 * (fabs(x) > 1.0 ? fabs(x) : 1.0);
  float f = (float)m;
  while ((double)f > m) f = nextafterf(f, -INFINITY);
  return f;
}
float widen_up(double x) {
  const double m = x + 1e-6 * (fabs(x) > 1.0 ? fabs(x) : 1.0);
  float f = (float)m;
  while ((double)f < m) f = nextafterf(f, INFINITY);
  return f;
}

struct Builder {
  const double *lo, *hi;
  std::vector<uint32_t> ids;
  BvhHost* out;
  int max_depth = 0;

  // node `at` covers ids[first, first + count)
  void make(uint32_t at, uint32_t first, uint32_t count, int depth) {
    max_depth = depth > max_depth ? depth : max_depth;
    double blo[3] = {INFINITY, INFINITY, INFINITY}, bhi[3] = {-INFINITY, -INFINITY, -INFINITY};
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t i = first; i < first + count; ++i) {
      const uint32_t b = ids[i];
      for (int k = 0; k < 3; ++k) {
        blo[k] = std::min(blo[k], lo[3 * b + k]);
        bhi[k] = std::max(bhi[k], hi[3 * b + k]);
        const double c = 0.5 * (lo[3 * b + k] + hi[3 * b + k]);
        clo[k] = std::min(clo[k], c);
        chi[k] = std::max(chi[k], c);
      }
    }
    BvhNode nd;
    for (int k = 0; k < 3; ++k) {
      nd.lo[k] = widen_down(blo[k]);
      nd.hi[k] = widen_up(bhi[k]);
    }
    if (count <= kBvhLeaf) {
      nd.a = first;
      nd.count = count;
      out->node[at] = nd;
      return;
    }
    int ax = 0;
    for (int k = 1; k < 3; ++k)
      if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
    const uint32_t half = count / 2;
    auto key = [&](uint32_t b) { return lo[3 * b + ax] + hi[3 * b + ax]; };
    std::nth_element(ids.begin() + first, ids.begin() + first + half, ids.begin() + first + count,
                     [&](uint32_t x, uint32_t y) { return key(x) < key(y) || (key(x) == key(y) && x < y); });
    const uint32_t left = (uint32_t)out->node.size();
    out->node.resize(left + 2);
    nd.a = left;
    nd.count = 0;
    out->node[at] = nd;
    make(left, first, half, depth + 1);
    make(left + 1, first + half, count - half, depth + 1);
  }
};

}  // namespace

bool build_bvh(const double* lo, const double* hi, uint32_t n, BvhHost& out, std::string& err) {
  out.node.assign(1, BvhNode{});
  out.box.resize((size_t)n * 6);
  for (uint32_t b = 0; b < n; ++b)
    for (int k = 0; k < 3; ++k) {
      out.box[(size_t)b * 6 + k] = lo[3 * b + k];
      out.box[(size_t)b * 6 + 3 + k] = hi[3 * b + k];
    }
  Builder bd;
  bd.lo = lo;
  bd.hi = hi;
  bd.out = &out;
  bd.ids.resize(n);
  for (uint32_t b = 0; b < n; ++b) bd.ids[b] = b;
  bd.make(0, 0, n, 0);
  out.leaf = bd.ids;
  // a depth-first walk that pushes both children holds at most depth + 1
  // entries
  if (bd.max_depth + 1 > kBvhStack) {
    err = "box hierarchy deeper than the traversal stack";
    return false;
  }
  return true;
}

}  // namespace ems
