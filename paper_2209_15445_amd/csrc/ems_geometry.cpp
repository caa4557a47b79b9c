// ems_geometry.cpp -- host construction of the box geometry's BVH.
#include "ems_geometry.hpp"

#include <math.h>

#include <algorithm>
#include <map>

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

  static double area(const double* l, const double* h) {
    const double dx = h[0] - l[0], dy = h[1] - l[1], dz = h[2] - l[2];
    return 2.0 * (dx * dy + dy * dz + dz * dx);
  }

  // Binned surface-area heuristic: among 16 centroid bins per axis, the
  // split minimising area(left) n_left + area(right) n_right (the expected
  // number of box tests of a ray through the node); when the depth left is
  // only enough for median splits, or no bin boundary separates the boxes,
  // the median of the widest centroid axis.
  // Returns false when no split separates the boxes.
  bool sah_split(uint32_t first, uint32_t count, const double* clo, const double* chi, int depth, int& ax_out,
                 double& cut_out) {
    // keep enough depth for median splits of what is left (leaves of
    // kBvhLeaf): the tree never outgrows the traversal stack
    int need = 1;
    for (uint32_t c = kBvhLeaf; c < count; c *= 2) ++need;
    if (depth + need >= kBvhStack - 2) return false;
    constexpr int kBins = 16;
    double best = INFINITY;
    for (int ax = 0; ax < 3; ++ax) {
      const double ext = chi[ax] - clo[ax];
      if (!(ext > 0.0)) continue;
      uint32_t cnt[kBins] = {};
      double bl[kBins][3], bh[kBins][3];
      for (int b = 0; b < kBins; ++b)
        for (int k = 0; k < 3; ++k) {
          bl[b][k] = INFINITY;
          bh[b][k] = -INFINITY;
        }
      for (uint32_t i = first; i < first + count; ++i) {
        const uint32_t id = ids[i];
        const double c = 0.5 * (lo[3 * id + ax] + hi[3 * id + ax]);
        int b = (int)((c - clo[ax]) / ext * kBins);
        b = b < 0 ? 0 : (b >= kBins ? kBins - 1 : b);
        cnt[b] += 1;
        for (int k = 0; k < 3; ++k) {
          bl[b][k] = std::min(bl[b][k], lo[3 * id + k]);
          bh[b][k] = std::max(bh[b][k], hi[3 * id + k]);
        }
      }
      // right-to-left sweep of areas and counts
      double ra[kBins];
      uint32_t rc[kBins];
      double rl[3] = {INFINITY, INFINITY, INFINITY}, rh[3] = {-INFINITY, -INFINITY, -INFINITY};
      uint32_t rn = 0;
      for (int b = kBins - 1; b > 0; --b) {
        rn += cnt[b];
        for (int k = 0; k < 3; ++k) {
          rl[k] = std::min(rl[k], bl[b][k]);
          rh[k] = std::max(rh[k], bh[b][k]);
        }
        rc[b] = rn;
        ra[b] = rn ? area(rl, rh) : 0.0;
      }
      double ll[3] = {INFINITY, INFINITY, INFINITY}, lh[3] = {-INFINITY, -INFINITY, -INFINITY};
      uint32_t ln = 0;
      for (int b = 0; b + 1 < kBins; ++b) {
        ln += cnt[b];
        for (int k = 0; k < 3; ++k) {
          ll[k] = std::min(ll[k], bl[b][k]);
          lh[k] = std::max(lh[k], bh[b][k]);
        }
        if (ln == 0 || rc[b + 1] == 0) continue;
        const double cost = area(ll, lh) * ln + ra[b + 1] * rc[b + 1];
        if (cost < best) {
          best = cost;
          ax_out = ax;
          cut_out = clo[ax] + ext * (double)(b + 1) / kBins;
        }
      }
    }
    return best < INFINITY;
  }

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
    double cut = 0.0;
    uint32_t half;
    if (sah_split(first, count, clo, chi, depth, ax, cut)) {
      auto mid = std::partition(ids.begin() + first, ids.begin() + first + count,
                                [&](uint32_t b) { return 0.5 * (lo[3 * b + ax] + hi[3 * b + ax]) < cut; });
      half = (uint32_t)(mid - (ids.begin() + first));
    } else {
      half = 0;
    }
    if (half == 0 || half == count) {  // median of the widest centroid axis
      ax = 0;
      for (int k = 1; k < 3; ++k)
        if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
      half = count / 2;
      auto key = [&](uint32_t b) { return lo[3 * b + ax] + hi[3 * b + ax]; };
      std::nth_element(ids.begin() + first, ids.begin() + first + half, ids.begin() + first + count,
                       [&](uint32_t x, uint32_t y) { return key(x) < key(y) || (key(x) == key(y) && x < y); });
    }
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

namespace {

// Per-face neighbour lists: box j is listed for face (i, axis, side) when
// its opposite face lies in the plane of that face and the two faces share
// at least one point.  Candidates come from the boxes whose lower (upper)
// bound on that axis equals the plane, sorted along the next axis.
void face_neighbours(const double* lo, const double* hi, uint32_t n, BvhHost& out) {
  std::map<std::pair<int, double>, std::vector<uint32_t>> at_lo, at_hi;
  for (uint32_t j = 0; j < n; ++j)
    for (int k = 0; k < 3; ++k) {
      at_lo[{k, lo[3 * j + k]}].push_back(j);
      at_hi[{k, hi[3 * j + k]}].push_back(j);
    }
  for (auto* m : {&at_lo, &at_hi})
    for (auto& kv : *m) {
      const int b1 = (kv.first.first + 1) % 3;
      std::sort(kv.second.begin(), kv.second.end(), [&](uint32_t x, uint32_t y) {
        return lo[3 * x + b1] < lo[3 * y + b1] || (lo[3 * x + b1] == lo[3 * y + b1] && x < y);
      });
    }
  out.nbr_off.assign((size_t)n * 6 + 1, 0);
  out.nbr.clear();
  for (uint32_t i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k)
      for (int side = 0; side < 2; ++side) {
        out.nbr_off[(size_t)i * 6 + k * 2 + side] = (uint32_t)out.nbr.size();
        const double plane = side ? hi[3 * i + k] : lo[3 * i + k];
        auto& m = side ? at_lo : at_hi;  // the upper face meets lower faces and vice versa
        auto it = m.find({k, plane});
        if (it == m.end()) continue;
        const int b1 = (k + 1) % 3, b2 = (k + 2) % 3;
        for (uint32_t j : it->second) {
          if (lo[3 * j + b1] > hi[3 * i + b1]) break;  // sorted along b1
          if (j == i || hi[3 * j + b1] < lo[3 * i + b1]) continue;
          if (lo[3 * j + b2] <= hi[3 * i + b2] && lo[3 * i + b2] <= hi[3 * j + b2]) out.nbr.push_back(j);
        }
      }
  out.nbr_off[(size_t)n * 6] = (uint32_t)out.nbr.size();
  out.rec.resize(n);
  for (uint32_t i = 0; i < n; ++i) {
    BoxRec& r = out.rec[i];
    for (int k = 0; k < 3; ++k) {
      r.lo[k] = lo[3 * i + k];
      r.hi[k] = hi[3 * i + k];
    }
    for (int f = 0; f < 6; ++f) {
      const uint32_t a = out.nbr_off[(size_t)i * 6 + f], e = out.nbr_off[(size_t)i * 6 + f + 1];
      r.link[f] = e == a ? kNoLink : (e - a == 1 ? out.nbr[a] : kManyLinks);
    }
    r.pad[0] = r.pad[1] = 0;
  }
}

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
  face_neighbours(lo, hi, n, out);
  // a depth-first walk that pushes both children holds at most depth + 1
  // entries
  if (bd.max_depth + 1 > kBvhStack) {
    err = "box hierarchy deeper than the traversal stack";
    return false;
  }
  return true;
}

}  // namespace ems
