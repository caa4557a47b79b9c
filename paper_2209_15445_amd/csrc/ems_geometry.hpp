// ems_geometry.hpp -- box geometry: non-overlapping axis-aligned boxes in a
// world box, navigated through a bounding-volume hierarchy.
//
// The paper names geometry navigation as the dominant cost of its GPU
// transport and points to bounding-volume hierarchies for it (sections 2.1
// and 5).  Here a geometry may be, instead of the slab stack, a set of boxes
// (volume v < n_boxes) inside a world box (volume n_boxes) that fills the
// rest; a track reaching the world's surface leaves the geometry.  A point on
// a face belongs to the box it moves into: per axis lo < p < hi, or p = lo
// moving with u >= 0, or p = hi moving with u < 0.  The host builds a binary
// BVH over the boxes (median split of the centroids along the widest axis,
// leaves of up to kBvhLeaf boxes); the device walks it with a small stack.
// Node bounds are single precision, widened outward so that every node test
// is conservative; the exact tests on a box use its double bounds and the
// same divisions as a brute-force walk over all boxes.
#pragma once
#include "ems_core.hpp"

namespace ems {

constexpr uint32_t kBvhLeaf = 4;    // boxes per leaf (at most)
constexpr int kBvhStack = 32;       // traversal stack = maximum tree depth

struct BvhNode {
  float lo[3], hi[3];
  uint32_t a;      // internal: left child (the right one is a + 1); leaf: first leaf entry
  uint32_t count;  // leaf: number of entries (> 0); internal: 0
};

// device (or host) view of a box geometry
struct BoxNav {
  const BvhNode* node;     // [n_nodes], root at 0
  const uint32_t* leaf;    // [n_boxes] box ids in leaf order
  const double* box;       // [n_boxes][6]: lo x y z, hi x y z, by box id
  double wlo[3], whi[3];   // world box
  uint32_t n_boxes;
};

struct Face {
  int ax;
  double f;
};

EMS_HD bool in_axis(double p, double lo, double hi, double u) {
  return (p > lo && p < hi) || (p == lo && u >= 0.0) || (p == hi && u < 0.0);
}
EMS_HD bool in_box(const double* lo, const double* hi, const double p[3], const double u[3]) {
  return in_axis(p[0], lo[0], hi[0], u[0]) && in_axis(p[1], lo[1], hi[1], u[1]) &&
         in_axis(p[2], lo[2], hi[2], u[2]);
}

// from inside a box: nearest exit face (the first axis on ties)
EMS_HD double ray_exit(const double* lo, const double* hi, const double p[3], const double u[3], Face& fc) {
  double s = __builtin_huge_val();
  for (int k = 0; k < 3; ++k) {
    double d = __builtin_huge_val(), f = 0.0;
    if (u[k] > 0.0) {
      d = (hi[k] - p[k]) / u[k];
      f = hi[k];
    } else if (u[k] < 0.0) {
      d = (lo[k] - p[k]) / u[k];
      f = lo[k];
    }
    if (d < s) {
      s = d;
      fc.ax = k;
      fc.f = f;
    }
  }
  return s;
}

// from outside a box: entry distance (slab method), infinity if the ray
// misses it, grazes an edge or moves away
EMS_HD double ray_entry(const double* lo, const double* hi, const double p[3], const double u[3], Face& fc) {
  double tn = -__builtin_huge_val(), tf = __builtin_huge_val();
  int a = -1;
  double f = 0.0;
  for (int k = 0; k < 3; ++k) {
    if (u[k] == 0.0) {
      if (!(p[k] >= lo[k] && p[k] < hi[k])) return __builtin_huge_val();
      continue;
    }
    const double t1 = (lo[k] - p[k]) / u[k], t2 = (hi[k] - p[k]) / u[k];
    const double nr = t1 < t2 ? t1 : t2, fr = t1 < t2 ? t2 : t1;
    if (nr > tn) {
      tn = nr;
      a = k;
      f = u[k] > 0.0 ? lo[k] : hi[k];
    }
    if (fr < tf) tf = fr;
  }
  if (a < 0 || !(tn < tf) || !(tf > 0.0)) return __builtin_huge_val();
  fc.ax = a;
  fc.f = f;
  return tn > 0.0 ? tn : 0.0;
}

// conservative ray test of a node against the best distance so far
EMS_HD bool node_hit(const BvhNode& nd, const double p[3], const double iu[3], const double u[3], double best) {
  double tn = 0.0, tf = best;
  for (int k = 0; k < 3; ++k) {
    const double lo = nd.lo[k], hi = nd.hi[k];
    if (u[k] == 0.0) {
      if (p[k] < lo || p[k] > hi) return false;
      continue;
    }
    const double t1 = (lo - p[k]) * iu[k], t2 = (hi - p[k]) * iu[k];
    const double nr = t1 < t2 ? t1 : t2, fr = t1 < t2 ? t2 : t1;
    tn = nr > tn ? nr : tn;
    tf = fr < tf ? fr : tf;
  }
  return tn <= tf;
}

// volume of point p moving along u: a box id, n_boxes for the world, -1
// outside it
EMS_HD int bvh_locate(const BoxNav& g, const double p[3], const double u[3]) {
  uint32_t stack[kBvhStack];
  int sp = 0;
  stack[sp++] = 0;
  while (sp > 0) {
    const BvhNode nd = g.node[stack[--sp]];
    if (p[0] < nd.lo[0] || p[0] > nd.hi[0] || p[1] < nd.lo[1] || p[1] > nd.hi[1] || p[2] < nd.lo[2] ||
        p[2] > nd.hi[2])
      continue;
    if (nd.count) {
      for (uint32_t i = 0; i < nd.count; ++i) {
        const uint32_t id = g.leaf[nd.a + i];
        const double* b = g.box + (size_t)id * 6;
        if (in_box(b, b + 3, p, u)) return (int)id;
      }
    } else if (sp + 2 <= kBvhStack) {
      stack[sp++] = nd.a + 1;
      stack[sp++] = nd.a;
    }
  }
  return in_box(g.wlo, g.whi, p, u) ? (int)g.n_boxes : -1;
}

// distance to the next boundary from volume v along u: a box's own faces;
// from the world the nearer of its exit and the first box entered (boxes
// win ties)
EMS_HD double box_distance(const BoxNav& g, int v, const double p[3], const double u[3], Face& fc) {
  if ((uint32_t)v < g.n_boxes) {
    const double* b = g.box + (size_t)v * 6;
    return ray_exit(b, b + 3, p, u, fc);
  }
  double best = ray_exit(g.wlo, g.whi, p, u, fc);
  const double iu[3] = {1.0 / u[0], 1.0 / u[1], 1.0 / u[2]};
  uint32_t stack[kBvhStack];
  int sp = 0;
  stack[sp++] = 0;
  while (sp > 0) {
    const BvhNode nd = g.node[stack[--sp]];
    if (!node_hit(nd, p, iu, u, best)) continue;
    if (nd.count) {
      for (uint32_t i = 0; i < nd.count; ++i) {
        const uint32_t id = g.leaf[nd.a + i];
        const double* b = g.box + (size_t)id * 6;
        Face f2;
        const double d = ray_entry(b, b + 3, p, u, f2);
        if (d <= best) {
          best = d;
          fc = f2;
        }
      }
    } else if (sp + 2 <= kBvhStack) {
      stack[sp++] = nd.a + 1;
      stack[sp++] = nd.a;
    }
  }
  return best;
}

// volume entered after reaching face fc at p (the coordinate is set to the
// face): -1 when it is on the world's surface or outside it
EMS_HD int box_cross(const BoxNav& g, double p[3], const double u[3], const Face& fc) {
  p[fc.ax] = fc.f;
  if (fc.f == g.wlo[fc.ax] || fc.f == g.whi[fc.ax]) return -1;
  return bvh_locate(g, p, u);
}

}  // namespace ems

#include <string>
#include <vector>
namespace ems {
// host-built hierarchy over n boxes given as lo[n][3], hi[n][3]; returns
// false (with a message) for a depth above kBvhStack
struct BvhHost {
  std::vector<BvhNode> node;
  std::vector<uint32_t> leaf;
  std::vector<double> box;  // [n][6]
};
bool build_bvh(const double* lo, const double* hi, uint32_t n, BvhHost& out, std::string& err);
}  // namespace ems
