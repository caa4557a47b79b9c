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
// BVH over the boxes (binned surface-area heuristic, median splits where the
// depth budget or the centroids require them, leaves of up to kBvhLeaf
// boxes); the device walks it front to back with a small stack.  After a crossing the volume entered is found among the
// boxes that touch the face crossed (per-face neighbour lists, complete, so
// the result is that of a search over all boxes), or the world.
// Node bounds are single precision, widened outward so that every node test
// is conservative; the exact tests on a box use its double bounds and the
// same divisions as a brute-force walk over all boxes.
#pragma once
#include "ems_core.hpp"

namespace ems {

constexpr uint32_t kBvhLeaf = 4;    // boxes per leaf (at most)
constexpr int kBvhStack = 32;       // traversal stack = maximum tree depth
constexpr uint32_t kFaceScan = 16;  // longer neighbour lists: locate through the hierarchy
constexpr uint32_t kNoLink = 0xFFFFFFFFu, kManyLinks = 0xFFFFFFFEu;

// a box as the navigator reads it: bounds, and per face (axis, side) the
// one box touching it (kNoLink: none, kManyLinks: several, see nbr lists)
struct BoxRec {
  double lo[3], hi[3];
  uint32_t link[6];
  uint32_t pad[2];
};

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
  const BoxRec* rec;       // [n_boxes] by box id
  const uint32_t* nbr_off; // [6 n_boxes + 1]: face (box, axis, side) -> range in nbr
  const uint32_t* nbr;     // boxes touching each face (sharing its plane and part of it)
  double wlo[3], whi[3];   // world box
  uint32_t n_boxes;
};

// a face reached: axis, coordinate, side (1: the upper face of its box) and
// the box it belongs to (-1: the world's)
struct Face {
  int ax;
  double f;
  int side;
  int box;
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
      fc.side = u[k] > 0.0 ? 1 : 0;
    }
  }
  return s;
}

// the same with the direction's reciprocals (a track that keeps its
// direction over several steps computes them once)
EMS_HD double ray_exit_inv(const double* lo, const double* hi, const double p[3], const double u[3],
                           const double iu[3], Face& fc) {
  double s = __builtin_huge_val();
  for (int k = 0; k < 3; ++k) {
    double d = __builtin_huge_val(), f = 0.0;
    if (u[k] > 0.0) {
      d = (hi[k] - p[k]) * iu[k];
      f = hi[k];
    } else if (u[k] < 0.0) {
      d = (lo[k] - p[k]) * iu[k];
      f = lo[k];
    }
    if (d < s) {
      s = d;
      fc.ax = k;
      fc.f = f;
      fc.side = u[k] > 0.0 ? 1 : 0;
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
  fc.side = u[a] > 0.0 ? 0 : 1;
  return tn > 0.0 ? tn : 0.0;
}

// conservative ray test of a node against the best distance so far: its
// entry distance (clamped at 0), or infinity when it cannot hold a nearer box
EMS_HD double node_entry(const BvhNode& nd, const double p[3], const double iu[3], const double u[3], double best) {
  double tn = 0.0, tf = best;
  for (int k = 0; k < 3; ++k) {
    const double lo = nd.lo[k], hi = nd.hi[k];
    if (u[k] == 0.0) {
      if (p[k] < lo || p[k] > hi) return __builtin_huge_val();
      continue;
    }
    const double t1 = (lo - p[k]) * iu[k], t2 = (hi - p[k]) * iu[k];
    const double nr = t1 < t2 ? t1 : t2, fr = t1 < t2 ? t2 : t1;
    tn = nr > tn ? nr : tn;
    tf = fr < tf ? fr : tf;
  }
  return tn <= tf ? tn : __builtin_huge_val();
}

// cheap screen before the exact entry test: with reciprocals instead of
// divisions and a margin far above their rounding, false only for boxes
// the ray cannot enter within best
EMS_HD bool maybe_entered(const double* lo, const double* hi, const double p[3], const double u[3],
                          const double iu[3], double best) {
  double tn = -__builtin_huge_val(), tf = __builtin_huge_val();
  for (int k = 0; k < 3; ++k) {
    if (u[k] == 0.0) {
      if (!(p[k] >= lo[k] && p[k] < hi[k])) return false;
      continue;
    }
    const double t1 = (lo[k] - p[k]) * iu[k], t2 = (hi[k] - p[k]) * iu[k];
    tn = fmax(tn, fmin(t1, t2));
    tf = fmin(tf, fmax(t1, t2));
  }
  const double m = 1e-9 * (fabs(tn) + fabs(tf) + fabs(best)) + 1e-12;
  return tn <= tf + m && tf > -m && tn <= best + m;
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
EMS_HD double box_distance(const BoxNav& g, int v, const double p[3], const double u[3], Face& fc,
                           const double* iu_cached = nullptr) {
  if ((uint32_t)v < g.n_boxes) {
    const BoxRec& b = g.rec[v];
    fc.box = v;
    return iu_cached ? ray_exit_inv(b.lo, b.hi, p, u, iu_cached, fc) : ray_exit(b.lo, b.hi, p, u, fc);
  }
  double best = ray_exit(g.wlo, g.whi, p, u, fc);
  fc.box = -1;
  const double iu[3] = {1.0 / u[0], 1.0 / u[1], 1.0 / u[2]};
  // front to back: the nearer child first, nodes entered beyond the best
  // distance so far skipped (entry distances kept beside the stack)
  uint32_t stack[kBvhStack];
  float tstack[kBvhStack];
  int sp = 0;
  const double t0 = node_entry(g.node[0], p, iu, u, best);
  if (t0 <= best) {
    stack[0] = 0;
    tstack[0] = (float)t0;
    sp = 1;
  }
  while (sp > 0) {
    --sp;
    if ((double)tstack[sp] > best * (1.0 + 1e-6)) continue;  // float copy: compare with margin
    const BvhNode nd = g.node[stack[sp]];
    if (nd.count) {
      for (uint32_t i = 0; i < nd.count; ++i) {
        const uint32_t id = g.leaf[nd.a + i];
        const double* b = g.box + (size_t)id * 6;
        if (!maybe_entered(b, b + 3, p, u, iu, best)) continue;
        Face f2;
        const double d = ray_entry(b, b + 3, p, u, f2);
        if (d <= best) {
          best = d;
          fc = f2;
          fc.box = (int)id;
        }
      }
    } else if (sp + 2 <= kBvhStack) {
      const double tl = node_entry(g.node[nd.a], p, iu, u, best);
      const double tr = node_entry(g.node[nd.a + 1], p, iu, u, best);
      const bool lfirst = tl <= tr;
      const double tn = lfirst ? tl : tr, tf = lfirst ? tr : tl;
      const uint32_t cn = lfirst ? nd.a : nd.a + 1, cf = lfirst ? nd.a + 1 : nd.a;
      if (tf <= best) {
        stack[sp] = cf;
        tstack[sp] = (float)tf;
        ++sp;
      }
      if (tn <= best) {
        stack[sp] = cn;
        tstack[sp] = (float)tn;
        ++sp;
      }
    }
  }
  return best;
}

// volume entered after reaching face fc at p (the coordinate is set to the
// face): -1 when it is on the world's surface or outside it.  A point on a
// box's face lies in that box, in a box touching the face, or in the world
// (boxes do not overlap), so those candidates decide it.
EMS_HD int box_cross(const BoxNav& g, double p[3], const double u[3], const Face& fc) {
  p[fc.ax] = fc.f;
  if (fc.f == g.wlo[fc.ax] || fc.f == g.whi[fc.ax]) return -1;
  if (fc.box < 0) return bvh_locate(g, p, u);
  const BoxRec& b = g.rec[fc.box];
  if (in_box(b.lo, b.hi, p, u)) return fc.box;
  const uint32_t link = b.link[fc.ax * 2 + fc.side];
  if (link < kManyLinks) {
    const BoxRec& c = g.rec[link];
    if (in_box(c.lo, c.hi, p, u)) return (int)link;
  }
  if (link != kManyLinks) return in_box(g.wlo, g.whi, p, u) ? (int)g.n_boxes : -1;
  const uint32_t fi = (uint32_t)fc.box * 6u + (uint32_t)fc.ax * 2u + (uint32_t)fc.side;
  const uint32_t lo = g.nbr_off[fi], hi = g.nbr_off[fi + 1];
  if (hi - lo > kFaceScan) return bvh_locate(g, p, u);
  for (uint32_t k = lo; k < hi; ++k) {
    const uint32_t id = g.nbr[k];
    const double* c = g.box + (size_t)id * 6;
    if (in_box(c, c + 3, p, u)) return (int)id;
  }
  return in_box(g.wlo, g.whi, p, u) ? (int)g.n_boxes : -1;
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
  std::vector<uint32_t> nbr_off, nbr;  // per-face neighbour lists
  std::vector<BoxRec> rec;
};
bool build_bvh(const double* lo, const double* hi, uint32_t n, BvhHost& out, std::string& err);
}  // namespace ems
