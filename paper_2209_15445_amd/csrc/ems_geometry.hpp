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
  // distance so far skipped (entry distances kept beside the stack).  The
  // walk descends into the nearer child with the bounds it has just read
  // and stacks only the farther one, so a descent costs one dependent read
  // per level; the order of the visits is that of pushing both children
  // and popping the nearer one.
  uint32_t stack[kBvhStack];
  float tstack[kBvhStack];
  int sp = 0;
  BvhNode nd = g.node[0];
  if (!(node_entry(nd, p, iu, u, best) <= best)) return best;
  for (;;) {
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
      const BvhNode cl = g.node[nd.a], cr = g.node[nd.a + 1];
      const double tl = node_entry(cl, p, iu, u, best);
      const double tr = node_entry(cr, p, iu, u, best);
      const bool lfirst = tl <= tr;
      const double tn = lfirst ? tl : tr, tf = lfirst ? tr : tl;
      const uint32_t cf = lfirst ? nd.a + 1 : nd.a;
      if (tf <= best) {
        stack[sp] = cf;
        tstack[sp] = (float)tf;
        ++sp;
      }
      if (tn <= best) {
        nd = lfirst ? cl : cr;
        continue;
      }
    }
    // the next stacked node still entered within the best distance
    // (float copy: compared with a margin)
    bool more = false;
    while (sp > 0) {
      --sp;
      if ((double)tstack[sp] > best * (1.0 + 1e-6)) continue;
      nd = g.node[stack[sp]];
      more = true;
      break;
    }
    if (!more) break;
  }
  return best;
}

// ---------------------------------------------------------------- helix
// A charged track in the field Bz turns about z: with psi = |kappa| s the
// angle turned after path s, its transverse position runs on the circle
// x = cx + rad sin(psi - phase), y = cy + sgn rad cos(psi - phase)
// (sgn the sign of kappa, rad = u_perp / |kappa|) and z = z0 + uz s.  A
// plane x = X or y = Y is met at angles from asin / acos, a z plane
// linearly; the boundary of a box is reached at the first such crossing
// (leaving a box: outward through any face; entering one: inward at a point
// within the face).
struct HelixPath {
  double p0[3], uz, ak, rad, cx, cy, phase;
  int sgn;
};

EMS_HD HelixPath helix_path(const double p[3], const double u[3], double kappa) {
  HelixPath h;
  for (int k = 0; k < 3; ++k) h.p0[k] = p[k];
  h.uz = u[2];
  h.ak = fabs(kappa);
  h.sgn = kappa > 0.0 ? 1 : -1;
  h.rad = sqrt(u[0] * u[0] + u[1] * u[1]) / h.ak;
  h.cx = p[0] + u[1] / kappa;
  h.cy = p[1] - u[0] / kappa;
  h.phase = h.sgn * atan2(u[1], u[0]);
  return h;
}

// angle from the start (psi = 0) forward to the circle angle th, in
// [0, 2 pi); within 1e-9 of a whole turn it is the start itself
EMS_HD double helix_advance(const HelixPath& h, double th) {
  constexpr double kTurn = 6.28318530717958647692;
  double d = fmod(th + h.phase, kTurn);
  if (d < 0.0) d += kTurn;
  return d > kTurn - 1e-9 ? 0.0 : d;
}

// first psi >= 0 at which the plane coordinate[axis] = v (axis 0 or 1) is
// crossed moving up (up = true) or down that axis; negative if never
EMS_HD double helix_plane(const HelixPath& h, int axis, double v, bool up) {
  if (!(h.rad > 0.0)) return -1.0;
  constexpr double kPiD = 3.14159265358979323846;
  if (axis == 0) {
    const double w = (v - h.cx) / h.rad;
    if (!(w >= -1.0 && w <= 1.0)) return -1.0;
    const double a = asin(w);  // x grows where cos(theta) > 0
    return helix_advance(h, up ? a : kPiD - a);
  }
  const double w = h.sgn * (v - h.cy) / h.rad;
  if (!(w >= -1.0 && w <= 1.0)) return -1.0;
  const double a = acos(w);    // y grows where sgn sin(theta) < 0
  return helix_advance(h, up ? -h.sgn * a : h.sgn * a);
}

// position after path s (the propagation's formulas)
EMS_HD void helix_point(const HelixPath& h, const double u[3], double kappa, double s, double q[3]) {
  const double ph = kappa * s;
  double sh, ch;
  sincos(0.5 * ph, &sh, &ch);
  const double sp = 2.0 * sh * ch, omc = 2.0 * sh * sh;
  q[0] = h.p0[0] + (u[0] * sp + u[1] * omc) / kappa;
  q[1] = h.p0[1] + (u[1] * sp - u[0] * omc) / kappa;
  q[2] = h.p0[2] + u[2] * s;
}

// leaving the box [lo, hi] from inside: path length to the first outward
// crossing (the first axis on ties), infinity if it never leaves
EMS_HD double helix_leave(const HelixPath& h, const double* lo, const double* hi, Face& fc) {
  double best = __builtin_huge_val();
  for (int k = 0; k < 3; ++k) {
    double d = __builtin_huge_val(), f = 0.0;
    int side = 0;
    if (k < 2) {
      const double a = helix_plane(h, k, hi[k], true), b = helix_plane(h, k, lo[k], false);
      if (a >= 0.0 && (b < 0.0 || a <= b)) {
        d = a / h.ak;
        f = hi[k];
        side = 1;
      } else if (b >= 0.0) {
        d = b / h.ak;
        f = lo[k];
      }
    } else if (h.uz != 0.0) {
      side = h.uz > 0.0 ? 1 : 0;
      f = side ? hi[2] : lo[2];
      d = (f - h.p0[2]) / h.uz;
      d = d < 0.0 ? 0.0 : d;
    }
    if (d < best) {
      best = d;
      fc.ax = k;
      fc.f = f;
      fc.side = side;
    }
  }
  return best;
}

// entering the box [lo, hi] from outside within path smax: the smallest
// path length at which the helix crosses a face plane inward at a point
// within the face (x and y planes once per turn each way), or infinity
EMS_HD double helix_enter(const HelixPath& h, const double u[3], double kappa, const double* lo, const double* hi,
                          double smax, Face& fc) {
  double best = __builtin_huge_val();
  for (int k = 0; k < 3; ++k) {
    for (int side = 0; side < 2; ++side) {
      const double v = side ? hi[k] : lo[k];
      double s0, turn = __builtin_huge_val();
      if (k < 2) {
        const double a = helix_plane(h, k, v, side == 0);
        if (a < 0.0) continue;
        s0 = a / h.ak;
        turn = 6.28318530717958647692 / h.ak;
      } else {
        if (h.uz == 0.0 || (h.uz > 0.0) != (side == 0)) continue;
        s0 = (v - h.p0[2]) / h.uz;
        if (s0 < 0.0) continue;
      }
      for (double sc = s0; sc <= smax && sc < best; sc += turn) {
        double q[3];
        helix_point(h, u, kappa, sc, q);
        q[k] = v;
        const int j1 = k == 0 ? 1 : 0, j2 = k == 2 ? 1 : 2;
        if (q[j1] >= lo[j1] && q[j1] <= hi[j1] && q[j2] >= lo[j2] && q[j2] <= hi[j2]) {
          best = sc;
          fc.ax = k;
          fc.f = v;
          fc.side = side;
          break;
        }
        if (!(turn < __builtin_huge_val())) break;
      }
    }
  }
  return best;
}

// path length along the helix of curvature kappa to the next boundary from
// volume v, searched up to smax (infinity: none within smax), with the face
// reached: a box's own faces; from the world the nearer of its exit and the
// first box entered (boxes win ties), the boxes found through the hierarchy
// by the bounding box of the arc
EMS_HD double helix_distance(const BoxNav& g, int v, const double p[3], const double u[3], double kappa,
                             double smax, Face& fc) {
  const HelixPath h = helix_path(p, u, kappa);
  double best;
  if ((uint32_t)v < g.n_boxes) {
    const BoxRec& b = g.rec[v];
    best = helix_leave(h, b.lo, b.hi, fc);
    fc.box = v;
  } else {
    best = helix_leave(h, g.wlo, g.whi, fc);
    fc.box = -1;
    double lim = smax < best ? smax : best;
    const double turn = 6.28318530717958647692 / h.ak;
    if (h.uz == 0.0 && turn < lim) lim = turn;  // a circle in a plane: one turn
    if (lim < __builtin_huge_val()) {
      // the arc over [0, lim] lies within the circle's box, within lim of
      // the start, and between the z of its ends
      double alo[3], ahi[3];
      alo[0] = fmax(h.cx - h.rad, p[0] - lim);
      ahi[0] = fmin(h.cx + h.rad, p[0] + lim);
      alo[1] = fmax(h.cy - h.rad, p[1] - lim);
      ahi[1] = fmin(h.cy + h.rad, p[1] + lim);
      alo[2] = fmin(p[2], p[2] + u[2] * lim);
      ahi[2] = fmax(p[2], p[2] + u[2] * lim);
      uint32_t stack[kBvhStack];
      int sp = 0;
      stack[sp++] = 0;
      while (sp > 0) {
        const BvhNode nd = g.node[stack[--sp]];
        if (ahi[0] < nd.lo[0] || alo[0] > nd.hi[0] || ahi[1] < nd.lo[1] || alo[1] > nd.hi[1] || ahi[2] < nd.lo[2] ||
            alo[2] > nd.hi[2])
          continue;
        if (nd.count) {
          for (uint32_t i = 0; i < nd.count; ++i) {
            const uint32_t id = g.leaf[nd.a + i];
            const double* b = g.box + (size_t)id * 6;
            Face f2{0, 0.0, 0, (int)id};
            const double d = helix_enter(h, u, kappa, b, b + 3, lim < best ? lim : best, f2);
            if (d <= best) {
              best = d;
              fc = f2;
              fc.box = (int)id;
            }
          }
        } else if (sp + 2 <= kBvhStack) {
          stack[sp++] = nd.a + 1;
          stack[sp++] = nd.a;
        }
      }
    }
  }
  return best <= smax ? best : __builtin_huge_val();
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
