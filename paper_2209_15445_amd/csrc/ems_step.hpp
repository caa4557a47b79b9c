// ems_step.hpp -- one transport step of one track.
//
// This is the per-thread body of the paper's stepping workflow (section 3):
// a thread takes one track of a species' current array, moves it one step
// (physics step limit, geometry limit, field propagation, continuous loss,
// discrete interaction) and hands back the surviving track plus at most two
// secondaries, which the caller appends to the next arrays.  The function is
// pure: every random number comes from the (seed, event key, id, step) Philox
// stream, so results do not depend on which thread or iteration runs it.
//
// The step is written for a real type R.  R = double is the FP64 form.
// R = float is the mixed form: tables, interpolation, step lengths, loss
// and sampling in FP32, while positions, boundary and safety distances, the
// helix and every energy (track, deposit, secondaries) stay FP64, so energy
// bookkeeping is exact in both forms.
#pragma once
#include "ems_geometry.hpp"
#include "ems_models.hpp"
#include "ems_tables.hpp"

namespace ems {

constexpr double kInf = __builtin_huge_val();

// Optional parts of the step, compiled into a kernel only when its
// configuration uses them (a kernel without one is launched only for
// configurations that leave it off; the host path has all of them): the
// helix in a field, multiple scattering, loss fluctuations, a compound
// target element, and the per-step records (step log, full ledger, exits,
// per-event live counters).
enum : int { kFField = 1, kFMsc = 2, kFFluct = 4, kFCompound = 8, kFRecord = 16, kFShort = 32, kFAll = 63 };

// Tables are held in two blocks so each kernel stages only its own: the
// photon block [mat][3][nodes] (tables 0..2) and the lepton block
// [mat][12][nodes] (tables 3..14).
constexpr int kGammaTables = 3, kLeptonTables = kNumDevTables - kGammaTables;

template <class R>
struct StepEnv {
  const R* tg;               // photon table block
  const R* tl;               // lepton table block
  const double* zplane;      // n_slabs + 1
  const uint32_t* slab_mat;  // n_slabs
  const MatRT* mat;
  BoxNav nav;                // box geometry (geometry kind 1)
  const double* elc;         // element screening constants [mat][4][2]
  const R* elt;              // partial pair / brems totals [mat][4][2][nodes]
  uint32_t nodes, n_slabs;
  R lnemin, dlog, inv_dlog;
  double half_xy, bz;
  double ecut, tcut, kcut;
  double alpha, rho, lin;
  uint32_t mask, seed, max_steps;

  EMS_HD const R* T(uint32_t m, int t) const {
    return t < kGammaTables ? tg + ((size_t)m * kGammaTables + t) * nodes
                            : tl + ((size_t)m * kLeptonTables + (t - kGammaTables)) * nodes;
  }
};

// the scalars of an environment in another arithmetic type (table pointers
// are left null)
template <class R, class S>
EMS_HD StepEnv<R> retype(const StepEnv<S>& a) {
  StepEnv<R> e;
  e.tg = nullptr;
  e.tl = nullptr;
  e.zplane = a.zplane;
  e.slab_mat = a.slab_mat;
  e.mat = a.mat;
  e.nav = a.nav;
  e.elc = a.elc;
  e.elt = nullptr;
  e.nodes = a.nodes;
  e.n_slabs = a.n_slabs;
  e.lnemin = (R)a.lnemin;
  e.dlog = (R)a.dlog;
  e.inv_dlog = (R)a.inv_dlog;
  e.half_xy = a.half_xy;
  e.bz = a.bz;
  e.ecut = a.ecut;
  e.tcut = a.tcut;
  e.kcut = a.kcut;
  e.alpha = a.alpha;
  e.rho = a.rho;
  e.lin = a.lin;
  e.mask = a.mask;
  e.seed = a.seed;
  e.max_steps = a.max_steps;
  return e;
}

template <class R>
struct Trk {
  double x, y, z;
  R ux, uy, uz;
  double E;
  uint64_t id;
  uint32_t ev, key, n;
  int32_t slab;  // < 0: track has ended
};

template <class R>
struct Sec {
  int sp;
  double E;
  R ux, uy, uz;
  uint64_t id;
};

template <class R>
struct StepOut {
  int nsec;
  Sec<R> sec[2];
  int slab;        // slab the step was taken in (deposits, secondaries)
  double dep;      // energy deposited in that slab
  double escaped;  // kinetic energy of the track leaving the stack
  double killed;   // kinetic energy removed by the watchdog
  double clen;     // charged path length
  int pair, annih, null;
  uint32_t limiter, process;
  bool pending;    // a discrete interaction `process` is selected but not yet sampled
  double step_len;
};

template <class R>
struct Bin {
  int j;
  R u;
};

template <class R>
EMS_HD Bin<R> bin_of(const StepEnv<R>& e, R lnE) {
  const R x = (lnE - e.lnemin) * e.inv_dlog;
  R f = xfloor(x);
  const R top = (R)(e.nodes - 2);
  f = f < R(0) ? R(0) : (f > top ? top : f);
  int j = (int)f;  // clamped again as an integer: a NaN never indexes outside
  j = j < 0 ? 0 : (j > (int)e.nodes - 2 ? (int)e.nodes - 2 : j);
  R u = x - (R)j;
  u = u < R(0) ? R(0) : (u > R(1) ? R(1) : u);
  return Bin<R>{j, u};
}
template <class R>
EMS_HD R lerp(const R* f, Bin<R> b) {
  return f[b.j] + b.u * (f[b.j + 1] - f[b.j]);
}

// largest node j <= jhi with R_j <= r (0 if none; clamped to the last bin),
// then the exact inverse of the range interpolant.  The loss over one step
// spans few bins, so the scan starts at the track's own bin and reads kWalk
// nodes below it at once (loads that do not wait on each other).  A step
// towards the end of the range goes down a dozen bins or more, and a wave
// waits for its longest scan: past the first kWalk nodes the scan reads
// every kWalk-th node to find the group of kWalk that holds the answer,
// then that group, so any scan of up to kWalk * (kWalk + 1) nodes takes
// three rounds of loads.
constexpr int kWalk = 8;
// first k of top, top - 1, ..., top - kWalk + 1 that is node 0 or holds
// R_j <= r (kWalk if none)
template <class R>
EMS_HD int walk_round(const R* Rt, R r, int top) {
  R v[kWalk];
#pragma unroll
  for (int k = 0; k < kWalk; ++k) v[k] = Rt[top > k ? top - k : 0];
  int d = kWalk;
#pragma unroll
  for (int k = kWalk - 1; k >= 0; --k)
    if (top <= k || !(v[k] > r)) d = k;
  return d;
}
// (the logarithm of the energy; inverse_range below is its exponential)
template <class R>
EMS_HD R inverse_range_ln(const StepEnv<R>& e, const R* Rt, R r, int jhi) {
  int lo = jhi > (int)e.nodes - 1 ? (int)e.nodes - 1 : jhi;
  if (lo > 0) {
    int d = walk_round(Rt, r, lo);
    if (d < kWalk) {
      lo -= d;
    } else {
      // nodes lo .. lo - kWalk + 1 all exceed r: look at every kWalk-th
      // node below (R grows with the node index, so the first one at or
      // below r bounds the group above it)
      lo -= kWalk;
      R v[kWalk];
#pragma unroll
      for (int c = 0; c < kWalk; ++c) v[c] = Rt[lo > kWalk * c ? lo - kWalk * c : 0];
      int g = kWalk;
#pragma unroll
      for (int c = kWalk - 1; c >= 0; --c)
        if (lo <= kWalk * c || !(v[c] > r)) g = c;
      if (g == 0) {
        // node lo is node 0 or at or below r
      } else if (g < kWalk) {
        // node lo - kWalk g is node 0 or at or below r, node lo - kWalk (g - 1)
        // and every node above it exceed r: the answer lies in the kWalk
        // nodes from lo - kWalk (g - 1) - 1 down
        const int top = lo - kWalk * (g - 1) - 1;
        lo = top - walk_round(Rt, r, top);
      } else {
        // node lo - kWalk (kWalk - 1) > 0 exceeds r: go on below it
        lo -= kWalk * (kWalk - 1) + 1;
        while (lo > 0) {
          d = walk_round(Rt, r, lo);
          if (d < kWalk) {
            lo -= d;
            break;
          }
          lo -= kWalk;
        }
      }
    }
  }
  if (lo > (int)e.nodes - 2) lo = (int)e.nodes - 2;
  return e.lnemin + (R)lo * e.dlog + e.dlog * (r - Rt[lo]) / (Rt[lo + 1] - Rt[lo]);
}
template <class R>
EMS_HD R inverse_range(const StepEnv<R>& e, const R* Rt, R r, int jhi) {
  return xexp(inverse_range_ln(e, Rt, r, jhi));
}

// energy lost over path s by a charged track of kinetic energy T (stopping
// power S and range Rv at T); FP64 result.  When the remaining energy comes
// from the range table, *ln_left receives its logarithm (as interpolated,
// before the subtraction from T) and *have_ln is set.
template <class R>
EMS_HD double cont_loss(const StepEnv<R>& e, const R* Rt, int jT, double T, R S, R Rv, double s,
                        R* ln_left = nullptr, bool* have_ln = nullptr) {
  double L;
  bool from_table = false;
  R x = R(0);
  if (s >= (double)Rv) {
    L = T;
  } else if (s < (double)(R(e.lin) * Rv)) {
    L = (double)((R)s * S);
  } else {
    x = inverse_range_ln(e, Rt, Rv - (R)s, jT + 1);
    L = T - (double)xexp(x);
    from_table = true;
  }
  if (L < 0.0) {
    L = 0.0;
    from_table = false;
  }
  if (T - L < e.ecut) {
    L = T;
    from_table = false;
  }
  if (ln_left) {
    *ln_left = x;
    *have_ln = from_table;
  }
  return L;
}

// Distance to the next discrete interaction, -ln(U0)/sigma, or kInf when it
// certainly lies beyond `reach` so that its value is not needed: from
// ln(1 - y) <= -y, u <= (1 - y)(1 - m) with y = sigma * reach gives
// -ln(u)/sigma >= reach (1 + m/y) >= reach (1 + m), and the margin m (1e-9
// in FP64, 1e-5 in FP32) is far above the rounding of the logarithm and the
// division, so every comparison of the result with `reach` comes out as it
// would with the exact value.
template <class R>
EMS_HD double phys_distance(Draws& r, R sig, double reach) {
  if (!(sig > R(0))) return kInf;
  const R u = r.u_at<R>(0);
  const double y = (double)sig * reach;
  const double m = sizeof(R) == 8 ? 1e-9 : 1e-5;
  if ((double)u <= (1.0 - y) * (1.0 - m)) return kInf;
  return (double)(-xlog(u) / sig);
}

template <class R>
EMS_HD void land_on_plane(const StepEnv<R>& e, Trk<R>& t, StepOut<R>& o, bool up) {
  // on the plane reached (the upper one if up), into the next slab; the
  // first and last planes are the stack's surface.  A track turned back on
  // an inner plane by multiple scattering stays in its slab.
  t.z = up ? e.zplane[t.slab + 1] : e.zplane[t.slab];
  const int next = up ? t.slab + 1 : t.slab - 1;
  const bool outer = next < 0 || next >= (int)e.n_slabs;
  if (outer || (up ? t.uz > R(0) : t.uz < R(0))) t.slab = next;
  if (t.slab < 0 || t.slab >= (int)e.n_slabs) {
    o.escaped += t.E;
    t.E = 0.0;
    t.slab = -1;
  }
}

// Geometry kinds: 0 = the slab stack, 1 = boxes (see ems_geometry.hpp).
// A boundary distance computed before the step (box geometries: the
// kernels compute the world volume's distances for several lanes at once),
// exactly the value the step would compute itself.
struct GeoPre {
  double s;
  Face fc;
};
// Box geometry: distance to the next boundary and the face reached.
template <class R>
EMS_HD double box_dist(const StepEnv<R>& e, const Trk<R>& t, Face& fc, const double* iu = nullptr) {
  const double p[3] = {t.x, t.y, t.z}, u[3] = {(double)t.ux, (double)t.uy, (double)t.uz};
  return box_distance(e.nav, t.slab, p, u, fc, iu);
}
// on the face reached, into the volume the track moves into, or out
template <class R>
EMS_HD void box_land(const StepEnv<R>& e, Trk<R>& t, StepOut<R>& o, const Face& fc) {
  double p[3] = {t.x, t.y, t.z};
  const double u[3] = {(double)t.ux, (double)t.uy, (double)t.uz};
  const int v = box_cross(e.nav, p, u, fc);
  t.x = p[0];
  t.y = p[1];
  t.z = p[2];
  if (v < 0) {
    o.escaped += t.E;
    t.E = 0.0;
    t.slab = -1;
  } else {
    t.slab = v;
  }
}

template <class R>
EMS_HD double dist_to_planes(const StepEnv<R>& e, const Trk<R>& t) {
  const double uz = t.uz;
  if (uz > 0.0) return (e.zplane[t.slab + 1] - t.z) / uz;
  if (uz < 0.0) return (e.zplane[t.slab] - t.z) / uz;
  return kInf;
}
template <class R>
EMS_HD double dist_to_walls(const StepEnv<R>& e, const Trk<R>& t) {
  const double h = e.half_xy, ux = t.ux, uy = t.uy;
  const double sx = ux > 0.0 ? (h - t.x) / ux : (ux < 0.0 ? (-h - t.x) / ux : kInf);
  const double sy = uy > 0.0 ? (h - t.y) / uy : (uy < 0.0 ? (-h - t.y) / uy : kInf);
  return sx < sy ? sx : sy;
}

// hand the interaction outcome to the caller: secondaries below the tracking
// cut (gamma, e-) are deposited where they are born, the rest are pushed
template <class R>
EMS_HD void put_sec(Sec<R>& s, const Outcome<R>& oc, int k, Draws& r) {
  s.sp = oc.sp[k];
  s.E = oc.e[k];
  s.ux = oc.u[k].x;
  s.uy = oc.u[k].y;
  s.uz = oc.u[k].z;
  s.id = r.child_id((uint32_t)k);
}
template <class R>
EMS_HD void settle(const StepEnv<R>& e, Trk<R>& t, const Outcome<R>& oc, Draws& r, StepOut<R>& o) {
  // (constant indices only: keeps the small arrays in registers)
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (k >= oc.n) break;
    if (oc.sp[k] != kPositron && oc.e[k] < e.ecut) {
      o.dep += oc.e[k];
      continue;
    }
    if (o.nsec == 0) put_sec(o.sec[0], oc, k, r);
    else put_sec(o.sec[1], oc, k, r);
    o.nsec += 1;
  }
  if (oc.survives) {
    t.E = oc.e_parent;
    t.ux = oc.u_parent.x;
    t.uy = oc.u_parent.y;
    t.uz = oc.u_parent.z;
  } else {
    t.E = 0.0;
    t.slab = -1;
  }
}

// process of a photon's discrete interaction (U1 against the partial sums)
template <class R>
EMS_HD void gamma_select(R sc, R sp, R sig, Draws& r, StepOut<R>& o) {
  const R pick = r.u_at<R>(1) * sig;
  o.process = pick < sc ? kXCompton : (pick < sc + sp ? kXPhot : kXConv);
  o.pending = true;
}

template <class R, int GEO = 0>
EMS_HD void gamma_step(const StepEnv<R>& e, Trk<R>& t, StepOut<R>& o) {
  if (t.E < e.ecut) {
    o.dep += t.E;
    t.E = 0.0;
    t.slab = -1;
    o.limiter = kLimSubcut;
    return;
  }
  const uint32_t m = e.slab_mat[t.slab];
  const double E = t.E;
  const Bin<R> b = bin_of(e, xlog((R)E));
  const R sc = lerp(e.T(m, tCompt), b);
  const R sp = lerp(e.T(m, tPhot), b);
  const R sv = E > 2.0 * kMe ? lerp(e.T(m, tConv), b) : R(0);
  const R sig = sc + sp + sv;
  Face fc{0, 0.0};
  double sz, sw = kInf;
  if constexpr (GEO == 1) {
    sz = box_dist(e, t, fc);
  } else {
    sz = dist_to_planes(e, t);
    sw = dist_to_walls(e, t);
  }
  const double sg = sz <= sw ? sz : sw;
  Draws r;
  r.init(e.seed, t.key, t.id, t.n);
  const double sphys = phys_distance(r, sig, sg);
  if (sg <= sphys) {
    t.x += sg * (double)t.ux;
    t.y += sg * (double)t.uy;
    t.z += sg * (double)t.uz;
    o.step_len = sg;
    if (sz <= sw) {
      o.limiter = kLimZ;
      if constexpr (GEO == 1) box_land(e, t, o, fc);
      else land_on_plane(e, t, o, t.uz > R(0));
    } else {
      o.limiter = kLimWall;
      o.escaped += t.E;
      t.E = 0.0;
      t.slab = -1;
    }
    return;
  }
  t.x += sphys * (double)t.ux;
  t.y += sphys * (double)t.uy;
  t.z += sphys * (double)t.uz;
  o.step_len = sphys;
  o.limiter = kLimDiscrete;
  gamma_select(sc, sp, sig, r, o);
}

// discrete e-/e+ processes: table id and threshold (cross section is zero at
// and below it), in selection order
struct LeptonProcs {
  int n;
  int tab[3];
  double th[3];
  uint32_t code[3];
};
template <class R>
EMS_HD LeptonProcs lepton_procs(const StepEnv<R>& e, bool positron) {
  LeptonProcs p;
  if (positron) {
    p.n = 3;
    p.tab[0] = tBhabha; p.th[0] = e.tcut; p.code[0] = kXBhabha;
    p.tab[1] = tBrem;   p.th[1] = e.kcut; p.code[1] = kXBrem;
    p.tab[2] = tAnnih;  p.th[2] = 0.0;    p.code[2] = kXAnnih;
  } else {
    p.n = 2;
    p.tab[0] = tMoller; p.th[0] = 2.0 * e.tcut; p.code[0] = kXMoller;
    p.tab[1] = tBrem;   p.th[1] = e.kcut;       p.code[1] = kXBrem;
    p.tab[2] = tBrem;   p.th[2] = 0.0;          p.code[2] = kXNone;
  }
  return p;
}

// right-continuous discrete total (process counted at its threshold)
template <class R>
EMS_HD R total_upper(const StepEnv<R>& e, uint32_t m, const LeptonProcs& p, double E, Bin<R> b) {
  R s = R(0);
#pragma unroll
  for (int i = 0; i < 3; ++i)
    if (i < p.n && E >= p.th[i]) s += lerp(e.T(m, p.tab[i]), b);
  return s;
}

// maximum of the discrete total over [a, b]: endpoints, grid nodes and
// thresholds inside; when a is the tracking cut the nodes below b come from
// the running-maximum table; the values at the thresholds are precomputed
template <class R>
EMS_HD R thinning_bound(const StepEnv<R>& e, uint32_t m, const LeptonProcs& p, bool positron, double a, double b,
                        Bin<R> bb, R lnb, bool from_cut, const R* ln_a = nullptr) {
  R best = total_upper(e, m, p, b, bb);
  const R xb = (lnb - e.lnemin) * e.inv_dlog;
  int jb = (int)xceil(xb) - 1;
  jb = jb > (int)e.nodes - 1 ? (int)e.nodes - 1 : jb;
  if (from_cut && jb >= 0) {
    // a is the tracking cut = node 0: the running maximum covers a and the
    // nodes below b
    const R v = e.T(m, positron ? tPMep : tPMem)[jb];
    best = v > best ? v : best;
  } else {
    // ln a: the range table's inverse already interpolated it when a is
    // the energy left after s_max (equal up to the rounding of T - (T - a))
    const R lna = ln_a ? *ln_a : xlog((R)a);
    const R va = total_upper(e, m, p, a, bin_of(e, lna));
    best = va > best ? va : best;
    if (jb >= 0) {
      const R xa = (lna - e.lnemin) * e.inv_dlog;
      int j = (int)xfloor(xa) + 1;
      j = j < 0 ? 0 : j;
      // the nodes' totals (summed over the processes when the tables were
      // packed), kWalk nodes a round with independent loads; a round past
      // jb reads node jb again, which leaves the maximum unchanged
      const R* tot = e.T(m, positron ? tSumEp : tSumEm);
      for (; j <= jb; j += kWalk) {
        R v[kWalk];
#pragma unroll
        for (int k = 0; k < kWalk; ++k) v[k] = tot[j + k <= jb ? j + k : jb];
#pragma unroll
        for (int k = 0; k < kWalk; ++k) best = v[k] > best ? v[k] : best;
      }
    }
  }
  const MatRT& mr = e.mat[m];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (p.th[i] > a && p.th[i] < b) {
      const R v = (R)(positron ? mr.up_ep[i] : mr.up_em[i]);
      best = v > best ? v : best;
    }
  }
  return best;
}

// Optional along-step processes of e-/e+.  Their draws sit far above the
// samplers' (which stop after kMaxTrials trials), so switching them on
// moves no other draw of a step.
constexpr uint32_t kDrawMsc = 1u << 16, kDrawFluct = (1u << 16) + 8u;
constexpr int kFluctTrials = 16;

// Highland's width of the projected angle after a path s (unit charge);
// zero where its logarithmic correction is not positive
template <class R>
EMS_HD R highland_width(double T, double s, double x0) {
  const R p = xsqrt((R)(T * (T + 2.0 * kMe)));
  const R beta = p / (R)(T + kMe);
  const R r = (R)(s / x0);
  const R corr = R(1) + R(0.038) * xlog(r / (beta * beta));
  return corr > R(0) ? R(13.6) / (beta * p) * xsqrt(r) * corr : R(0);
}

// Gaussian multiple scattering: independent normal plane angles of width
// th0 give the space angle th0 sqrt(-2 ln u1) (capped at pi) and a uniform
// azimuth 2 pi u2 about the current direction
template <class R>
EMS_HD void msc_deflect(R th0, Draws& r, Trk<R>& t) {
  const R u1 = r.u_at<R>(kDrawMsc), u2 = r.u_at<R>(kDrawMsc + 1);
  if (!(th0 > R(0))) return;
  R th = th0 * xsqrt(R(-2) * xlog(u1));
  th = th > R(kPi) ? R(kPi) : th;
  R st, ct;
  xsincos(th, &st, &ct);
  const V3T<R> d = about_axis(V3T<R>{t.ux, t.uy, t.uz}, ct, st, R(kTwoPi) * u2);
  t.ux = d.x;
  t.uy = d.y;
  t.uz = d.z;
}

// variance of the restricted loss over a path s: second moment of the
// sub-cut delta rays of the spin-0 Bethe cross section,
// n_el s (2 pi r_e^2 m_e / beta^2) (W_up - beta^2 W_up^2 / (2 W_max))
template <class R>
EMS_HD R loss_variance(double nel, double cut, double T, double s, bool positron) {
  const R g = (R)(T / kMe + 1.0), b2 = R(1) - R(1) / (g * g);
  const R wmax = (R)(positron ? T : 0.5 * T);
  const R wup = (R)cut < wmax ? (R)cut : wmax;
  return (R)(nel * s * (2.0 * kPi * kRe * kRe * kMe)) / b2 * (wup - b2 * wup * wup / (R(2) * wmax));
}

// a loss drawn from the gamma law of the given mean and variance
// (Marsaglia-Tsang 2000; shape raised by one and the result scaled by
// u^(1/k) below k = 1); kFluctTrials trials of three draws at fixed
// indices, after which the mode of the raised shape is taken
template <class R>
EMS_HD R gamma_loss(R mean, R var, Draws& r) {
  const R k = mean * mean / var, theta = var / mean;
  const R kk = k < R(1) ? k + R(1) : k;
  const R d = kk - R(1) / R(3), cc = R(1) / xsqrt(R(9) * d);
  R x = d;
  for (int i = 0; i < kFluctTrials; ++i) {
    const uint32_t b = kDrawFluct + 3u * (uint32_t)i;
    const R u1 = r.u_at<R>(b), u2 = r.u_at<R>(b + 1), u3 = r.u_at<R>(b + 2);
    const R z = xsqrt(R(-2) * xlog(u1)) * xcos(R(kTwoPi) * u2);
    R v = R(1) + cc * z;
    if (v <= R(0)) continue;
    v = v * v * v;
    if (xlog(u3) < R(0.5) * z * z + d - d * v + d * xlog(v)) {
      x = d * v;
      break;
    }
  }
  if (k < R(1)) x *= xpow(r.u_at<R>(kDrawFluct + 3u * kFluctTrials), R(1) / k);
  return x * theta;
}

template <class R, int GEO = 0, int F = kFAll>
EMS_HD void lepton_step(const StepEnv<R>& e, bool positron, Trk<R>& t, StepOut<R>& o, const GeoPre* pre = nullptr) {
  Draws r;
  r.init(e.seed, t.key, t.id, t.n);
  const double T = t.E;
  if (T < e.ecut) {
    o.dep += T;
    o.limiter = kLimSubcut;
    t.E = 0.0;
    if (positron) {
      o.process = kXAnnihRest;  // the track ends with the interaction
      o.pending = true;
    } else {
      t.slab = -1;
    }
    return;
  }
  const uint32_t m = e.slab_mat[t.slab];
  const bool cont = (e.mask & kPCont) != 0;
  const bool fluct = (F & kFFluct) && cont && (e.mask & kPFluct) != 0;
  const R lnT = xlog((R)T);
  const Bin<R> b = bin_of(e, lnT);
  const R* Rt = e.T(m, positron ? tRep : tRem);
  R S = R(0), Rv = (R)kInf, scont = (R)kInf;
  if (cont) {
    S = lerp(e.T(m, positron ? tSep : tSem), b);
    Rv = lerp(Rt, b);
    const R al = (R)e.alpha, rh = (R)e.rho;
    scont = Rv <= rh ? Rv : al * Rv + rh * (R(1) - al) * (R(2) - rh / Rv);
  }
  const bool field = (F & kFField) && e.bz != 0.0;
  Face fc{0, 0.0, 0, -1};
  double sg;
  bool zlim;
  if constexpr (GEO == 1) {
    if (field) {
      // the boundary along the helix, searched up to the continuous-loss
      // limit (beyond it the boundary cannot limit the step)
      const double kap = (positron ? kKB : -kKB) * e.bz / sqrt(T * (T + 2.0 * kMe));
      const double p[3] = {t.x, t.y, t.z}, u[3] = {(double)t.ux, (double)t.uy, (double)t.uz};
      sg = helix_distance(e.nav, t.slab, p, u, kap, (double)scont, fc);
      zlim = true;
      if (!(sg < kInf) && !((double)scont < kInf)) {
        sg = kTwoPi / fabs(kap);  // nothing limits the step: one turn, no crossing
        zlim = false;
      }
    } else {
      if (pre) {
        sg = pre->s;
        fc = pre->fc;
      } else {
        sg = box_dist(e, t, fc);
      }
      zlim = true;
    }
  } else {
    const double sz = dist_to_planes(e, t);
    if (field) {
      const double ax = fabs(t.x), ay = fabs(t.y);
      const double dw = e.half_xy - (ax > ay ? ax : ay);
      if (dw < kSafetyMin) {
        o.limiter = kLimEscapeSafety;
        o.escaped += T;
        t.E = 0.0;
        t.slab = -1;
        return;
      }
      zlim = sz <= dw;
      sg = zlim ? sz : dw;
    } else {
      // The distance along the track to a transverse wall is at least the
      // perpendicular distance to the nearest wall (|u_x|, |u_y| <= 1 up to
      // the rounding of a unit vector, covered by the 2^-20 margin), so the
      // wall can only limit the step when that perpendicular distance does
      // not exceed the plane distance; otherwise sz <= sw holds and the two
      // divisions are skipped, with the same result.
      double sw = kInf;
      const double ax = fabs(t.x), ay = fabs(t.y);
      const double dperp = e.half_xy - (ax > ay ? ax : ay);
      if (!(dperp * (1.0 - 0x1p-20) > sz)) sw = dist_to_walls(e, t);
      zlim = sz <= sw;
      sg = zlim ? sz : sw;
    }
  }
  const double smax = (double)scont <= sg ? (double)scont : sg;
  double elo = T, loss_max = 0.0;
  R ln_lo = R(0);
  bool have_ln = false;
  if (cont) {
    // (FP64 form only: in the mixed form the longer live range of the
    // logarithm costs the register-limited kernel more than the log saves)
    loss_max = sizeof(R) == 8 ? cont_loss(e, Rt, b.j, T, S, Rv, smax, &ln_lo, &have_ln)
                              : cont_loss(e, Rt, b.j, T, S, Rv, smax);
    elo = T - loss_max;
    const R lin = (R)e.lin * Rv;
    if (smax >= (double)lin) {
      const double e2 = T - (double)(lin * S);
      if (e2 < elo) {
        elo = e2;
        have_ln = false;
      }
    }
  }
  const bool from_cut = fluct || !(elo > e.ecut);  // with fluctuations: anything down to the cut
  const double a = from_cut ? e.ecut : elo;
  const LeptonProcs pl = lepton_procs(e, positron);
  const R bound = thinning_bound(e, m, pl, positron, a, T, b, lnT, from_cut, have_ln ? &ln_lo : nullptr);
  const double sphys = phys_distance(r, bound, smax);
  double s;
  uint32_t lim;
  if (sphys < smax) {
    s = sphys;
    lim = kLimDiscrete;
  } else if (sg <= (double)scont) {
    s = sg;
    lim = zlim ? kLimZ : (field ? kLimSafety : kLimWall);
  } else {
    s = (double)scont;
    lim = kLimCont;
  }
  if (field) {
    // exact helix about z (FP64 in both forms)
    const double p = sqrt(T * (T + 2.0 * kMe));
    const double kap = (positron ? kKB : -kKB) * e.bz / p;
    const double ph = kap * s;
    // sin and cos of the turn from those of its half (one reduction):
    // sin = 2 sh ch, 1 - cos = 2 sh^2 (no cancellation for small turns)
    double sh, ch;
    sincos(0.5 * ph, &sh, &ch);
    const double sp = 2.0 * sh * ch, omc = 2.0 * sh * sh, cp = 1.0 - omc;
    const double ux = t.ux, uy = t.uy;
    t.x += (ux * sp + uy * omc) / kap;
    t.y += (uy * sp - ux * omc) / kap;
    t.z += (double)t.uz * s;
    t.ux = (R)(ux * cp + uy * sp);
    t.uy = (R)(-ux * sp + uy * cp);
  } else {
    t.x += s * (double)t.ux;
    t.y += s * (double)t.uy;
    t.z += s * (double)t.uz;
  }
  o.step_len = s;
  o.clen += s;
  // the step ends at s_max unless a discrete interaction came first
  double dE = !cont ? 0.0 : (lim == kLimDiscrete ? cont_loss(e, Rt, b.j, T, S, Rv, s) : loss_max);
  if (fluct && dE > 0.0 && dE < T) {
    const R var = loss_variance<R>(e.mat[m].nel, e.tcut, T, s, positron);
    if (var > R(0)) {
      const double x = (double)gamma_loss<R>((R)dE, var, r);
      dE = x > T ? T : x;
    }
  }
  o.dep += dE;
  const double Tp = T - dE;
  t.E = Tp;
  o.limiter = lim;
  if (Tp == 0.0) {
    o.limiter = kLimStopped;
    if (positron) {
      o.process = kXAnnihRest;
      o.pending = true;
    } else {
      t.slab = -1;
    }
    return;
  }
  const bool up = t.uz > R(0);  // the plane reached, fixed before any deflection
  if ((F & kFMsc) && (e.mask & kPMsc) && s > 0.0) msc_deflect(highland_width<R>(T, s, e.mat[m].x0), r, t);
  if (lim == kLimZ) {
    if constexpr (GEO == 1) box_land(e, t, o, fc);
    else land_on_plane(e, t, o, up);
    return;
  }
  if (lim == kLimWall) {
    o.escaped += Tp;
    t.E = 0.0;
    t.slab = -1;
    return;
  }
  if (lim != kLimDiscrete) return;
  const R pick = r.u_at<R>(1) * bound;
  const Bin<R> bp = bin_of(e, xlog((R)Tp));
  R cum = R(0);
  uint32_t code = kXNull;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (i >= pl.n || code != kXNull) continue;
    if (Tp > pl.th[i]) cum += lerp(e.T(m, pl.tab[i]), bp);
    if (pick < cum) code = pl.code[i];
  }
  if (code == kXNull) {
    o.process = kXNull;
    o.null += 1;
    return;
  }
  o.process = code;
  o.pending = true;
}

// Target element of a pair (w = 0) or bremsstrahlung (w = 1) interaction at
// energy E in material m.  In a compound the next draw u picks the first
// element whose running sum of interpolated partial totals exceeds u times
// their sum; a single element takes no draw.
template <int F, class R>
EMS_HD MatRT target_element(const StepEnv<R>& e, uint32_t m, int w, double E, Draws& r) {
  MatRT me = e.mat[m];
  const uint32_t n = me.n_el;
  if (!(F & kFCompound) || n <= 1) return me;
  const R u = r.u<R>();
  const Bin<R> b = bin_of(e, xlog((R)E));
  R s[kMaxElements];
  R tot = R(0);
#pragma unroll
  for (int i = 0; i < kMaxElements; ++i) {
    s[i] = (uint32_t)i < n ? lerp(e.elt + (((size_t)m * kMaxElements + i) * 2 + w) * e.nodes, b) : R(0);
    tot += s[i];
  }
  uint32_t k = n - 1;
  R cum = R(0);
  bool found = false;
#pragma unroll
  for (int i = 0; i + 1 < kMaxElements; ++i) {
    if ((uint32_t)i + 1 >= n || found) continue;
    cum += s[i];
    if (u * tot < cum) {
      k = (uint32_t)i;
      found = true;
    }
  }
  me.c136 = e.elc[((size_t)m * kMaxElements + k) * 2];
  me.gshift = e.elc[((size_t)m * kMaxElements + k) * 2 + 1];
  return me;
}

// The discrete interaction selected by the step (o.process, o.pending):
// sampling from the step's draws U2, U3, ... (U1, U2 for annihilation at
// rest), secondaries handed out, parent updated, then the step counter and
// watchdog.  Running it right after the step or later in a batch with other
// tracks gives the same result.  KIND: 0 = photon processes only, 1 = e-/e+
// processes only, 2 = any.
template <int KIND, int F = kFAll, class R>
EMS_HD void interact(const StepEnv<R>& e, Trk<R>& t, StepOut<R>& o) {
  Draws r;
  r.init(e.seed, t.key, t.id, t.n);
  Outcome<R> oc;
  const double E = t.E;
  const V3T<R> u{t.ux, t.uy, t.uz};
  const uint32_t m = e.slab_mat[t.slab];
  const uint32_t p = o.process;
  if (KIND != 1 && p == kXCompton) {
    compton(E, u, r, oc);
  } else if (KIND != 1 && p == kXPhot) {
    photo(E, u, oc);
  } else if (KIND != 1 && p == kXConv) {
    pair(target_element<F>(e, m, 0, E, r), E, u, r, oc);
    o.pair += 1;
  } else if (KIND != 0 && p == kXMoller) {
    moller(E, e.tcut, u, r, oc);
  } else if (KIND != 0 && p == kXBhabha) {
    bhabha(E, e.tcut, u, r, oc);
  } else if (KIND != 0 && p == kXBrem) {
    brem(target_element<F>(e, m, 1, E, r), E, e.kcut, u, r, oc);
  } else if (KIND != 0 && p == kXAnnih) {
    annihilate(E, u, r, oc);
    o.annih += 1;
  } else if (KIND != 0) {  // kXAnnihRest
    annihilate_at_rest(r, oc);
    o.annih += 1;
  } else {
    oc.survives = true;  // not reached: photon steps select only the three above
    oc.e_parent = E;
    oc.u_parent = u;
    oc.n = 0;
  }
  settle(e, t, oc, r, o);
  o.pending = false;
  watchdog(e, t, o);
}

template <class R>
EMS_HD void clear_out(const Trk<R>& t, StepOut<R>& o) {
  o.nsec = 0;
  o.slab = t.slab;
  o.dep = o.escaped = o.killed = o.clen = o.step_len = 0.0;
  o.pair = o.annih = o.null = 0;
  o.limiter = 0;
  o.process = kXNone;
  o.pending = false;
}

template <class R>
EMS_HD void watchdog(const StepEnv<R>& e, Trk<R>& t, StepOut<R>& o) {
  t.n += 1;
  if (t.slab >= 0 && t.n >= e.max_steps) {
    o.killed += t.E;
    t.E = 0.0;
    t.slab = -1;
  }
}

// One full step of a track of species sp: dispatch, step counter, watchdog.
// KIND: 0 = photons only, 1 = e-/e+ only, 2 = any species (host use).
template <int KIND, class R, int GEO = 0>
EMS_HD void take_step_k(const StepEnv<R>& e, int sp, Trk<R>& t, StepOut<R>& o) {
  clear_out(t, o);
  if (KIND == 0 || (KIND == 2 && sp == kGamma)) gamma_step<R, GEO>(e, t, o);
  else lepton_step<R, GEO>(e, sp == kPositron, t, o);
  if (o.pending) interact<KIND>(e, t, o);
  else watchdog(e, t, o);
}
template <class R, int GEO = 0>
EMS_HD void take_step(const StepEnv<R>& e, int sp, Trk<R>& t, StepOut<R>& o) {
  take_step_k<2, R, GEO>(e, sp, t, o);
}

// Photon visit state: between interactions a photon keeps its energy and
// direction, so ln E, its table bin and the inverse direction are computed
// once per visit; each crossing then costs one Philox block, one log and the
// geometry.
template <class R>
struct PhotonCache {
  Bin<R> b;
  bool conv;
  double iux, iuy, iuz;
};

template <class R>
EMS_HD void photon_begin(const StepEnv<R>& e, const Trk<R>& t, PhotonCache<R>& pc) {
  pc.b = bin_of(e, xlog((R)(t.E > e.ecut ? t.E : e.ecut)));
  pc.conv = t.E > 2.0 * kMe;
  pc.iux = 1.0 / (double)t.ux;
  pc.iuy = 1.0 / (double)t.uy;
  pc.iuz = 1.0 / (double)t.uz;
}

// One photon step with the visit cache: exactly gamma_step followed by the
// step count and watchdog of take_step.  Returns true when the visit must
// end after it (the photon interacted or is gone).
template <class R, int GEO = 0>
EMS_HD bool photon_substep(const StepEnv<R>& e, const PhotonCache<R>& pc, Trk<R>& t, StepOut<R>& o,
                           const GeoPre* pre = nullptr) {
  clear_out(t, o);
  const double E = t.E;
  if (E < e.ecut) {
    o.dep += E;
    t.E = 0.0;
    t.slab = -1;
    o.limiter = kLimSubcut;
  } else {
    const uint32_t m = e.slab_mat[t.slab];
    const R sc = lerp(e.T(m, tCompt), pc.b);
    const R sp = lerp(e.T(m, tPhot), pc.b);
    const R sv = pc.conv ? lerp(e.T(m, tConv), pc.b) : R(0);
    const R sig = sc + sp + sv;
    const double ux = t.ux, uy = t.uy, uz = t.uz;
    Face fc{0, 0.0};
    double sz, sw;
    if constexpr (GEO == 1) {
      if (pre) {
        sz = pre->s;
        fc = pre->fc;
      } else {
        const double iu[3] = {pc.iux, pc.iuy, pc.iuz};
        sz = box_dist(e, t, fc, iu);
      }
      sw = kInf;
    } else {
      const double h = e.half_xy;
      sz = uz > 0.0 ? (e.zplane[t.slab + 1] - t.z) * pc.iuz : (uz < 0.0 ? (e.zplane[t.slab] - t.z) * pc.iuz : kInf);
      const double sx = ux > 0.0 ? (h - t.x) * pc.iux : (ux < 0.0 ? (-h - t.x) * pc.iux : kInf);
      const double sy = uy > 0.0 ? (h - t.y) * pc.iuy : (uy < 0.0 ? (-h - t.y) * pc.iuy : kInf);
      sw = sx < sy ? sx : sy;
    }
    const double sg = sz <= sw ? sz : sw;
    Draws r;
    r.init(e.seed, t.key, t.id, t.n);
    const double sphys = phys_distance(r, sig, sg);
    if (sg <= sphys) {
      t.x += sg * ux;
      t.y += sg * uy;
      t.z += sg * uz;
      o.step_len = sg;
      if (sz <= sw) {
        o.limiter = kLimZ;
        if constexpr (GEO == 1) box_land(e, t, o, fc);
        else land_on_plane(e, t, o, t.uz > R(0));
      } else {
        o.limiter = kLimWall;
        o.escaped += t.E;
        t.E = 0.0;
        t.slab = -1;
      }
    } else {
      t.x += sphys * ux;
      t.y += sphys * uy;
      t.z += sphys * uz;
      o.step_len = sphys;
      o.limiter = kLimDiscrete;
      gamma_select(sc, sp, sig, r, o);
    }
  }
  if (!o.pending) watchdog(e, t, o);
  // any interaction changes E and u (even one whose electron was deposited
  // on the spot), so the visit ends there
  return t.slab < 0 || o.limiter == kLimDiscrete;
}

// Per-lane state of a visit.  KIND: 0 = photons, 1 = e-/e+, 2 = any (host).
template <class R>
struct VisitState {
  PhotonCache<R> pc;
  int steps;  // steps taken in this visit
};

template <int KIND, class R>
EMS_HD void visit_begin(const StepEnv<R>& e, int sp, const Trk<R>& t, VisitState<R>& vs) {
  vs.steps = 0;
  if (KIND == 0 || (KIND == 2 && sp == kGamma)) photon_begin(e, t, vs.pc);
}

// One step of a visit; returns true when the visit ends after it.  A visit
// is a run of consecutive steps of one track by one thread; it ends at a
// step with a discrete interaction (every real one changes the track and
// all but a few create secondaries), when the track ends, or after
// max_steps steps.  Every step draws from its own (id, step) stream, so a
// run of visits is step for step the one-step-at-a-time loop.  The step's
// interaction is left pending (o.pending) for the caller to run with
// interact(), so that a wave samples its interactions together.
template <int KIND, class R, int GEO = 0, int F = kFAll>
EMS_HD bool visit_step(const StepEnv<R>& e, int sp, VisitState<R>& vs, Trk<R>& t, StepOut<R>& o, int max_steps,
                       const GeoPre* pre = nullptr) {
  bool end;
  if (KIND == 0 || (KIND == 2 && sp == kGamma)) {
    end = photon_substep<R, GEO>(e, vs.pc, t, o, pre);
  } else {
    clear_out(t, o);
    lepton_step<R, GEO, F>(e, sp == kPositron, t, o, pre);
    if (!o.pending) watchdog(e, t, o);
    end = t.slab < 0 || o.pending;
  }
  vs.steps += 1;
  return end || vs.steps >= max_steps;
}

}  // namespace ems
