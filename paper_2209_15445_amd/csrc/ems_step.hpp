// ems_step.hpp -- one transport step of one track.
//
// This is the per-thread body of the paper's stepping workflow (section 3):
// a thread takes one track of a species' current array, moves it one step
// (physics step limit, geometry limit, field propagation, continuous loss,
// discrete interaction) and hands back the surviving track plus at most two
// secondaries, which the caller appends to the next arrays.  The function is
// pure: every random number comes from the (seed, event key, id, step) Philox
// stream, so results do not depend on which thread or iteration runs it.
#pragma once
#include "ems_models.hpp"
#include "ems_tables.hpp"

namespace ems {

constexpr double kInf = __builtin_huge_val();

// Tables are held in two blocks so each kernel stages only its own: the
// photon block [mat][3][nodes] (tables 0..2) and the lepton block
// [mat][10][nodes] (tables 3..12).
constexpr int kGammaTables = 3, kLeptonTables = kNumTables - kGammaTables;

struct StepEnv {
  const double* tg;          // photon table block
  const double* tl;          // lepton table block
  const double* zplane;      // n_slabs + 1
  const uint32_t* slab_mat;  // n_slabs
  const MatRT* mat;
  uint32_t nodes, n_slabs;
  double lnemin, dlog, inv_dlog;
  double half_xy, bz;
  double ecut, tcut, kcut;
  double alpha, rho, lin;
  uint32_t mask, seed, max_steps;

  EMS_HD const double* T(uint32_t m, int t) const {
    return t < kGammaTables ? tg + ((size_t)m * kGammaTables + t) * nodes
                            : tl + ((size_t)m * kLeptonTables + (t - kGammaTables)) * nodes;
  }
};

struct Trk {
  double x, y, z, ux, uy, uz, E;
  uint64_t id;
  uint32_t ev, key, n;
  int32_t slab;  // < 0: track has ended
};

struct Sec {
  int sp;
  double E, ux, uy, uz;
  uint64_t id;
};

struct StepOut {
  int nsec;
  Sec sec[2];
  int slab;        // slab the step was taken in (deposits, secondaries)
  double dep;      // energy deposited in that slab
  double escaped;  // kinetic energy of the track leaving the stack
  double killed;   // kinetic energy removed by the watchdog
  double clen;     // charged path length
  int pair, annih, null;
  uint32_t limiter, process;
  double step_len;
};

struct Bin {
  int j;
  double u;
};

EMS_HD Bin bin_of(const StepEnv& e, double lnE) {
  const double x = (lnE - e.lnemin) * e.inv_dlog;
  double f = floor(x);
  const double top = (double)(e.nodes - 2);
  f = f < 0.0 ? 0.0 : (f > top ? top : f);
  int j = (int)f;  // clamped again as an integer: a NaN never indexes outside
  j = j < 0 ? 0 : (j > (int)e.nodes - 2 ? (int)e.nodes - 2 : j);
  double u = x - (double)j;
  u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
  return Bin{j, u};
}
EMS_HD double lerp(const double* f, Bin b) { return f[b.j] + b.u * (f[b.j + 1] - f[b.j]); }

// largest node j <= jhi with R_j <= r (0 if none; clamped to the last bin),
// then the exact inverse of the range interpolant.  The loss over one step
// spans few bins, so the scan starts at the track's own bin and walks down.
EMS_HD double inverse_range(const StepEnv& e, const double* R, double r, int jhi) {
  int lo = jhi > (int)e.nodes - 1 ? (int)e.nodes - 1 : jhi;
  while (lo > 0 && R[lo] > r) --lo;
  if (lo > (int)e.nodes - 2) lo = (int)e.nodes - 2;
  return exp(e.lnemin + lo * e.dlog + e.dlog * (r - R[lo]) / (R[lo + 1] - R[lo]));
}

// energy lost over path s by a charged track of kinetic energy T
EMS_HD double cont_loss(const StepEnv& e, const double* R, int jT, double T, double S, double Rt, double s) {
  double L;
  if (s >= Rt) L = T;
  else if (s < e.lin * Rt) L = s * S;
  else L = T - inverse_range(e, R, Rt - s, jT + 1);
  return (T - L < e.ecut) ? T : L;
}

EMS_HD void land_on_plane(const StepEnv& e, Trk& t, StepOut& o) {
  if (t.uz > 0.0) {
    t.z = e.zplane[t.slab + 1];
    t.slab += 1;
  } else {
    t.z = e.zplane[t.slab];
    t.slab -= 1;
  }
  if (t.slab < 0 || t.slab >= (int)e.n_slabs) {
    o.escaped += t.E;
    t.E = 0.0;
    t.slab = -1;
  }
}

EMS_HD double dist_to_planes(const StepEnv& e, const Trk& t) {
  if (t.uz > 0.0) return (e.zplane[t.slab + 1] - t.z) / t.uz;
  if (t.uz < 0.0) return (e.zplane[t.slab] - t.z) / t.uz;
  return kInf;
}
EMS_HD double dist_to_walls(const StepEnv& e, const Trk& t) {
  const double h = e.half_xy;
  const double sx = t.ux > 0.0 ? (h - t.x) / t.ux : (t.ux < 0.0 ? (-h - t.x) / t.ux : kInf);
  const double sy = t.uy > 0.0 ? (h - t.y) / t.uy : (t.uy < 0.0 ? (-h - t.y) / t.uy : kInf);
  return sx < sy ? sx : sy;
}

// hand the interaction outcome to the caller: secondaries below the tracking
// cut (gamma, e-) are deposited where they are born, the rest are pushed
EMS_HD void put_sec(Sec& s, const Outcome& oc, int k, Draws& r) {
  s.sp = oc.sp[k];
  s.E = oc.e[k];
  s.ux = oc.u[k].x;
  s.uy = oc.u[k].y;
  s.uz = oc.u[k].z;
  s.id = r.child_id((uint32_t)k);
}
EMS_HD void settle(const StepEnv& e, Trk& t, const Outcome& oc, Draws& r, StepOut& o) {
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

EMS_HD void gamma_step(const StepEnv& e, Trk& t, StepOut& o) {
  if (t.E < e.ecut) {
    o.dep += t.E;
    t.E = 0.0;
    t.slab = -1;
    o.limiter = kLimSubcut;
    return;
  }
  const uint32_t m = e.slab_mat[t.slab];
  const double E = t.E;
  const Bin b = bin_of(e, log(E));
  const double sc = lerp(e.T(m, tCompt), b);
  const double sp = lerp(e.T(m, tPhot), b);
  const double sv = E > 2.0 * kMe ? lerp(e.T(m, tConv), b) : 0.0;
  const double sig = sc + sp + sv;
  const double sz = dist_to_planes(e, t), sw = dist_to_walls(e, t);
  const double sg = sz <= sw ? sz : sw;
  Draws r;
  r.init(e.seed, t.key, t.id, t.n);
  const double sphys = sig > 0.0 ? -log(r.at(0)) / sig : kInf;
  if (sg <= sphys) {
    t.x += sg * t.ux;
    t.y += sg * t.uy;
    t.z += sg * t.uz;
    o.step_len = sg;
    if (sz <= sw) {
      o.limiter = kLimZ;
      land_on_plane(e, t, o);
    } else {
      o.limiter = kLimWall;
      o.escaped += t.E;
      t.E = 0.0;
      t.slab = -1;
    }
    return;
  }
  t.x += sphys * t.ux;
  t.y += sphys * t.uy;
  t.z += sphys * t.uz;
  o.step_len = sphys;
  o.limiter = kLimDiscrete;
  const double pick = r.at(1) * sig;
  const V3 u{t.ux, t.uy, t.uz};
  Outcome oc;
  if (pick < sc) {
    o.process = kXCompton;
    compton(E, u, r, oc);
  } else if (pick < sc + sp) {
    o.process = kXPhot;
    photo(E, u, oc);
  } else {
    o.process = kXConv;
    pair(e.mat[m], E, u, r, oc);
    o.pair += 1;
  }
  settle(e, t, oc, r, o);
}

// discrete e-/e+ processes: table id and threshold (cross section is zero at
// and below it), in selection order
struct LeptonProcs {
  int n;
  int tab[3];
  double th[3];
  uint32_t code[3];
};
EMS_HD LeptonProcs lepton_procs(const StepEnv& e, bool positron) {
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
EMS_HD double total_upper(const StepEnv& e, uint32_t m, const LeptonProcs& p, double E, Bin b) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
    if (i < p.n && E >= p.th[i]) s += lerp(e.T(m, p.tab[i]), b);
  return s;
}

// maximum of the discrete total over [a, b]: endpoints, grid nodes and
// thresholds inside; when a is the tracking cut the nodes below b come from
// the running-maximum table; the values at the thresholds are precomputed
EMS_HD double thinning_bound(const StepEnv& e, uint32_t m, const LeptonProcs& p, bool positron, double a,
                             double b, Bin bb, double lnb, bool from_cut) {
  double best = total_upper(e, m, p, b, bb);
  const double xb = (lnb - e.lnemin) * e.inv_dlog;
  int jb = (int)ceil(xb) - 1;
  jb = jb > (int)e.nodes - 1 ? (int)e.nodes - 1 : jb;
  if (from_cut && jb >= 0) {
    // a is the tracking cut = node 0: the running maximum covers a and the
    // nodes below b
    const double v = e.T(m, positron ? tPMep : tPMem)[jb];
    best = v > best ? v : best;
  } else {
    const double lna = log(a);
    const double va = total_upper(e, m, p, a, bin_of(e, lna));
    best = va > best ? va : best;
    if (jb >= 0) {
      const double xa = (lna - e.lnemin) * e.inv_dlog;
      int j = (int)floor(xa) + 1;
      j = j < 0 ? 0 : j;
      for (; j <= jb; ++j) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
          if (i < p.n) s += e.T(m, p.tab[i])[j];
        best = s > best ? s : best;
      }
    }
  }
  const MatRT& mr = e.mat[m];
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (p.th[i] > a && p.th[i] < b) {
      const double v = positron ? mr.up_ep[i] : mr.up_em[i];
      best = v > best ? v : best;
    }
  }
  return best;
}

EMS_HD void lepton_step(const StepEnv& e, bool positron, Trk& t, StepOut& o) {
  Draws r;
  r.init(e.seed, t.key, t.id, t.n);
  Outcome oc;
  const double T = t.E;
  if (T < e.ecut) {
    o.dep += T;
    o.limiter = kLimSubcut;
    t.E = 0.0;
    if (positron) {
      o.process = kXAnnihRest;
      annihilate_at_rest(r, oc);
      o.annih += 1;
      settle(e, t, oc, r, o);
    }
    t.slab = -1;
    return;
  }
  const bool field = e.bz != 0.0;
  const double sz = dist_to_planes(e, t);
  double sg;
  bool zlim;
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
    const double sw = dist_to_walls(e, t);
    zlim = sz <= sw;
    sg = zlim ? sz : sw;
  }
  const uint32_t m = e.slab_mat[t.slab];
  const bool cont = (e.mask & kPCont) != 0;
  const double lnT = log(T);
  const Bin b = bin_of(e, lnT);
  const double* Rt = e.T(m, positron ? tRep : tRem);
  double S = 0.0, R = kInf, scont = kInf;
  if (cont) {
    S = lerp(e.T(m, positron ? tSep : tSem), b);
    R = lerp(Rt, b);
    scont = R <= e.rho ? R : e.alpha * R + e.rho * (1.0 - e.alpha) * (2.0 - e.rho / R);
  }
  const double smax = scont <= sg ? scont : sg;
  double elo = T, loss_max = 0.0;
  if (cont) {
    loss_max = cont_loss(e, Rt, b.j, T, S, R, smax);
    elo = T - loss_max;
    const double lin = e.lin * R;
    if (smax >= lin) {
      const double e2 = T - lin * S;
      elo = e2 < elo ? e2 : elo;
    }
  }
  const bool from_cut = !(elo > e.ecut);
  const double a = from_cut ? e.ecut : elo;
  const LeptonProcs pl = lepton_procs(e, positron);
  const double bound = thinning_bound(e, m, pl, positron, a, T, b, lnT, from_cut);
  const double sphys = bound > 0.0 ? -log(r.at(0)) / bound : kInf;
  double s;
  uint32_t lim;
  if (sphys < smax) {
    s = sphys;
    lim = kLimDiscrete;
  } else if (sg <= scont) {
    s = sg;
    lim = zlim ? kLimZ : (field ? kLimSafety : kLimWall);
  } else {
    s = scont;
    lim = kLimCont;
  }
  if (field) {
    const double p = sqrt(T * (T + 2.0 * kMe));
    const double kap = (positron ? kKB : -kKB) * e.bz / p;
    const double ph = kap * s;
    const double sp = sin(ph), cp = cos(ph), h = sin(0.5 * ph);
    const double omc = 2.0 * h * h;
    const double ux = t.ux, uy = t.uy;
    t.x += (ux * sp + uy * omc) / kap;
    t.y += (uy * sp - ux * omc) / kap;
    t.z += t.uz * s;
    t.ux = ux * cp + uy * sp;
    t.uy = -ux * sp + uy * cp;
  } else {
    t.x += s * t.ux;
    t.y += s * t.uy;
    t.z += s * t.uz;
  }
  o.step_len = s;
  o.clen += s;
  // the step ends at s_max unless a discrete interaction came first
  const double dE = !cont ? 0.0 : (lim == kLimDiscrete ? cont_loss(e, Rt, b.j, T, S, R, s) : loss_max);
  o.dep += dE;
  const double Tp = T - dE;
  t.E = Tp;
  o.limiter = lim;
  if (Tp == 0.0) {
    o.limiter = kLimStopped;
    if (positron) {
      o.process = kXAnnihRest;
      annihilate_at_rest(r, oc);
      o.annih += 1;
      settle(e, t, oc, r, o);
    }
    t.slab = -1;
    return;
  }
  if (lim == kLimZ) {
    land_on_plane(e, t, o);
    return;
  }
  if (lim == kLimWall) {
    o.escaped += Tp;
    t.E = 0.0;
    t.slab = -1;
    return;
  }
  if (lim != kLimDiscrete) return;
  const double pick = r.at(1) * bound;
  const Bin bp = bin_of(e, log(Tp));
  double cum = 0.0;
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
  const V3 u{t.ux, t.uy, t.uz};
  switch (code) {
    case kXMoller: moller(Tp, e.tcut, u, r, oc); break;
    case kXBhabha: bhabha(Tp, e.tcut, u, r, oc); break;
    case kXBrem: brem(e.mat[m], Tp, e.kcut, u, r, oc); break;
    default:
      annihilate(Tp, u, r, oc);
      o.annih += 1;
      break;
  }
  settle(e, t, oc, r, o);
}

// One full step of a track of species sp: dispatch, step counter, watchdog.
// KIND: 0 = photons only, 1 = e-/e+ only, 2 = any species (host use).
template <int KIND>
EMS_HD void take_step_k(const StepEnv& e, int sp, Trk& t, StepOut& o) {
  o.nsec = 0;
  o.slab = t.slab;
  o.dep = o.escaped = o.killed = o.clen = o.step_len = 0.0;
  o.pair = o.annih = o.null = 0;
  o.limiter = 0;
  o.process = kXNone;
  if (KIND == 0 || (KIND == 2 && sp == kGamma)) gamma_step(e, t, o);
  else lepton_step(e, sp == kPositron, t, o);
  t.n += 1;
  if (t.slab >= 0 && t.n >= e.max_steps) {
    o.killed += t.E;
    t.E = 0.0;
    t.slab = -1;
  }
}
EMS_HD void take_step(const StepEnv& e, int sp, Trk& t, StepOut& o) { take_step_k<2>(e, sp, t, o); }

// A visit: consecutive steps of one track by one thread, until a step
// produces secondaries, the track ends, or max_steps steps were taken.  The
// sequence of steps is exactly the one-step-at-a-time sequence (every step
// draws from its own (id, step) stream); only the queue round trips between
// them are saved.  Steps without secondaries are handed to sink.apply() as
// they happen.  If the last step produced secondaries it is NOT applied: `o`
// holds it, `before` holds the track as it was before that step, and the
// caller either commits it (sink.apply + push) or carries `before`.
// Returns the number of steps taken.
// Photon visit state: between interactions a photon keeps its energy and
// direction, so ln E, its table bin and the inverse direction are computed
// once per visit; each crossing then costs one Philox block, one log and the
// geometry.
struct PhotonCache {
  Bin b;
  bool conv;
  double iux, iuy, iuz;
};

EMS_HD void photon_begin(const StepEnv& e, const Trk& t, PhotonCache& pc) {
  pc.b = bin_of(e, log(t.E > e.ecut ? t.E : e.ecut));
  pc.conv = t.E > 2.0 * kMe;
  pc.iux = 1.0 / t.ux;
  pc.iuy = 1.0 / t.uy;
  pc.iuz = 1.0 / t.uz;
}

// One photon step with the visit cache: exactly gamma_step followed by the
// step count and watchdog of take_step.  Returns true when the visit must
// end after it (the photon interacted or is gone).
EMS_HD bool photon_substep(const StepEnv& e, const PhotonCache& pc, Trk& t, StepOut& o) {
  o.nsec = 0;
  o.slab = t.slab;
  o.dep = o.escaped = o.killed = o.clen = o.step_len = 0.0;
  o.pair = o.annih = o.null = 0;
  o.limiter = 0;
  o.process = kXNone;
  const double E = t.E;
  if (E < e.ecut) {
    o.dep += E;
    t.E = 0.0;
    t.slab = -1;
    o.limiter = kLimSubcut;
  } else {
    const uint32_t m = e.slab_mat[t.slab];
    const double sc = lerp(e.T(m, tCompt), pc.b);
    const double sp = lerp(e.T(m, tPhot), pc.b);
    const double sv = pc.conv ? lerp(e.T(m, tConv), pc.b) : 0.0;
    const double sig = sc + sp + sv;
    const double h = e.half_xy;
    const double sz = t.uz > 0.0 ? (e.zplane[t.slab + 1] - t.z) * pc.iuz
                                 : (t.uz < 0.0 ? (e.zplane[t.slab] - t.z) * pc.iuz : kInf);
    const double sx = t.ux > 0.0 ? (h - t.x) * pc.iux : (t.ux < 0.0 ? (-h - t.x) * pc.iux : kInf);
    const double sy = t.uy > 0.0 ? (h - t.y) * pc.iuy : (t.uy < 0.0 ? (-h - t.y) * pc.iuy : kInf);
    const double sw = sx < sy ? sx : sy;
    const double sg = sz <= sw ? sz : sw;
    Draws r;
    r.init(e.seed, t.key, t.id, t.n);
    const double sphys = sig > 0.0 ? -log(r.at(0)) / sig : kInf;
    if (sg <= sphys) {
      t.x += sg * t.ux;
      t.y += sg * t.uy;
      t.z += sg * t.uz;
      o.step_len = sg;
      if (sz <= sw) {
        o.limiter = kLimZ;
        land_on_plane(e, t, o);
      } else {
        o.limiter = kLimWall;
        o.escaped += t.E;
        t.E = 0.0;
        t.slab = -1;
      }
    } else {
      t.x += sphys * t.ux;
      t.y += sphys * t.uy;
      t.z += sphys * t.uz;
      o.step_len = sphys;
      o.limiter = kLimDiscrete;
      const double pick = r.at(1) * sig;
      const V3 u{t.ux, t.uy, t.uz};
      Outcome oc;
      if (pick < sc) {
        o.process = kXCompton;
        compton(E, u, r, oc);
      } else if (pick < sc + sp) {
        o.process = kXPhot;
        photo(E, u, oc);
      } else {
        o.process = kXConv;
        pair(e.mat[m], E, u, r, oc);
        o.pair += 1;
      }
      settle(e, t, oc, r, o);
    }
  }
  t.n += 1;
  if (t.slab >= 0 && t.n >= e.max_steps) {
    o.killed += t.E;
    t.E = 0.0;
    t.slab = -1;
  }
  // any interaction changes E and u (even one whose electron was deposited
  // on the spot), so the visit ends there
  return t.slab < 0 || o.limiter == kLimDiscrete;
}

// Per-lane state of a visit.  KIND: 0 = photons, 1 = e-/e+, 2 = any (host).
struct VisitState {
  PhotonCache pc;
  int steps;  // steps taken in this visit
};

template <int KIND>
EMS_HD void visit_begin(const StepEnv& e, int sp, const Trk& t, VisitState& vs) {
  vs.steps = 0;
  if (KIND == 0 || (KIND == 2 && sp == kGamma)) photon_begin(e, t, vs.pc);
}

// One step of a visit; returns true when the visit ends after it.  A visit
// is a run of consecutive steps of one track by one thread; it ends at a
// step that creates secondaries, when the track ends, or after max_steps
// steps.  Every step draws from its own (id, step) stream, so a run of
// visits is step for step the one-step-at-a-time loop.
template <int KIND>
EMS_HD bool visit_step(const StepEnv& e, int sp, VisitState& vs, Trk& t, StepOut& o, int max_steps) {
  bool end;
  if (KIND == 0 || (KIND == 2 && sp == kGamma)) {
    end = photon_substep(e, vs.pc, t, o);
  } else {
    take_step_k<1>(e, sp, t, o);
    end = t.slab < 0;
  }
  vs.steps += 1;
  return end || o.nsec > 0 || vs.steps >= max_steps;
}

}  // namespace ems
