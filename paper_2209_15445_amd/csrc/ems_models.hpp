// ems_models.hpp -- electromagnetic interaction models of the transport loop.
//
// The paper takes its e-/e+/gamma physics from G4HepEm (section 2.2) and
// states no formula; the models here are the textbook ones listed with their
// sources beside each function.  Cross sections and stopping powers are
// evaluated on the host when the tables are built; the samplers and screening
// functions are __host__ __device__ and run inside the step kernel.
//
// Every sampler is written for a real type R (double: FP64 form, float:
// mixed form).  Sampled fractions and angles are R; the energies handed back
// are FP64 and split so that parent and secondaries add up to the parent's
// energy in FP64 whatever R is.
#pragma once
#include "ems_core.hpp"

namespace ems {

// Material constants needed at run time by the samplers and the
// null-collision bound.
constexpr int kMaxElements = 4;  // elements of a compound material

struct MatRT {
  double c136;    // 136 Z^{-1/3}: screening variable prefactor (first element)
  double gshift;  // ln Z / 3 + f_c: subtracted from phi / 4 (first element)
  // right-continuous discrete totals at the process thresholds (1/mm):
  // e- at 2 T_cut (Moller) and k_c (brems); e+ at T_cut (Bhabha) and k_c
  double up_em[2], up_ep[2];
  uint32_t n_el;  // elements (1: pair and brems target needs no draw)
  uint32_t pad_;
  double x0;      // radiation length (mm)
  double nel;     // electrons per mm^3
};

// Thomas-Fermi screening functions in the Butcher-Messel parametrisation.
template <class R>
EMS_HD R screen_phi1(R d) {
  return d > R(1) ? R(21.12) - R(4.184) * xlog(d + R(0.952)) : R(20.867) + d * (R(-3.242) + R(0.625) * d);
}
template <class R>
EMS_HD R screen_phi2(R d) {
  return d > R(1) ? R(21.12) - R(4.184) * xlog(d + R(0.952)) : R(20.209) + d * (R(-1.930) - R(0.086) * d);
}
// sup over [d, inf): phi jumps upward when d crosses 1
template <class R>
EMS_HD R screen_phi1_env(R d) {
  const R at1 = R(21.12) - R(4.184) * xlog(R(1.952));
  const R v = screen_phi1(d);
  return (d <= R(1) && at1 > v) ? at1 : v;
}
template <class R>
EMS_HD R screen_phi2_env(R d) {
  const R at1 = R(21.12) - R(4.184) * xlog(R(1.952));
  const R v = screen_phi2(d);
  return (d <= R(1) && at1 > v) ? at1 : v;
}
template <class R>
EMS_HD R screen_g(const MatRT& m, R phi) {
  const R g = R(0.25) * phi - R(m.gshift);
  return g < R(0) ? R(0) : g;
}

// Bethe-Heitler pair brace F(eps) for photon energy E (eps = e+ or e- total
// energy fraction): [eps^2 + (1-eps)^2] G1 + 2/3 eps(1-eps) G2.
template <class R>
EMS_HD R pair_brace(const MatRT& m, R E, R eps) {
  const R w = eps * (R(1) - eps);
  const R d = R(m.c136) * (R(kMe) / E) / w;
  return (R(1) - R(2) * w) * screen_g(m, screen_phi1(d)) + (R(2) / R(3)) * w * screen_g(m, screen_phi2(d));
}
template <class R>
EMS_HD R pair_bound(const MatRT& m, R E) {
  const R dmin = R(4) * R(m.c136) * (R(kMe) / E);
  return screen_g(m, screen_phi1_env(dmin)) + screen_g(m, screen_phi2_env(dmin)) / R(6);
}

// Screened 1/k bremsstrahlung brace for lepton kinetic energy T and photon k:
// max(0, [1 + (1-y)^2] G1 - 2/3 (1-y) G2), y = k / (T + m).
template <class R>
EMS_HD R brem_brace(const MatRT& m, R T, R k) {
  const R et = T + R(kMe);
  const R y = k / et, w = R(1) - y;
  const R d = R(m.c136) * R(kMe) * y / (et * w);
  const R v = (R(1) + w * w) * screen_g(m, screen_phi1(d)) - (R(2) / R(3)) * w * screen_g(m, screen_phi2(d));
  return v > R(0) ? v : R(0);
}
template <class R>
EMS_HD R brem_bound(const MatRT& m, R T, R kc) {
  const R et = T + R(kMe);
  const R y = kc / et;
  const R d = R(m.c136) * R(kMe) * y / (et * (R(1) - y));
  return R(2) * screen_g(m, screen_phi1_env(d));
}

// ---------------------------------------------------------------- samplers
// Outcome of one discrete interaction.  Energies are kinetic (photon: total)
// and FP64; directions are in the arithmetic type.
template <class R>
struct Outcome {
  bool survives;
  double e_parent;
  V3T<R> u_parent;
  int n;           // secondaries 0..2, numbered k = 0, 1 in this order
  int sp[2];
  double e[2];
  V3T<R> u[2];
};

// Klein-Nishina Compton scattering; Butcher-Messel mixture of the 1/eps and
// eps envelopes with the KN rejection factor (three draws per trial).
template <class R>
EMS_HD void compton(double E, V3T<R> u, Draws& r, Outcome<R>& o) {
  const R Er = (R)E;
  const R kap = Er / R(kMe);
  const R e0 = R(1) / (R(1) + R(2) * kap);
  const R a1 = -xlog(e0), a2 = R(0.5) * (R(1) - e0 * e0);
  R eps = R(1), omc = R(0);
  for (int trial = 1;; ++trial) {
    const R ra = r.u<R>(), rb = r.u<R>(), rc = r.u<R>();
    eps = (ra * (a1 + a2) < a1) ? xexp(-a1 * rb) : xsqrt(e0 * e0 + (R(1) - e0 * e0) * rb);
    omc = (R(1) - eps) / (kap * eps);
    const R s2 = omc * (R(2) - omc);
    if (rc <= R(1) - eps * s2 / (R(1) + eps * eps) || trial >= kMaxTrials) break;
  }
  const R cost = R(1) - omc;
  const R s2 = R(1) - cost * cost;
  const V3T<R> ug = about_axis(u, cost, xsqrt(s2 > R(0) ? s2 : R(0)), R(kTwoPi) * r.u<R>());
  const R ep = eps * Er;  // scattered photon energy in the arithmetic type
  o.survives = true;
  o.e_parent = (double)eps * E;
  o.u_parent = ug;
  o.n = 1;
  o.sp[0] = kElectron;
  o.e[0] = E - (double)eps * E;
  o.u[0] = unit(V3T<R>{Er * u.x - ep * ug.x, Er * u.y - ep * ug.y, Er * u.z - ep * ug.z});
}

// Photo-effect: the photon is absorbed, the electron carries E along u.
template <class R>
EMS_HD void photo(double E, V3T<R> u, Outcome<R>& o) {
  o.survives = false;
  o.n = 1;
  o.sp[0] = kElectron;
  o.e[0] = E;
  o.u[0] = u;
}

// Bethe-Heitler pair production: eps uniform on [eps0, 1/2] with rejection
// on F(eps) / bound, then one more draw decides which lepton takes eps.
template <class R>
EMS_HD void pair(const MatRT& m, double E, V3T<R> u, Draws& r, Outcome<R>& o) {
  const R Er = (R)E;
  const R e0 = R(kMe) / Er, fmax = pair_bound(m, Er);
  R eps = R(0.5);
  for (int trial = 1;; ++trial) {
    const R ra = r.u<R>(), rb = r.u<R>();
    eps = e0 + ra * (R(0.5) - e0);
    if (rb * fmax <= pair_brace(m, Er, eps) || trial >= kMaxTrials) break;
  }
  const double epos = (r.u<R>() < R(0.5)) ? (double)eps * E : (1.0 - (double)eps) * E;
  o.survives = false;
  o.n = 2;
  o.sp[0] = kElectron;
  o.e[0] = (E - epos) - kMe;
  o.sp[1] = kPositron;
  o.e[1] = epos - kMe;
  o.u[0] = u;
  o.u[1] = u;
}

// Bremsstrahlung photon above kc: k = kc (T/kc)^a, rejection on the brace.
template <class R>
EMS_HD void brem(const MatRT& m, double T, double kc, V3T<R> u, Draws& r, Outcome<R>& o) {
  const R Tr = (R)T, kr = (R)kc;
  const R bound = brem_bound(m, Tr, kr);
  const R lr = xlog(Tr / kr);
  R k = kr;
  for (int trial = 1;; ++trial) {
    const R ra = r.u<R>(), rb = r.u<R>();
    k = kr * xexp(ra * lr);
    if (rb * bound <= brem_brace(m, Tr, k) || trial >= kMaxTrials) break;
  }
  o.survives = true;
  o.e_parent = T - (double)k;
  o.u_parent = u;
  o.n = 1;
  o.sp[0] = kGamma;
  o.e[0] = (double)k;
  o.u[0] = u;
}

// Two-body kinematics of a delta ray (free electron at rest).
template <class R>
EMS_HD void delta_ray(double T, double td, V3T<R> u, Draws& r, Outcome<R>& o) {
  const R Tr = (R)T, tr = (R)td;
  const R c = xsqrt(tr * (Tr + R(2) * R(kMe)) / (Tr * (tr + R(2) * R(kMe))));
  const R s2 = R(1) - c * c;
  const V3T<R> ud = about_axis(u, c, xsqrt(s2 > R(0) ? s2 : R(0)), R(kTwoPi) * r.u<R>());
  const R p = xsqrt(Tr * (Tr + R(2) * R(kMe))), pd = xsqrt(tr * (tr + R(2) * R(kMe)));
  o.survives = true;
  o.e_parent = T - td;
  o.u_parent = unit(V3T<R>{p * u.x - pd * ud.x, p * u.y - pd * ud.y, p * u.z - pd * ud.z});
  o.n = 1;
  o.sp[0] = kElectron;
  o.e[0] = td;
  o.u[0] = ud;
}

// Moller scattering: eps on [x, 1/2] from the 1/eps^2 envelope.
template <class R>
EMS_HD void moller(double T, double tcut, V3T<R> u, Draws& r, Outcome<R>& o) {
  const R x = (R)(tcut / T), g = (R)(T / kMe + 1.0);
  const R gg = (g - R(1)) / g, c = gg * gg, d = (R(2) * g - R(1)) / (g * g);
  const R bound = R(2) + R(0.25) * c;
  R eps = x;
  for (int trial = 1;; ++trial) {
    const R ra = r.u<R>(), rb = r.u<R>();
    eps = x / (R(1) - ra * (R(1) - R(2) * x));
    const R q = eps / (R(1) - eps);
    const R f = c * eps * eps + R(1) + q * q - d * q;
    if (rb * bound <= f || trial >= kMaxTrials) break;
  }
  delta_ray(T, (double)eps * T, u, r, o);
}

// Bhabha scattering: eps on [x, 1] from the 1/eps^2 envelope, bound 1/beta^2.
template <class R>
EMS_HD void bhabha(double T, double tcut, V3T<R> u, Draws& r, Outcome<R>& o) {
  const R x = (R)(tcut / T), g = (R)(T / kMe + 1.0);
  const R y = R(1) / (g + R(1)), w = R(1) - R(2) * y;
  const R ib2 = R(1) / (R(1) - R(1) / (g * g));
  const R b1 = R(2) - y * y, b2 = w * (R(3) + y * y), b4 = w * w * w, b3 = b4 + w * w;
  R eps = x;
  for (int trial = 1;; ++trial) {
    const R ra = r.u<R>(), rb = r.u<R>();
    eps = x / (R(1) - ra * (R(1) - x));
    const R f = ib2 + eps * (-b1 + eps * (b2 + eps * (-b3 + eps * b4)));
    if (rb * ib2 <= f || trial >= kMaxTrials) break;
  }
  delta_ray(T, (double)eps * T, u, r, o);
}

// Heitler two-photon annihilation in flight: first photon fraction eps from
// the 1/eps envelope on [emin, 1-emin] with rejection g(eps) <= 1.
template <class R>
EMS_HD void annihilate(double T, V3T<R> u, Draws& r, Outcome<R>& o) {
  const R g = (R)(T / kMe + 1.0), s = xsqrt((g - R(1)) * (g + R(1)));
  const R emin = R(1) / (g + R(1) + s), emax = R(1) - emin;
  const R lr = xlog(emax / emin);
  const R gp2 = (g + R(1)) * (g + R(1));
  R eps = emin;
  for (int trial = 1;; ++trial) {
    const R ra = r.u<R>(), rb = r.u<R>();
    eps = emin * xexp(ra * lr);
    if (rb <= R(1) - eps + (R(2) * g * eps - R(1)) / (eps * gp2) || trial >= kMaxTrials) break;
  }
  const double etot = T + 2.0 * kMe;
  R c = (eps * (g + R(1)) - R(1)) / (eps * s);
  c = c > R(1) ? R(1) : (c < R(-1) ? R(-1) : c);
  const V3T<R> u0 = about_axis(u, c, xsqrt(R(1) - c * c), R(kTwoPi) * r.u<R>());
  const double k0 = (double)eps * etot;
  const R k0r = (R)k0, p = (R)sqrt(T * (T + 2.0 * kMe));
  o.survives = false;
  o.n = 2;
  o.sp[0] = kGamma;
  o.sp[1] = kGamma;
  o.e[0] = k0;
  o.e[1] = (1.0 - (double)eps) * etot;
  o.u[0] = u0;
  o.u[1] = unit(V3T<R>{p * u.x - k0r * u0.x, p * u.y - k0r * u0.y, p * u.z - k0r * u0.z});
}

// Annihilation at rest: back-to-back photons of m_e, cos(theta) = 2 U1 - 1,
// phi = 2 pi U2.
template <class R>
EMS_HD void annihilate_at_rest(Draws& r, Outcome<R>& o) {
  const R c = R(2) * r.u_at<R>(1) - R(1);
  const R phi = R(kTwoPi) * r.u_at<R>(2);
  const R s2 = R(1) - c * c;
  const R sn = xsqrt(s2 > R(0) ? s2 : R(0));
  R sp, cp;
  xsincos(phi, &sp, &cp);
  const V3T<R> a{sn * cp, sn * sp, c};
  o.survives = false;
  o.n = 2;
  o.sp[0] = kGamma;
  o.sp[1] = kGamma;
  o.e[0] = kMe;
  o.e[1] = kMe;
  o.u[0] = a;
  o.u[1] = V3T<R>{-a.x, -a.y, -a.z};
}

}  // namespace ems
