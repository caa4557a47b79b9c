// ems_models.hpp -- electromagnetic interaction models of the transport loop.
//
// The paper takes its e-/e+/gamma physics from G4HepEm (section 2.2) and
// states no formula; the models here are the textbook ones listed with their
// sources beside each function.  Cross sections and stopping powers are
// evaluated on the host when the tables are built; the samplers and screening
// functions are __host__ __device__ and run inside the step kernel.
#pragma once
#include "ems_core.hpp"

namespace ems {

// Material constants needed at run time by the samplers and the
// null-collision bound.
struct MatRT {
  double c136;    // 136 Z^{-1/3}: screening variable prefactor
  double gshift;  // ln Z / 3 + f_c: subtracted from phi / 4
  // right-continuous discrete totals at the process thresholds (1/mm):
  // e- at 2 T_cut (Moller) and k_c (brems); e+ at T_cut (Bhabha) and k_c
  double up_em[2], up_ep[2];
};

// Thomas-Fermi screening functions in the Butcher-Messel parametrisation.
EMS_HD double screen_phi1(double d) {
  return d > 1.0 ? 21.12 - 4.184 * log(d + 0.952) : 20.867 + d * (-3.242 + 0.625 * d);
}
EMS_HD double screen_phi2(double d) {
  return d > 1.0 ? 21.12 - 4.184 * log(d + 0.952) : 20.209 + d * (-1.930 - 0.086 * d);
}
// sup over [d, inf): phi jumps upward when d crosses 1
EMS_HD double screen_phi1_env(double d) {
  const double at1 = 21.12 - 4.184 * log(1.952);
  const double v = screen_phi1(d);
  return (d <= 1.0 && at1 > v) ? at1 : v;
}
EMS_HD double screen_phi2_env(double d) {
  const double at1 = 21.12 - 4.184 * log(1.952);
  const double v = screen_phi2(d);
  return (d <= 1.0 && at1 > v) ? at1 : v;
}
EMS_HD double screen_g(const MatRT& m, double phi) {
  const double g = 0.25 * phi - m.gshift;
  return g < 0.0 ? 0.0 : g;
}

// Bethe-Heitler pair brace F(eps) for photon energy E (eps = e+ or e- total
// energy fraction): [eps^2 + (1-eps)^2] G1 + 2/3 eps(1-eps) G2.
EMS_HD double pair_brace(const MatRT& m, double E, double eps) {
  const double w = eps * (1.0 - eps);
  const double d = m.c136 * (kMe / E) / w;
  return (1.0 - 2.0 * w) * screen_g(m, screen_phi1(d)) + (2.0 / 3.0) * w * screen_g(m, screen_phi2(d));
}
EMS_HD double pair_bound(const MatRT& m, double E) {
  const double dmin = 4.0 * m.c136 * (kMe / E);
  return screen_g(m, screen_phi1_env(dmin)) + screen_g(m, screen_phi2_env(dmin)) / 6.0;
}

// Screened 1/k bremsstrahlung brace for lepton kinetic energy T and photon k:
// max(0, [1 + (1-y)^2] G1 - 2/3 (1-y) G2), y = k / (T + m).
EMS_HD double brem_brace(const MatRT& m, double T, double k) {
  const double et = T + kMe;
  const double y = k / et, w = 1.0 - y;
  const double d = m.c136 * kMe * y / (et * w);
  const double v = (1.0 + w * w) * screen_g(m, screen_phi1(d)) - (2.0 / 3.0) * w * screen_g(m, screen_phi2(d));
  return v > 0.0 ? v : 0.0;
}
EMS_HD double brem_bound(const MatRT& m, double T, double kc) {
  const double et = T + kMe;
  const double y = kc / et;
  const double d = m.c136 * kMe * y / (et * (1.0 - y));
  return 2.0 * screen_g(m, screen_phi1_env(d));
}

// ---------------------------------------------------------------- samplers
// Outcome of one discrete interaction.  Energies are kinetic (photon: total).
struct Outcome {
  bool survives;
  double e_parent;
  V3 u_parent;
  int n;           // secondaries 0..2, numbered k = 0, 1 in this order
  int sp[2];
  double e[2];
  V3 u[2];
};

// Klein-Nishina Compton scattering; Butcher-Messel mixture of the 1/eps and
// eps envelopes with the KN rejection factor (three draws per trial).
EMS_HD void compton(double E, V3 u, Draws& r, Outcome& o) {
  const double kap = E / kMe;
  const double e0 = 1.0 / (1.0 + 2.0 * kap);
  const double a1 = -log(e0), a2 = 0.5 * (1.0 - e0 * e0);
  double eps = 1.0, omc = 0.0;
  for (int trial = 1;; ++trial) {
    const double ra = r.next(), rb = r.next(), rc = r.next();
    eps = (ra * (a1 + a2) < a1) ? exp(-a1 * rb) : sqrt(e0 * e0 + (1.0 - e0 * e0) * rb);
    omc = (1.0 - eps) / (kap * eps);
    const double s2 = omc * (2.0 - omc);
    if (rc <= 1.0 - eps * s2 / (1.0 + eps * eps) || trial >= kMaxTrials) break;
  }
  const double cost = 1.0 - omc;
  const double s2 = 1.0 - cost * cost;
  const V3 ug = about_axis(u, cost, sqrt(s2 > 0.0 ? s2 : 0.0), kTwoPi * r.next());
  o.survives = true;
  o.e_parent = eps * E;
  o.u_parent = ug;
  o.n = 1;
  o.sp[0] = kElectron;
  o.e[0] = E - eps * E;
  o.u[0] = unit(V3{E * u.x - eps * E * ug.x, E * u.y - eps * E * ug.y, E * u.z - eps * E * ug.z});
}

// Photo-effect: the photon is absorbed, the electron carries E along u.
EMS_HD void photo(double E, V3 u, Outcome& o) {
  o.survives = false;
  o.n = 1;
  o.sp[0] = kElectron;
  o.e[0] = E;
  o.u[0] = u;
}

// Bethe-Heitler pair production: eps uniform on [eps0, 1/2] with rejection
// on F(eps) / bound, then one more draw decides which lepton takes eps.
EMS_HD void pair(const MatRT& m, double E, V3 u, Draws& r, Outcome& o) {
  const double e0 = kMe / E, fmax = pair_bound(m, E);
  double eps = 0.5;
  for (int trial = 1;; ++trial) {
    const double ra = r.next(), rb = r.next();
    eps = e0 + ra * (0.5 - e0);
    if (rb * fmax <= pair_brace(m, E, eps) || trial >= kMaxTrials) break;
  }
  const double epos = (r.next() < 0.5) ? eps * E : (1.0 - eps) * E;
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
EMS_HD void brem(const MatRT& m, double T, double kc, V3 u, Draws& r, Outcome& o) {
  const double bound = brem_bound(m, T, kc);
  const double lr = log(T / kc);
  double k = kc;
  for (int trial = 1;; ++trial) {
    const double ra = r.next(), rb = r.next();
    k = kc * exp(ra * lr);
    if (rb * bound <= brem_brace(m, T, k) || trial >= kMaxTrials) break;
  }
  o.survives = true;
  o.e_parent = T - k;
  o.u_parent = u;
  o.n = 1;
  o.sp[0] = kGamma;
  o.e[0] = k;
  o.u[0] = u;
}

// Two-body kinematics of a delta ray (free electron at rest).
EMS_HD void delta_ray(double T, double td, V3 u, Draws& r, Outcome& o) {
  const double c = sqrt(td * (T + 2.0 * kMe) / (T * (td + 2.0 * kMe)));
  const double s2 = 1.0 - c * c;
  const V3 ud = about_axis(u, c, sqrt(s2 > 0.0 ? s2 : 0.0), kTwoPi * r.next());
  const double p = sqrt(T * (T + 2.0 * kMe)), pd = sqrt(td * (td + 2.0 * kMe));
  o.survives = true;
  o.e_parent = T - td;
  o.u_parent = unit(V3{p * u.x - pd * ud.x, p * u.y - pd * ud.y, p * u.z - pd * ud.z});
  o.n = 1;
  o.sp[0] = kElectron;
  o.e[0] = td;
  o.u[0] = ud;
}

// Moller scattering: eps on [x, 1/2] from the 1/eps^2 envelope.
EMS_HD void moller(double T, double tcut, V3 u, Draws& r, Outcome& o) {
  const double x = tcut / T, g = T / kMe + 1.0;
  const double gg = (g - 1.0) / g, c = gg * gg, d = (2.0 * g - 1.0) / (g * g);
  const double bound = 2.0 + 0.25 * c;
  double eps = x;
  for (int trial = 1;; ++trial) {
    const double ra = r.next(), rb = r.next();
    eps = x / (1.0 - ra * (1.0 - 2.0 * x));
    const double q = eps / (1.0 - eps);
    const double f = c * eps * eps + 1.0 + q * q - d * q;
    if (rb * bound <= f || trial >= kMaxTrials) break;
  }
  delta_ray(T, eps * T, u, r, o);
}

// Bhabha scattering: eps on [x, 1] from the 1/eps^2 envelope, bound 1/beta^2.
EMS_HD void bhabha(double T, double tcut, V3 u, Draws& r, Outcome& o) {
  const double x = tcut / T, g = T / kMe + 1.0;
  const double y = 1.0 / (g + 1.0), w = 1.0 - 2.0 * y;
  const double ib2 = 1.0 / (1.0 - 1.0 / (g * g));
  const double b1 = 2.0 - y * y, b2 = w * (3.0 + y * y), b4 = w * w * w, b3 = b4 + w * w;
  double eps = x;
  for (int trial = 1;; ++trial) {
    const double ra = r.next(), rb = r.next();
    eps = x / (1.0 - ra * (1.0 - x));
    const double f = ib2 + eps * (-b1 + eps * (b2 + eps * (-b3 + eps * b4)));
    if (rb * ib2 <= f || trial >= kMaxTrials) break;
  }
  delta_ray(T, eps * T, u, r, o);
}

// Heitler two-photon annihilation in flight: first photon fraction eps from
// the 1/eps envelope on [emin, 1-emin] with rejection g(eps) <= 1.
EMS_HD void annihilate(double T, V3 u, Draws& r, Outcome& o) {
  const double g = T / kMe + 1.0, s = sqrt((g - 1.0) * (g + 1.0));
  const double emin = 1.0 / (g + 1.0 + s), emax = 1.0 - emin;
  const double lr = log(emax / emin);
  const double gp2 = (g + 1.0) * (g + 1.0);
  double eps = emin;
  for (int trial = 1;; ++trial) {
    const double ra = r.next(), rb = r.next();
    eps = emin * exp(ra * lr);
    if (rb <= 1.0 - eps + (2.0 * g * eps - 1.0) / (eps * gp2) || trial >= kMaxTrials) break;
  }
  const double etot = T + 2.0 * kMe;
  double c = (eps * (g + 1.0) - 1.0) / (eps * s);
  c = c > 1.0 ? 1.0 : (c < -1.0 ? -1.0 : c);
  const V3 u0 = about_axis(u, c, sqrt(1.0 - c * c), kTwoPi * r.next());
  const double k0 = eps * etot, p = sqrt(T * (T + 2.0 * kMe));
  o.survives = false;
  o.n = 2;
  o.sp[0] = kGamma;
  o.sp[1] = kGamma;
  o.e[0] = k0;
  o.e[1] = (1.0 - eps) * etot;
  o.u[0] = u0;
  o.u[1] = unit(V3{p * u.x - k0 * u0.x, p * u.y - k0 * u0.y, p * u.z - k0 * u0.z});
}

// Annihilation at rest: back-to-back photons of m_e, cos(theta) = 2 U1 - 1,
// phi = 2 pi U2.
EMS_HD void annihilate_at_rest(Draws& r, Outcome& o) {
  const double c = 2.0 * r.at(1) - 1.0;
  const double phi = kTwoPi * r.at(2);
  const double s2 = 1.0 - c * c;
  const double s = sqrt(s2 > 0.0 ? s2 : 0.0);
  const V3 a{s * cos(phi), s * sin(phi), c};
  o.survives = false;
  o.n = 2;
  o.sp[0] = kGamma;
  o.sp[1] = kGamma;
  o.e[0] = kMe;
  o.e[1] = kMe;
  o.u[0] = a;
  o.u[1] = V3{-a.x, -a.y, -a.z};
}

}  // namespace ems
