// ems_tables.cpp -- host table builder (cross sections, restricted stopping
// powers, ranges, and the running maxima used by the null-collision bound).
//
// Model sources: Klein-Nishina (1929) total cross section; Heitler's K-shell
// Born photo-effect x 5/4; Bethe-Heitler pair and screened 1/k
// bremsstrahlung with Butcher-Messel screening and the Davies-Bethe-Maximon
// Coulomb correction; Moller (1932) and Bhabha (1936) cross sections above the
// delta-ray cut; Berger-Seltzer restricted collision loss (ICRU 37) with an
// asymptotic density correction; Heitler's two-photon annihilation.
#include "ems_tables.hpp"

#include <math.h>

#include <algorithm>
#include <functional>

namespace ems {

namespace {

// n-point Gauss-Legendre abscissae and weights on [-1, 1] (Newton's method on
// the three-term recurrence, symmetric pairs).
struct GaussRule {
  std::vector<double> x, w;
  explicit GaussRule(int n) : x(n), w(n) {
    for (int i = 0; i < (n + 1) / 2; ++i) {
      double z = cos(kPi * (i + 0.75) / (n + 0.5)), dp = 0.0;
      for (int iter = 0; iter < 64; ++iter) {
        double pm = 0.0, p = 1.0;
        for (int k = 1; k <= n; ++k) {
          const double pn = ((2 * k - 1) * z * p - (k - 1) * pm) / k;
          pm = p;
          p = pn;
        }
        dp = n * (z * p - pm) / (z * z - 1.0);
        const double dz = p / dp;
        z -= dz;
        if (fabs(dz) <= 1e-16) {
          pm = 0.0;
          p = 1.0;
          for (int k = 1; k <= n; ++k) {
            const double pn = ((2 * k - 1) * z * p - (k - 1) * pm) / k;
            pm = p;
            p = pn;
          }
          dp = n * (z * p - pm) / (z * z - 1.0);
          break;
        }
      }
      x[i] = -z;
      x[n - 1 - i] = z;
      w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
  }
};

const GaussRule& gl8() {
  static const GaussRule r(8);
  return r;
}
const GaussRule& gl16() {
  static const GaussRule r(16);
  return r;
}

double panels(const std::function<double(double)>& f, double a, double b, int np, const GaussRule& g) {
  const double h = (b - a) / np;
  double s = 0.0;
  for (int p = 0; p < np; ++p) {
    const double c = a + (p + 0.5) * h;
    for (size_t i = 0; i < g.x.size(); ++i) s += 0.5 * h * g.w[i] * f(c + 0.5 * h * g.x[i]);
  }
  return s;
}

// split [a, b] at the given interior points; 16 panels x 8 points per piece
double pieces(const std::function<double(double)>& f, double a, double b, std::vector<double> cuts) {
  std::sort(cuts.begin(), cuts.end());
  double s = 0.0, lo = a;
  for (double c : cuts) {
    if (c <= lo || c >= b) continue;
    s += panels(f, lo, c, 16, gl8());
    lo = c;
  }
  return s + panels(f, lo, b, 16, gl8());
}

// delta at which G_i vanishes on the logarithmic branch of phi
double delta_g0(const MatFull& m) { return exp((21.12 - 4.0 * m.rt.gshift) / 4.184) - 0.952; }

double pref(const MatFull& m) { return 4.0 * kAlpha * kRe * kRe * m.Z * (m.Z + 1.0); }

}  // namespace

namespace {
// one element present with nat atoms per mm^3
MatFull derive_element(double Z, double nat) {
  MatFull m;
  m.Z = Z;
  m.nat = nat;
  m.nel = Z * nat;
  m.I = m.plasma = 0.0;
  const double az2 = (kAlpha * Z) * (kAlpha * Z);
  const double fc = az2 * (1.0 / (1.0 + az2) + 0.20206 + az2 * (-0.0369 + az2 * (0.0083 - 0.002 * az2)));
  m.rt.c136 = 136.0 / cbrt(Z);
  m.rt.gshift = log(Z) / 3.0 + fc;
  m.rt.up_em[0] = m.rt.up_em[1] = m.rt.up_ep[0] = m.rt.up_ep[1] = 0.0;
  m.rt.n_el = 1;
  m.rt.pad_ = 0;
  // Tsai's radiation logarithms (tabulated below Z = 5):
  // 1/X0 = n_at 4 alpha r_e^2 [Z^2 (L_rad - f_c) + Z L'_rad]
  static const double lrad[4] = {5.31, 4.79, 4.74, 4.71}, lprad[4] = {6.144, 5.621, 5.805, 5.924};
  const int iz = (int)floor(Z + 0.5);
  const bool light = iz >= 1 && iz <= 4 && Z == (double)iz;
  const double l = light ? lrad[iz - 1] : log(184.15 / cbrt(Z));
  const double lp = light ? lprad[iz - 1] : log(1194.0 / (cbrt(Z) * cbrt(Z)));
  m.rt.x0 = 1.0 / (nat * 4.0 * kAlpha * kRe * kRe * (Z * Z * (l - fc) + Z * lp));
  m.rt.nel = m.nel;
  return m;
}
}  // namespace

MatSet derive_material(const MaterialIn& in) {
  MatSet s;
  double zpu, apu;  // electrons and grams per mole of formula units
  if (in.n_el == 0) {
    s.n = 1;
    s.el[0] = derive_element(in.Z, in.rho * kNA / in.A * 1e-3);  // per mm^3
    zpu = in.Z;
    apu = in.A;
  } else {
    s.n = in.n_el;
    zpu = apu = 0.0;
    for (uint32_t i = 0; i < s.n; ++i) {
      zpu += in.el_atoms[i] * in.el_Z[i];
      apu += in.el_atoms[i] * in.el_A[i];
    }
    const double units = in.rho * kNA / apu * 1e-3;  // formula units per mm^3
    for (uint32_t i = 0; i < s.n; ++i) s.el[i] = derive_element(in.el_Z[i], in.el_atoms[i] * units);
  }
  s.bulk = s.el[0];
  s.bulk.nel = 0.0;
  for (uint32_t i = 0; i < s.n; ++i) s.bulk.nel += s.el[i].nel;
  s.bulk.I = in.I_eV * 1e-6;
  s.bulk.plasma = 28.816e-6 * sqrt(in.rho * zpu / apu);
  s.bulk.rt.n_el = s.n;
  s.bulk.rt.nel = s.bulk.nel;
  double inv_x0 = 0.0;
  for (uint32_t i = 0; i < s.n; ++i) inv_x0 += 1.0 / s.el[i].rt.x0;
  s.bulk.rt.x0 = 1.0 / inv_x0;
  return s;
}

double kn_sigma(double E) {
  const long double k = (long double)E / kMe;
  const long double q = 1.0L + 2.0L * k, lq = logl(q);
  const long double t1 = (1.0L + k) / (k * k) * (2.0L * (1.0L + k) / q - lq / k);
  const long double t2 = lq / (2.0L * k) - (1.0L + 3.0L * k) / (q * q);
  return (double)(2.0L * (long double)kPi * (long double)kRe * (long double)kRe * (t1 + t2));
}

double photo_sigma(const MatFull& m, double E) {
  const double st = 8.0 * kPi / 3.0 * kRe * kRe;
  const double a2 = kAlpha * kAlpha, z2 = m.Z * m.Z;
  return 5.0 * sqrt(2.0) * a2 * a2 * z2 * z2 * m.Z * st * pow(kMe / E, 3.5);
}

double pair_sigma(const MatFull& m, double E) {
  if (E <= 2.0 * kMe) return 0.0;
  const double e0 = kMe / E;
  std::vector<double> cuts;
  for (double d : {1.0, delta_g0(m)}) {
    const double q = 4.0 * m.rt.c136 * e0 / d;  // eps(1-eps) = q/4 where delta = d
    if (q < 1.0) cuts.push_back(log(0.5 * (1.0 - sqrt(1.0 - q))));
  }
  auto f = [&](double w) {
    const double eps = exp(w);
    return pair_brace(m.rt, E, eps) * eps;
  };
  return 2.0 * pref(m) * pieces(f, log(e0), log(0.5), cuts);
}

double brem_sigma(const MatFull& m, double T, double kc) {
  if (T <= kc) return 0.0;
  const double et = T + kMe;
  // v = ln(k / (E_t - k)); d ln k = (1 - y) dv; delta = d at v = ln(d E_t/(c136 m))
  std::vector<double> cuts;
  for (double d : {1.0, delta_g0(m)}) cuts.push_back(log(d * et / (m.rt.c136 * kMe)));
  auto f = [&](double v) {
    const double y = 1.0 / (1.0 + exp(-v));
    return brem_brace(m.rt, T, y * et) * (1.0 - y);
  };
  return pref(m) * pieces(f, log(kc / (et - kc)), log(T / (et - T)), cuts);
}

double brem_loss(const MatFull& m, double T, double kc) {
  const double et = T + kMe, kmax = std::min(kc, T);
  std::vector<double> cuts;
  for (double d : {1.0, delta_g0(m)}) {
    const double r = d * et / (m.rt.c136 * kMe);
    cuts.push_back(et * r / (1.0 + r));
  }
  auto f = [&](double k) { return brem_brace(m.rt, T, k); };
  return m.nat * pref(m) * pieces(f, 0.0, kmax, cuts);
}

double moller_sigma(double T, double tcut) {
  if (T <= 2.0 * tcut) return 0.0;
  const double x = tcut / T, g = T / kMe + 1.0, b2 = 1.0 - 1.0 / (g * g);
  const double gg = (g - 1.0) / g;
  const double br = gg * gg * (0.5 - x) + 1.0 / x - 1.0 / (1.0 - x) - (2.0 * g - 1.0) / (g * g) * log((1.0 - x) / x);
  return 2.0 * kPi * kRe * kRe * kMe / (b2 * T) * br;
}

double bhabha_sigma(double T, double tcut) {
  if (T <= tcut) return 0.0;
  const double x = tcut / T, g = T / kMe + 1.0, b2 = 1.0 - 1.0 / (g * g);
  const double y = 1.0 / (g + 1.0), w = 1.0 - 2.0 * y;
  const double b1 = 2.0 - y * y, bb2 = w * (3.0 + y * y), b4 = w * w * w, b3 = b4 + w * w;
  const double br = (1.0 / x - 1.0) / b2 + b1 * log(x) + bb2 * (1.0 - x) - 0.5 * b3 * (1.0 - x * x) +
                    b4 * (1.0 - x * x * x) / 3.0;
  return 2.0 * kPi * kRe * kRe * kMe / T * br;
}

double ion_loss(const MatFull& m, double T, double tcut, bool positron) {
  const double tau = T / kMe, g = tau + 1.0, g2 = g * g, b2 = 1.0 - 1.0 / g2;
  const double dmax = positron ? tau : 0.5 * tau;
  const double d = std::min(tcut / kMe, dmax);
  double f;
  if (positron) {
    const double y = 1.0 / (g + 1.0);
    const double bracket = tau + 2.0 * d - 1.5 * d * d * y - (d - d * d * d / 3.0) * y * y -
                           (0.5 * d * d - tau * d * d * d / 3.0 + 0.25 * d * d * d * d) * y * y * y;
    f = log(tau * d) - b2 / tau * bracket;
  } else {
    f = -1.0 - b2 + log((tau - d) * d) + tau / (tau - d) + (0.5 * d * d + (2.0 * tau + 1.0) * log(1.0 - d / tau)) / g2;
  }
  const double im = m.I / kMe;
  double dens = 2.0 * log(m.plasma / m.I) + log(b2 * g2) - 1.0;  // 2 ln(beta gamma) = ln(b2 g2)
  if (dens < 0.0) dens = 0.0;
  const double s = 2.0 * kPi * kRe * kRe * kMe * m.nel / b2 * (log(2.0 * (tau + 2.0) / (im * im)) + f - dens);
  return s > 0.0 ? s : 0.0;
}

double heitler_sigma(double T) {
  const double g = T / kMe + 1.0, gm = (g - 1.0) * (g + 1.0), s = sqrt(gm);
  return kPi * kRe * kRe / (g + 1.0) * ((g * g + 4.0 * g + 1.0) / gm * log(g + s) - (g + 3.0) / s);
}

TableSet build_tables(const TableParams& p, const std::vector<MaterialIn>& mats) {
  TableSet ts;
  ts.n_mat = (uint32_t)mats.size();
  ts.nodes = p.n_bins + 1;
  ts.lnemin = log(p.emin);
  ts.dlog = (log(p.emax) - log(p.emin)) / p.n_bins;
  ts.v.assign((size_t)ts.n_mat * kNumTables * ts.nodes, 0.0);
  ts.el.assign((size_t)ts.n_mat * kMaxElements * 2 * ts.nodes, 0.0);
  ts.elc.assign((size_t)ts.n_mat * kMaxElements * 2, 0.0);
  const uint32_t N = ts.nodes;
  auto T = [&](uint32_t m, int t) { return &ts.v[((size_t)m * kNumTables + t) * N]; };
  const bool on_c = p.process_mask & kPCompton, on_p = p.process_mask & kPPhot,
             on_v = p.process_mask & kPConv, on_i = p.process_mask & kPEIoni,
             on_b = p.process_mask & kPEBrem, on_a = p.process_mask & kPAnnih;
  for (uint32_t mi = 0; mi < ts.n_mat; ++mi) {
    const MatSet ms = derive_material(mats[mi]);
    const MatFull& m = ms.bulk;
    ts.rt.push_back(m.rt);
    for (uint32_t i = 0; i < ms.n; ++i) {
      ts.elc[((size_t)mi * kMaxElements + i) * 2] = ms.el[i].rt.c136;
      ts.elc[((size_t)mi * kMaxElements + i) * 2 + 1] = ms.el[i].rt.gshift;
    }
    for (uint32_t j = 0; j < N; ++j) {
      const double E = exp(ts.lnemin + j * ts.dlog);
      // per-atom processes: sums over the elements (Bragg additivity)
      double sp = 0.0, sv = 0.0, sb = 0.0, rl = 0.0;
      for (uint32_t i = 0; i < ms.n; ++i) {
        const MatFull& el = ms.el[i];
        const double v = on_v ? el.nat * pair_sigma(el, E) : 0.0;
        const double b = on_b ? el.nat * brem_sigma(el, E, p.gamma_cut) : 0.0;
        ts.el[(((size_t)mi * kMaxElements + i) * 2) * N + j] = v;
        ts.el[(((size_t)mi * kMaxElements + i) * 2 + 1) * N + j] = b;
        sp += on_p ? el.nat * photo_sigma(el, E) : 0.0;
        sv += v;
        sb += b;
        rl += brem_loss(el, E, p.gamma_cut);
      }
      T(mi, tCompt)[j] = on_c ? m.nel * kn_sigma(E) : 0.0;
      T(mi, tPhot)[j] = sp;
      T(mi, tConv)[j] = sv;
      T(mi, tBrem)[j] = sb;
      T(mi, tMoller)[j] = on_i ? m.nel * moller_sigma(E, p.electron_cut) : 0.0;
      T(mi, tBhabha)[j] = on_i ? m.nel * bhabha_sigma(E, p.electron_cut) : 0.0;
      T(mi, tAnnih)[j] = on_a ? m.nel * heitler_sigma(E) : 0.0;
      T(mi, tSem)[j] = ion_loss(m, E, p.electron_cut, false) + rl;
      T(mi, tSep)[j] = ion_loss(m, E, p.electron_cut, true) + rl;
    }
    // range: R_0 = E_0 / (2 S_0), then the integral of dE / S_interp per bin,
    // 16-point Gauss-Legendre in t = (ln E - ln E_{j-1}) / D
    for (int sp : {tSem, tSep}) {
      const double* S = T(mi, sp);
      double* R = T(mi, sp + 1);
      R[0] = p.emin / (2.0 * S[0]);
      for (uint32_t j = 1; j < N; ++j) {
        const double e0 = exp(ts.lnemin + (j - 1) * ts.dlog);
        auto f = [&](double t) { return e0 * exp(t * ts.dlog) / (S[j - 1] + t * (S[j] - S[j - 1])); };
        R[j] = R[j - 1] + ts.dlog * panels(f, 0.0, 1.0, 1, gl16());
      }
    }
    // running maxima of the e-/e+ discrete totals over nodes and thresholds
    struct Proc {
      int t;
      double th;
    };
    const Proc pe[2] = {{tMoller, 2.0 * p.electron_cut}, {tBrem, p.gamma_cut}};
    const Proc pp[3] = {{tBhabha, p.electron_cut}, {tBrem, p.gamma_cut}, {tAnnih, 0.0}};
    auto interp_at = [&](int t, double E) {
      const double x = (log(E) - ts.lnemin) / ts.dlog;
      int j = (int)floor(x);
      j = std::max(0, std::min(j, (int)N - 2));
      const double u = std::min(1.0, std::max(0.0, x - j));
      const double* f = T(mi, t);
      return f[j] + u * (f[j + 1] - f[j]);
    };
    auto upper_total = [&](const Proc* pr, int np, double E) {
      double s = 0.0;
      for (int i = 0; i < np; ++i)
        if (E >= pr[i].th) s += interp_at(pr[i].t, E);
      return s;
    };
    ts.rt[mi].up_em[0] = upper_total(pe, 2, pe[0].th);
    ts.rt[mi].up_em[1] = upper_total(pe, 2, pe[1].th);
    ts.rt[mi].up_ep[0] = upper_total(pp, 3, pp[0].th);
    ts.rt[mi].up_ep[1] = upper_total(pp, 3, pp[1].th);
    for (int which = 0; which < 2; ++which) {
      const Proc* pr = which ? pp : pe;
      const int np = which ? 3 : 2;
      double* PM = T(mi, which ? tPMep : tPMem);
      double run = 0.0;
      for (uint32_t j = 0; j < N; ++j) {
        double s = 0.0;
        for (int i = 0; i < np; ++i) s += T(mi, pr[i].t)[j];
        run = std::max(run, s);
        const double Ej = exp(ts.lnemin + j * ts.dlog);
        const double Eprev = j ? exp(ts.lnemin + (j - 1) * ts.dlog) : 0.0;
        for (int i = 0; i < np; ++i)
          if (pr[i].th > Eprev && pr[i].th <= Ej) run = std::max(run, upper_total(pr, np, pr[i].th));
        PM[j] = run;
      }
    }
  }
  return ts;
}

}  // namespace ems
