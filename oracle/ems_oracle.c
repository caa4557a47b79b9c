/*
 * ems_oracle.c -- plain FP64 CPU oracle (test infrastructure only; see
 * ems_oracle.h).  Written to be read against the paper and the physics
 * readings, not to be fast: no blocking, no fusion, no reordering.
 *
 * Paper passages followed:
 *  - "Stepping workflow" (section 3): tracks are stepped one at a time by a
 *    CPU thread; secondaries go on a stack; the species is implicit.
 *  - "Physics integration and validation" (section 2.2): physics is run-time
 *    functions taking scalar arguments plus an abstracted RNG.
 *  - "Magnetic field" (section 2.3): charged tracks propagate in a constant
 *    field; here the helix is exact and tracks killed by the watchdog are
 *    accounted for (the paper accounts killed tracks' energy the same way).
 *  - "Geant4 integration" (section 4): per-event hit arrays.
 * The physics formulas are textbook readings (the paper delegates physics to
 * G4HepEm); each function names its source.
 */
#include "ems_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Constants (CODATA 2018; k_B converts p[MeV/c] = k_B * B[T] * R[mm])  */
/* ------------------------------------------------------------------ */
static const double ME = 0.51099895;            /* electron mass, MeV  */
static const double RE = 2.8179403262e-12;      /* classical radius, mm */
static const double ALPHA = 1.0 / 137.035999084;
static const double NAVO = 6.02214076e23;
static const double KB = 0.299792458;
static const double PI = 3.14159265358979323846;

/* sampler trial cap: after this many rejected trials the last candidate
 * is accepted (keeps every loop finite; never reached with valid bounds) */
#define OR_MAX_TRIALS 1000
#define OR_SAFETY_EPS 1e-6  /* mm: helix track this close to a wall escapes */

/* table ids in the export layout */
enum {
  T_COMPT = 0, T_PHOT = 1, T_CONV = 2,
  T_S_EM = 3, T_R_EM = 4, T_MOLLER = 5, T_BREM = 6,
  T_S_EP = 7, T_R_EP = 8, T_BHABHA = 9, T_ANNIH = 10
};

typedef struct {
  double Z, A, rho, I_eV;
  double n_at, n_el;     /* atoms / electrons per mm^3 */
  double I;              /* mean excitation energy, MeV */
  double plasma;         /* plasma energy, MeV          */
  double zm13, lnz, fc;  /* Z^{-1/3}, ln Z, Coulomb correction */
  double x0;             /* radiation length, mm (of the element alone at
                            its atom density, or of the whole material) */
} or_mat;

enum { OR_MAX_EL = 4 };

struct or_ctx {
  or_setup s;
  uint32_t n_slabs, n_mat, nb;       /* nb = n_bins: nodes 0..nb */
  uint32_t n_cols;                   /* deposit columns: slabs, or boxes + world */
  uint32_t nbox;                     /* box geometry: boxes (0: slab stack) */
  double *blo, *bhi;                 /* [nbox][3] */
  uint32_t* bmat;
  double wlo[3], whi[3];
  uint32_t wmat;
  double* z;
  uint32_t* slab_mat;
  or_mat* mat;                       /* material as a whole: electron density, I, plasma energy */
  or_mat* el;                        /* [n_mat][OR_MAX_EL]: elements with their own atom densities */
  uint32_t* n_el;                    /* elements per material */
  double* eltab;                     /* [n_mat][OR_MAX_EL][2][nb+1]: per-element pair, brems Sigma */
  double lnemin, dlog, ecut, tcut, kcut;
  double* tab;                       /* [n_mat][OR_N_TABLES][nb+1] */
};

/* ------------------------------------------------------------------ */
/* Gauss-Legendre rules by Newton iteration on P_n (standard method)   */
/* ------------------------------------------------------------------ */
static double legendre(int n, double r, double* pn1) {
  double p0 = 1.0, p1 = r;
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2.0 * k - 1.0) * r * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *pn1 = p0;   /* P_{n-1}(r) */
  return p1;   /* P_n(r)     */
}
static void gauss_legendre(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double r = cos(PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double q, p = legendre(n, r, &q);
      double dr = p / (n * (r * p - q) / (r * r - 1.0));
      r -= dr;
      if (fabs(dr) < 1e-16) break;
    }
    double q, p = legendre(n, r, &q);
    double dp = n * (r * p - q) / (r * r - 1.0);
    x[i] = r;
    w[i] = 2.0 / ((1.0 - r * r) * dp * dp);
  }
}

/* composite rule: np panels of an ng-point Gauss-Legendre rule on [a,b] */
typedef double (*or_fn)(const void* par, double x);
static double integrate(or_fn f, const void* par, double a, double b, int np,
                        int ng) {
  double gx[16], gw[16];
  gauss_legendre(ng, gx, gw);
  double h = (b - a) / np, sum = 0.0;
  for (int p = 0; p < np; ++p) {
    double lo = a + p * h, mid = lo + 0.5 * h;
    for (int i = 0; i < ng; ++i) sum += gw[i] * 0.5 * h * f(par, mid + 0.5 * h * gx[i]);
  }
  return sum;
}

/* ------------------------------------------------------------------ */
/* Materials                                                           */
/* ------------------------------------------------------------------ */
/* Tsai's radiation logarithms L_rad and L'_rad (PDG RPP, radiation
 * length); below Z = 5 his tabulated values */
static void rad_logs(double Z, double* l, double* lp) {
  static const double tl[4] = {5.31, 4.79, 4.74, 4.71};
  static const double tlp[4] = {6.144, 5.621, 5.805, 5.924};
  int z = (int)floor(Z + 0.5);
  if (z >= 1 && z <= 4 && Z == (double)z) {
    *l = tl[z - 1];
    *lp = tlp[z - 1];
  } else {
    *l = log(184.15 * pow(Z, -1.0 / 3.0));
    *lp = log(1194.0 * pow(Z, -2.0 / 3.0));
  }
}

/* one element of atomic number Z and molar mass A present with n_at atoms
 * per mm^3 */
static void derive_element(double Z, double A, double n_at, or_mat* m) {
  m->Z = Z;
  m->A = A;
  m->n_at = n_at;
  m->n_el = Z * n_at;
  m->zm13 = pow(Z, -1.0 / 3.0);
  m->lnz = log(Z);
  /* Davies-Bethe-Maximon Coulomb correction (PDG RPP form) */
  double a2 = (ALPHA * Z) * (ALPHA * Z);
  m->fc = a2 * (1.0 / (1.0 + a2) + 0.20206 - 0.0369 * a2 + 0.0083 * a2 * a2 -
                0.002 * a2 * a2 * a2);
  /* 1/X0 = n_at 4 alpha r_e^2 [Z^2 (L_rad - f_c) + Z L'_rad] */
  double l, lp;
  rad_logs(Z, &l, &lp);
  m->x0 = 1.0 / (n_at * 4.0 * ALPHA * RE * RE * (Z * Z * (l - m->fc) + Z * lp));
}

/* the material as a whole (m) and its elements (el[0..*n)); a single
 * element is its own only element */
static void derive_material_el(const or_material* in, or_mat* m, or_mat* el, uint32_t* n) {
  double zsum = 0.0, msum = 0.0;  /* electrons and grams per formula unit (per mol) */
  if (in->n_elements == 0) {
    *n = 1;
    derive_element(in->Z, in->A_g_mol, in->density_g_cm3 * NAVO / in->A_g_mol * 1e-3, &el[0]);  /* cm^-3 -> mm^-3 */
    zsum = in->Z;
    msum = in->A_g_mol;
  } else {
    *n = in->n_elements;
    for (uint32_t i = 0; i < *n; ++i) msum += in->el_atoms[i] * in->el_A[i];
    const double n_formula = in->density_g_cm3 * NAVO / msum * 1e-3;
    for (uint32_t i = 0; i < *n; ++i) {
      derive_element(in->el_Z[i], in->el_A[i], in->el_atoms[i] * n_formula, &el[i]);
      zsum += in->el_atoms[i] * in->el_Z[i];
    }
  }
  *m = el[0];
  m->rho = in->density_g_cm3;
  m->I_eV = in->I_eV;
  m->n_el = 0.0;
  for (uint32_t i = 0; i < *n; ++i) m->n_el += el[i].n_el;
  m->I = in->I_eV * 1e-6;
  /* radiation lengths combine as 1/X0 = sum_i 1/X0_i */
  double inv_x0 = 0.0;
  for (uint32_t i = 0; i < *n; ++i) inv_x0 += 1.0 / el[i].x0;
  m->x0 = 1.0 / inv_x0;
  /* plasma energy 28.816 eV * sqrt(rho <Z/A>)  (PDG RPP, passage of
   * particles through matter) */
  m->plasma = 28.816e-6 * sqrt(in->density_g_cm3 * zsum / msum);
}
static void derive_material(const or_material* in, or_mat* m) {
  or_mat el[OR_MAX_EL];
  uint32_t n;
  derive_material_el(in, m, el, &n);
}

/* ------------------------------------------------------------------ */
/* Compton: Klein-Nishina total cross section per electron             */
/* ------------------------------------------------------------------ */
static double xs_compton(double E) {
  /* long double: at k ~ 2e-3 the bracket cancels about 5 digits */
  long double k = (long double)E / ME;
  long double a = 1.0L + 2.0L * k;
  long double L = logl(a);
  long double br = ((1.0L + k) / (k * k)) * (2.0L * (1.0L + k) / a - L / k) +
                   L / (2.0L * k) - (1.0L + 3.0L * k) / (a * a);
  return (double)(2.0L * (long double)PI * (long double)RE * (long double)RE * br);
}

/* Butcher-Messel form of d sigma / d eps, eps = E'/E */
static double dsde_compton(double E, double eps) {
  double k = E / ME;
  double t = (1.0 - eps) / (k * eps);
  double sin2 = t * (2.0 - t);
  return PI * RE * RE / k * (1.0 / eps + eps) * (1.0 - eps * sin2 / (1.0 + eps * eps));
}

/* ------------------------------------------------------------------ */
/* Photo-effect: Heitler K-shell Born formula x 5/4 for outer shells    */
/* ------------------------------------------------------------------ */
static double xs_photo(const or_mat* m, double E) {
  double sig_t = 8.0 * PI / 3.0 * RE * RE;
  double a4 = ALPHA * ALPHA * ALPHA * ALPHA;
  double z5 = m->Z * m->Z * m->Z * m->Z * m->Z;
  return 1.25 * 4.0 * sqrt(2.0) * a4 * z5 * sig_t * pow(ME / E, 3.5);
}

/* ------------------------------------------------------------------ */
/* Thomas-Fermi screening functions (Butcher-Messel parametrisation)   */
/* ------------------------------------------------------------------ */
static double phi1(double d) {
  if (d <= 1.0) return 20.867 - 3.242 * d + 0.625 * d * d;
  return 21.12 - 4.184 * log(d + 0.952);
}
static double phi2(double d) {
  if (d <= 1.0) return 20.209 - 1.930 * d - 0.086 * d * d;
  return 21.12 - 4.184 * log(d + 0.952);
}
/* non-increasing envelopes: sup of phi_i over [d, inf) (phi jumps up at 1) */
static double phi1_env(double d) {
  if (d <= 1.0) {
    double p = phi1(d), q = 21.12 - 4.184 * log(1.952);
    return p > q ? p : q;
  }
  return phi1(d);
}
static double phi2_env(double d) {
  if (d <= 1.0) {
    double p = phi2(d), q = 21.12 - 4.184 * log(1.952);
    return p > q ? p : q;
  }
  return phi2(d);
}
static double gfun(const or_mat* m, double phi) {
  double g = 0.25 * phi - m->lnz / 3.0 - m->fc;
  return g > 0.0 ? g : 0.0;
}

/* ------------------------------------------------------------------ */
/* Pair production (Bethe-Heitler, screened, Coulomb corrected)        */
/* ------------------------------------------------------------------ */
/* F(eps): the brace of d sigma / d eps, eps = total-energy fraction */
static double pair_F(const or_mat* m, double E, double eps) {
  double eps0 = ME / E;
  double d = 136.0 * m->zm13 * eps0 / (eps * (1.0 - eps));
  double g1 = gfun(m, phi1(d)), g2 = gfun(m, phi2(d));
  return (eps * eps + (1.0 - eps) * (1.0 - eps)) * g1 +
         (2.0 / 3.0) * eps * (1.0 - eps) * g2;
}
static double pair_pref(const or_mat* m) {
  return 4.0 * ALPHA * RE * RE * m->Z * (m->Z + 1.0);
}
/* sampler bound: eps^2+(1-eps)^2 <= 1, 2/3 eps(1-eps) <= 1/6, and the
 * screening functions are bounded by their envelopes at the smallest
 * delta, reached at eps = 1/2 */
static double pair_Fmax(const or_mat* m, double E) {
  double dmin = 136.0 * m->zm13 * 4.0 * ME / E;
  return gfun(m, phi1_env(dmin)) + gfun(m, phi2_env(dmin)) / 6.0;
}
typedef struct { const or_mat* m; double E; } pair_par;
/* integrand in w = ln eps: F(eps) * eps */
static double pair_integrand(const void* p, double w) {
  const pair_par* q = (const pair_par*)p;
  double eps = exp(w);
  return pair_F(q->m, q->E, eps) * eps;
}
/* screening kinks: phi_i jumps at delta = 1, and G_i reaches zero (and
 * stays there) at delta_G on the logarithmic branch */
static double delta_zero(const or_mat* m) {
  return exp((21.12 - 4.0 * (m->lnz / 3.0 + m->fc)) / 4.184) - 0.952;
}
/* integral of f over [a, b] split at the sorted interior points brk[],
 * 16 panels of 8-point Gauss-Legendre on each piece */
static double integrate_pieces(or_fn f, const void* par, double a, double b,
                               const double* brk, int nbrk) {
  double lo = a, sum = 0.0;
  for (int i = 0; i <= nbrk; ++i) {
    double hi = (i < nbrk) ? brk[i] : b;
    if (hi > b) hi = b;
    if (hi > lo) {
      sum += integrate(f, par, lo, hi, 16, 8);
      lo = hi;
    }
  }
  return sum;
}
static double xs_pair(const or_mat* m, double E) {
  if (E <= 2.0 * ME) return 0.0;
  pair_par p = {m, E};
  double eps0 = ME / E;
  /* eps(1-eps) = 136 Z^{-1/3} eps0 / d gives the eps where delta = d;
   * delta decreases with eps on [eps0, 1/2] */
  double dk[2] = {delta_zero(m), 1.0}, brk[2];
  int nb = 0;
  for (int i = 0; i < 2; ++i) {
    double q = 4.0 * 136.0 * m->zm13 * eps0 / dk[i];
    if (q < 1.0) {
      double e = 0.5 * (1.0 - sqrt(1.0 - q));
      if (e > eps0 && e < 0.5) brk[nb++] = log(e);
    }
  }
  return 2.0 * pair_pref(m) * integrate_pieces(pair_integrand, &p, log(eps0), log(0.5), brk, nb);
}

/* ------------------------------------------------------------------ */
/* Bremsstrahlung: screened 1/k spectrum with the same screening       */
/* ------------------------------------------------------------------ */
/* brace(T, k) so that d sigma / d k = pref * brace / k */
static double brem_brace(const or_mat* m, double T, double k) {
  double et = T + ME;
  double y = k / et;
  double d = 136.0 * m->zm13 * ME * y / (et * (1.0 - y));
  double v = (1.0 + (1.0 - y) * (1.0 - y)) * gfun(m, phi1(d)) -
             (2.0 / 3.0) * (1.0 - y) * gfun(m, phi2(d));
  return v > 0.0 ? v : 0.0;
}
/* sampler bound on [k_c, T]: brace <= 2 G1(delta) and delta grows with k */
static double brem_bound(const or_mat* m, double T, double kc) {
  double et = T + ME;
  double y = kc / et;
  double d = 136.0 * m->zm13 * ME * y / (et * (1.0 - y));
  return 2.0 * gfun(m, phi1_env(d));
}
typedef struct { const or_mat* m; double T; } brem_par;
/* integrand in v = ln(k / (E_t - k)): d ln k = (1 - y) dv */
static double brem_logit_integrand(const void* p, double v) {
  const brem_par* q = (const brem_par*)p;
  double et = q->T + ME;
  double y = 1.0 / (1.0 + exp(-v));
  return brem_brace(q->m, q->T, y * et) * (1.0 - y);
}
static double brem_k_integrand(const void* p, double k) {
  const brem_par* q = (const brem_par*)p;
  return brem_brace(q->m, q->T, k);
}
/* photon energy k at which delta reaches d (delta grows with k) */
static double brem_k_of_delta(const or_mat* m, double T, double d) {
  double et = T + ME;
  double r = d * et / (136.0 * m->zm13 * ME);
  return et * r / (1.0 + r);
}
/* per-atom cross section for photons above k_c; delta = d at
 * v = ln(d E_t / (136 Z^{-1/3} m)) */
static double xs_brem(const or_mat* m, double T, double kc) {
  if (T <= kc) return 0.0;
  brem_par p = {m, T};
  double et = T + ME;
  double va = log(kc / (et - kc)), vb = log(T / (et - T));
  double dk[2] = {1.0, delta_zero(m)}, brk[2];
  int nb = 0;
  for (int i = 0; i < 2; ++i) {
    double v = log(dk[i] * et / (136.0 * m->zm13 * ME));
    if (v > va && v < vb) brk[nb++] = v;
  }
  return pair_pref(m) * integrate_pieces(brem_logit_integrand, &p, va, vb, brk, nb);
}
/* restricted radiative loss, MeV/mm: n_at * int_0^{min(kc,T)} k dsigma/dk */
static double sbrem(const or_mat* m, double T, double kc) {
  double kmax = T < kc ? T : kc;
  brem_par p = {m, T};
  double brk[2] = {brem_k_of_delta(m, T, 1.0), brem_k_of_delta(m, T, delta_zero(m))};
  int nb = 0;
  double b2[2];
  for (int i = 0; i < 2; ++i)
    if (brk[i] > 0.0 && brk[i] < kmax) b2[nb++] = brk[i];
  return m->n_at * pair_pref(m) * integrate_pieces(brem_k_integrand, &p, 0.0, kmax, b2, nb);
}

/* ------------------------------------------------------------------ */
/* Ionisation: Moller (e-e-) and Bhabha (e+e-) per electron            */
/* ------------------------------------------------------------------ */
static double xs_moller(double T, double tcut) {
  if (T <= 2.0 * tcut) return 0.0;
  double x = tcut / T, g = T / ME + 1.0, b2 = 1.0 - 1.0 / (g * g);
  double c = ((g - 1.0) / g) * ((g - 1.0) / g), d = (2.0 * g - 1.0) / (g * g);
  double br = c * (0.5 - x) + 1.0 / x - 1.0 / (1.0 - x) - d * log((1.0 - x) / x);
  return 2.0 * PI * RE * RE * ME / (b2 * T) * br;
}
static double dsde_moller(double T, double eps) {
  double g = T / ME + 1.0, b2 = 1.0 - 1.0 / (g * g);
  double c = ((g - 1.0) / g) * ((g - 1.0) / g), d = (2.0 * g - 1.0) / (g * g);
  double br = c + 1.0 / (eps * eps) + 1.0 / ((1.0 - eps) * (1.0 - eps)) -
              d / (eps * (1.0 - eps));
  return 2.0 * PI * RE * RE * ME / (b2 * T) * br;
}
typedef struct { double b1, b2, b3, b4, beta2; } bhabha_c;
static bhabha_c bhabha_coef(double T) {
  bhabha_c c;
  double g = T / ME + 1.0;
  double y = 1.0 / (g + 1.0), w = 1.0 - 2.0 * y;
  c.beta2 = 1.0 - 1.0 / (g * g);
  c.b1 = 2.0 - y * y;
  c.b2 = w * (3.0 + y * y);
  c.b4 = w * w * w;
  c.b3 = c.b4 + w * w;
  return c;
}
static double xs_bhabha(double T, double tcut) {
  if (T <= tcut) return 0.0;
  double x = tcut / T;
  bhabha_c c = bhabha_coef(T);
  double br = (1.0 / c.beta2) * (1.0 / x - 1.0) - c.b1 * log(1.0 / x) + c.b2 * (1.0 - x) -
              0.5 * c.b3 * (1.0 - x * x) + (c.b4 / 3.0) * (1.0 - x * x * x);
  return 2.0 * PI * RE * RE * ME / T * br;
}
static double dsde_bhabha(double T, double eps) {
  bhabha_c c = bhabha_coef(T);
  double br = 1.0 / (c.beta2 * eps * eps) - c.b1 / eps + c.b2 - c.b3 * eps + c.b4 * eps * eps;
  return 2.0 * PI * RE * RE * ME / T * br;
}

/* restricted collision stopping power (Berger-Seltzer as in ICRU 37),
 * MeV/mm; positron = 0 for e-, 1 for e+ */
static double sion(const or_mat* m, double T, double tcut, int positron) {
  double tau = T / ME, g = tau + 1.0, b2 = 1.0 - 1.0 / (g * g);
  double tmax = positron ? T : 0.5 * T;
  double dl = (tcut < tmax ? tcut : tmax) / ME;
  double im = m->I / ME;
  double f;
  if (!positron) {
    f = -1.0 - b2 + log((tau - dl) * dl) + tau / (tau - dl) +
        (0.5 * dl * dl + (2.0 * tau + 1.0) * log(1.0 - dl / tau)) / (g * g);
  } else {
    double y = 1.0 / (g + 1.0);
    double d2 = dl * dl, d3 = d2 * dl, d4 = d3 * dl;
    f = log(tau * dl) -
        (b2 / tau) * (tau + 2.0 * dl - 1.5 * d2 * y - (dl - d3 / 3.0) * y * y -
                      (0.5 * d2 - tau * d3 / 3.0 + 0.25 * d4) * y * y * y);
  }
  /* asymptotic density-effect correction, clamped at zero */
  double bg = sqrt(b2) * g;
  double dd = 2.0 * log(m->plasma / m->I) + 2.0 * log(bg) - 1.0;
  if (dd < 0.0) dd = 0.0;
  double v = 2.0 * PI * RE * RE * ME * m->n_el / b2 *
             (log(2.0 * (tau + 2.0) / (im * im)) + f - dd);
  return v > 0.0 ? v : 0.0;
}

/* ------------------------------------------------------------------ */
/* Annihilation in flight: Heitler two-photon cross section per e-      */
/* ------------------------------------------------------------------ */
static double xs_annih(double T) {
  double g = T / ME + 1.0, g2 = g * g, s = sqrt(g2 - 1.0);
  return PI * RE * RE / (g + 1.0) *
         ((g2 + 4.0 * g + 1.0) / (g2 - 1.0) * log(g + s) - (g + 3.0) / s);
}

/* ------------------------------------------------------------------ */
/* Tables on the log-energy grid                                       */
/* ------------------------------------------------------------------ */
static double* tab_ptr(const or_ctx* c, uint32_t m, uint32_t t) {
  return c->tab + ((size_t)m * OR_N_TABLES + t) * (c->nb + 1);
}
static double node_energy(const or_ctx* c, int j) {
  return exp(c->lnemin + j * c->dlog);
}
/* bin j in [0, nb-1] and fraction t in [0,1] of log-energy lnE */
static void bin_of(const or_ctx* c, double lnE, int* j, double* t) {
  double x = (lnE - c->lnemin) / c->dlog;
  double f = floor(x);
  int jj;
  if (f < 0.0) jj = 0;
  else if (f > (double)(c->nb - 1)) jj = (int)c->nb - 1;
  else jj = (int)f;
  double tt = x - jj;
  if (tt < 0.0) tt = 0.0;
  if (tt > 1.0) tt = 1.0;
  *j = jj;
  *t = tt;
}
static double interp(const double* f, int j, double t) {
  return f[j] + t * (f[j + 1] - f[j]);
}

typedef struct { const double* S; double e0, dlog; int j; } range_par;
static double range_integrand(const void* p, double t) {
  const range_par* q = (const range_par*)p;
  double E = q->e0 * exp(t * q->dlog);
  double S = q->S[q->j - 1] + t * (q->S[q->j] - q->S[q->j - 1]);
  return E / S;
}
static void build_range(const or_ctx* c, const double* S, double* R) {
  R[0] = node_energy(c, 0) / (2.0 * S[0]);
  for (uint32_t j = 1; j <= c->nb; ++j) {
    range_par p = {S, node_energy(c, (int)j - 1), c->dlog, (int)j};
    R[j] = R[j - 1] + c->dlog * integrate(range_integrand, &p, 0.0, 1.0, 1, 16);
  }
}

static double* eltab_ptr(const or_ctx* c, uint32_t m, uint32_t el, int brem) {
  return c->eltab + (((size_t)m * OR_MAX_EL + el) * 2 + brem) * (c->nb + 1);
}

static void build_tables(or_ctx* c) {
  uint32_t mask = c->s.process_mask;
  for (uint32_t mi = 0; mi < c->n_mat; ++mi) {
    const or_mat* m = &c->mat[mi];
    const or_mat* el = &c->el[(size_t)mi * OR_MAX_EL];
    for (uint32_t j = 0; j <= c->nb; ++j) {
      double E = node_energy(c, (int)j);
      /* per-atom processes add up over the elements; per-electron ones
       * scale with the material's electron density */
      double sp = 0.0, sv = 0.0, sr = 0.0, sb = 0.0;
      for (uint32_t i = 0; i < c->n_el[mi]; ++i) {
        sp += el[i].n_at * xs_photo(&el[i], E);
        double v = el[i].n_at * xs_pair(&el[i], E);
        double r = el[i].n_at * xs_brem(&el[i], E, c->kcut);
        eltab_ptr(c, mi, i, 0)[j] = (mask & OR_P_CONV) ? v : 0.0;
        eltab_ptr(c, mi, i, 1)[j] = (mask & OR_P_EBREM) ? r : 0.0;
        sv += v;
        sr += r;
        sb += sbrem(&el[i], E, c->kcut);
      }
      tab_ptr(c, mi, T_COMPT)[j] = m->n_el * xs_compton(E);
      tab_ptr(c, mi, T_PHOT)[j] = sp;
      tab_ptr(c, mi, T_CONV)[j] = sv;
      tab_ptr(c, mi, T_BREM)[j] = sr;
      tab_ptr(c, mi, T_MOLLER)[j] = m->n_el * xs_moller(E, c->tcut);
      tab_ptr(c, mi, T_BHABHA)[j] = m->n_el * xs_bhabha(E, c->tcut);
      tab_ptr(c, mi, T_ANNIH)[j] = m->n_el * xs_annih(E);
      tab_ptr(c, mi, T_S_EM)[j] = sion(m, E, c->tcut, 0) + sb;
      tab_ptr(c, mi, T_S_EP)[j] = sion(m, E, c->tcut, 1) + sb;
    }
    build_range(c, tab_ptr(c, mi, T_S_EM), tab_ptr(c, mi, T_R_EM));
    build_range(c, tab_ptr(c, mi, T_S_EP), tab_ptr(c, mi, T_R_EP));
    /* processes switched off contribute nothing */
    uint32_t off[7][2] = {{OR_P_COMPTON, T_COMPT}, {OR_P_PHOT, T_PHOT},
                          {OR_P_CONV, T_CONV},     {OR_P_EIONI, T_MOLLER},
                          {OR_P_EIONI, T_BHABHA},  {OR_P_EBREM, T_BREM},
                          {OR_P_ANNIH, T_ANNIH}};
    for (int k = 0; k < 7; ++k)
      if (!(mask & off[k][0])) memset(tab_ptr(c, mi, off[k][1]), 0, sizeof(double) * (c->nb + 1));
  }
}

/* cross-section value with an explicit threshold: zero at and below th */
static double xs_lookup(const or_ctx* c, uint32_t m, uint32_t t, double E,
                        double th) {
  if (E <= th) return 0.0;
  int j;
  double u;
  bin_of(c, log(E), &j, &u);
  return interp(tab_ptr(c, m, t), j, u);
}
static double plain_lookup(const or_ctx* c, uint32_t m, uint32_t t, double E) {
  int j;
  double u;
  bin_of(c, log(E), &j, &u);
  return interp(tab_ptr(c, m, t), j, u);
}

/* inverse of the range interpolant: largest node j with R_j <= r */
static double inv_range(const or_ctx* c, const double* R, double r) {
  int lo = 0, hi = (int)c->nb;
  if (r < R[0]) lo = 0;
  else {
    while (hi - lo > 1) {
      int mid = (lo + hi) / 2;
      if (R[mid] <= r) lo = mid;
      else hi = mid;
    }
    if (R[hi] <= r) lo = hi;
  }
  if (lo > (int)c->nb - 1) lo = (int)c->nb - 1;
  double lnE = c->lnemin + lo * c->dlog + c->dlog * (r - R[lo]) / (R[lo + 1] - R[lo]);
  return exp(lnE);
}

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)                   */
/* ------------------------------------------------------------------ */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* two 32-bit words -> uniform in (0,1): 52 random bits, centred */
static double u_of(uint32_t lo, uint32_t hi) {
  uint64_t x = ((uint64_t)hi << 32) | (uint64_t)lo;
  return ((double)(x >> 12) + 0.5) * 0x1p-52;
}

double or_uniform(const uint32_t key[2], uint64_t id, uint32_t step, uint32_t i) {
  uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), step, i / 2u};
  uint32_t w[4];
  or_philox(ctr, key, w);
  return (i % 2u == 0u) ? u_of(w[0], w[1]) : u_of(w[2], w[3]);
}

uint64_t or_child_id(const uint32_t key[2], uint64_t id, uint32_t step, uint32_t k) {
  uint32_t ctr[4] = {(uint32_t)id, (uint32_t)(id >> 32), step, 0x80000000u | k};
  uint32_t w[4];
  or_philox(ctr, key, w);
  return (uint64_t)w[0] | ((uint64_t)w[1] << 32);
}

/* draw stream of one step: U_i addressed by index */
typedef struct {
  uint32_t key[2];
  uint64_t id;
  uint32_t step;
  uint32_t next;   /* next index handed out by draw() */
} or_stream;
static double draw_at(const or_stream* s, uint32_t i) {
  return or_uniform(s->key, s->id, s->step, i);
}
static double draw(or_stream* s) {
  return draw_at(s, s->next++);
}

/* ------------------------------------------------------------------ */
/* Directions                                                          */
/* ------------------------------------------------------------------ */
/* rotate the local direction (sin t cos p, sin t sin p, cos t), given in a
 * frame whose z axis is u, to the lab frame: columns of the rotation are
 * e1 = (ux uz, uy uz, -(ux^2+uy^2))/|u_perp|, e2 = (-uy, ux, 0)/|u_perp|, u */
static void rotate_to(const double u[3], double sint, double cost, double phi,
                      double out[3]) {
  double lx = sint * cos(phi), ly = sint * sin(phi), lz = cost;
  double up2 = u[0] * u[0] + u[1] * u[1];
  if (up2 > 0.0) {
    double up = sqrt(up2);
    out[0] = (u[0] * u[2] * lx - u[1] * ly) / up + u[0] * lz;
    out[1] = (u[1] * u[2] * lx + u[0] * ly) / up + u[1] * lz;
    out[2] = -up * lx + u[2] * lz;
  } else if (u[2] > 0.0) {
    out[0] = lx; out[1] = ly; out[2] = lz;
  } else {
    out[0] = -lx; out[1] = ly; out[2] = -lz;
  }
}
static void normalise(double v[3]) {
  double n = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  v[0] /= n; v[1] /= n; v[2] /= n;
}

/* ------------------------------------------------------------------ */
/* Interaction samplers (draws from index 2 onward, in program order)   */
/* ------------------------------------------------------------------ */
typedef struct {
  int parent_alive;
  double parent_E, parent_dir[3];
  int n_sec;
  int sec_species[2];
  double sec_E[2], sec_dir[2][3];
  double var;
  int trials;
} or_inter;

/* Compton: Klein-Nishina by the Butcher-Messel mixture of 1/eps and eps */
static void sample_compton(double E, const double u[3], or_stream* rs, or_inter* o) {
  double k = E / ME;
  double eps0 = 1.0 / (1.0 + 2.0 * k);
  double a1 = -log(eps0), a2 = 0.5 * (1.0 - eps0 * eps0);
  double eps = 1.0, t = 0.0;
  int n = 0;
  for (;;) {
    double a = draw(rs), b = draw(rs), cc = draw(rs);
    ++n;
    if (a * (a1 + a2) < a1) eps = exp(-a1 * b);
    else eps = sqrt(eps0 * eps0 + (1.0 - eps0 * eps0) * b);
    t = (1.0 - eps) / (k * eps);
    double sin2 = t * (2.0 - t);
    if (cc <= 1.0 - eps * sin2 / (1.0 + eps * eps) || n >= OR_MAX_TRIALS) break;
  }
  double cost = 1.0 - t;
  double s2 = 1.0 - cost * cost;
  double sint = sqrt(s2 > 0.0 ? s2 : 0.0);
  double phi = 2.0 * PI * draw(rs);
  o->var = eps;
  o->trials = n;
  o->parent_alive = 1;
  o->parent_E = eps * E;
  rotate_to(u, sint, cost, phi, o->parent_dir);
  o->n_sec = 1;
  o->sec_species[0] = OR_ELECTRON;
  o->sec_E[0] = E - eps * E;
  for (int i = 0; i < 3; ++i) o->sec_dir[0][i] = E * u[i] - eps * E * o->parent_dir[i];
  normalise(o->sec_dir[0]);
}

/* photo-effect: the photon is absorbed, the electron takes E along u */
static void sample_photo(double E, const double u[3], or_inter* o) {
  o->var = E;
  o->trials = 0;
  o->parent_alive = 0;
  o->n_sec = 1;
  o->sec_species[0] = OR_ELECTRON;
  o->sec_E[0] = E;
  for (int i = 0; i < 3; ++i) o->sec_dir[0][i] = u[i];
}

/* pair: uniform eps on [eps0, 1/2], rejection on F(eps)/F_max, then the
 * next draw decides which lepton takes eps; both collinear with u */
/* target element of a pair (brem = 0) or bremsstrahlung (brem = 1)
 * interaction at energy E in material m: with several elements, the next
 * draw u picks the first element whose partial sum of interpolated
 * per-element cross sections exceeds u times their total */
static const or_mat* pick_element(const or_ctx* c, uint32_t m, int brem, double E, or_stream* rs) {
  const or_mat* el = &c->el[(size_t)m * OR_MAX_EL];
  uint32_t n = c->n_el[m];
  if (n == 1) return &el[0];
  double u = draw(rs);
  int j;
  double t;
  bin_of(c, log(E), &j, &t);
  double s[OR_MAX_EL], tot = 0.0;
  for (uint32_t i = 0; i < n; ++i) {
    s[i] = interp(eltab_ptr(c, m, i, brem), j, t);
    tot += s[i];
  }
  double cum = 0.0;
  for (uint32_t i = 0; i + 1 < n; ++i) {
    cum += s[i];
    if (u * tot < cum) return &el[i];
  }
  return &el[n - 1];
}

static void sample_pair(const or_mat* m, double E, const double u[3], or_stream* rs,
                        or_inter* o) {
  double eps0 = ME / E, fmax = pair_Fmax(m, E);
  double eps = 0.5;
  int n = 0;
  for (;;) {
    double a = draw(rs), b = draw(rs);
    ++n;
    eps = eps0 + a * (0.5 - eps0);
    if (b * fmax <= pair_F(m, E, eps) || n >= OR_MAX_TRIALS) break;
  }
  double c = draw(rs);
  double ep = (c < 0.5) ? eps * E : (1.0 - eps) * E;
  double em = E - ep;
  o->var = eps;
  o->trials = n;
  o->parent_alive = 0;
  o->n_sec = 2;
  o->sec_species[0] = OR_ELECTRON;
  o->sec_E[0] = em - ME;
  o->sec_species[1] = OR_POSITRON;
  o->sec_E[1] = ep - ME;
  for (int i = 0; i < 3; ++i) o->sec_dir[0][i] = o->sec_dir[1][i] = u[i];
}

/* bremsstrahlung above k_c: k from the 1/k envelope, rejection on brace */
static void sample_brem(const or_mat* m, double T, double kc, const double u[3],
                        or_stream* rs, or_inter* o) {
  double bound = brem_bound(m, T, kc);
  double k = kc;
  int n = 0;
  for (;;) {
    double a = draw(rs), b = draw(rs);
    ++n;
    k = kc * pow(T / kc, a);
    if (b * bound <= brem_brace(m, T, k) || n >= OR_MAX_TRIALS) break;
  }
  o->var = k;
  o->trials = n;
  o->parent_alive = 1;
  o->parent_E = T - k;
  for (int i = 0; i < 3; ++i) o->parent_dir[i] = u[i];
  o->n_sec = 1;
  o->sec_species[0] = OR_GAMMA;
  o->sec_E[0] = k;
  for (int i = 0; i < 3; ++i) o->sec_dir[0][i] = u[i];
}

/* shared two-body kinematics of a delta ray of kinetic energy td */
static void delta_kinematics(double T, double td, const double u[3], or_stream* rs,
                             or_inter* o) {
  double cost = sqrt(td * (T + 2.0 * ME) / (T * (td + 2.0 * ME)));
  double s2 = 1.0 - cost * cost;
  double sint = sqrt(s2 > 0.0 ? s2 : 0.0);
  double phi = 2.0 * PI * draw(rs);
  double ud[3];
  rotate_to(u, sint, cost, phi, ud);
  double p = sqrt(T * (T + 2.0 * ME)), pd = sqrt(td * (td + 2.0 * ME));
  o->parent_alive = 1;
  o->parent_E = T - td;
  for (int i = 0; i < 3; ++i) o->parent_dir[i] = p * u[i] - pd * ud[i];
  normalise(o->parent_dir);
  o->n_sec = 1;
  o->sec_species[0] = OR_ELECTRON;
  o->sec_E[0] = td;
  for (int i = 0; i < 3; ++i) o->sec_dir[0][i] = ud[i];
}

/* Moller: eps in [x, 1/2] from the 1/eps^2 envelope */
static void sample_moller(double T, double tcut, const double u[3], or_stream* rs,
                          or_inter* o) {
  double x = tcut / T, g = T / ME + 1.0;
  double c = ((g - 1.0) / g) * ((g - 1.0) / g), d = (2.0 * g - 1.0) / (g * g);
  double bound = 2.0 + 0.25 * c;
  double eps = x;
  int n = 0;
  for (;;) {
    double a = draw(rs), b = draw(rs);
    ++n;
    eps = x / (1.0 - a * (1.0 - 2.0 * x));
    double f = c * eps * eps + 1.0 + (eps * eps) / ((1.0 - eps) * (1.0 - eps)) -
               d * eps / (1.0 - eps);
    if (b * bound <= f || n >= OR_MAX_TRIALS) break;
  }
  o->var = eps;
  o->trials = n;
  delta_kinematics(T, eps * T, u, rs, o);
}

/* Bhabha: eps in [x, 1] from the 1/eps^2 envelope, bound 1/beta^2 */
static void sample_bhabha(double T, double tcut, const double u[3], or_stream* rs,
                          or_inter* o) {
  double x = tcut / T;
  bhabha_c c = bhabha_coef(T);
  double bound = 1.0 / c.beta2;
  double eps = x;
  int n = 0;
  for (;;) {
    double a = draw(rs), b = draw(rs);
    ++n;
    eps = x / (1.0 - a * (1.0 - x));
    double e2 = eps * eps;
    double f = 1.0 / c.beta2 - c.b1 * eps + c.b2 * e2 - c.b3 * e2 * eps + c.b4 * e2 * e2;
    if (b * bound <= f || n >= OR_MAX_TRIALS) break;
  }
  o->var = eps;
  o->trials = n;
  delta_kinematics(T, eps * T, u, rs, o);
}

/* annihilation in flight (Heitler): photon-energy fraction eps from the
 * 1/eps envelope on [eps_min, 1 - eps_min], rejection on g(eps) <= 1 */
static void sample_annih(double T, const double u[3], or_stream* rs, or_inter* o) {
  double g = T / ME + 1.0, s = sqrt(g * g - 1.0);
  double emin = 1.0 / (g + 1.0 + s), emax = 1.0 - emin;
  double eps = emin;
  int n = 0;
  for (;;) {
    double a = draw(rs), b = draw(rs);
    ++n;
    eps = emin * pow(emax / emin, a);
    double gr = 1.0 - eps + (2.0 * g * eps - 1.0) / (eps * (g + 1.0) * (g + 1.0));
    if (b <= gr || n >= OR_MAX_TRIALS) break;
  }
  double etot = T + 2.0 * ME;
  double cost = (eps * (g + 1.0) - 1.0) / (eps * s);
  if (cost > 1.0) cost = 1.0;
  if (cost < -1.0) cost = -1.0;
  double sint = sqrt(1.0 - cost * cost);
  double phi = 2.0 * PI * draw(rs);
  o->var = eps;
  o->trials = n;
  o->parent_alive = 0;
  o->n_sec = 2;
  o->sec_species[0] = o->sec_species[1] = OR_GAMMA;
  o->sec_E[0] = eps * etot;
  o->sec_E[1] = (1.0 - eps) * etot;
  rotate_to(u, sint, cost, phi, o->sec_dir[0]);
  double p = sqrt(T * (T + 2.0 * ME));
  for (int i = 0; i < 3; ++i) o->sec_dir[1][i] = p * u[i] - o->sec_E[0] * o->sec_dir[0][i];
  normalise(o->sec_dir[1]);
}

/* annihilation at rest: two back-to-back photons of energy m, isotropic,
 * from draws U1 (cos theta) and U2 (phi) */
static void annih_at_rest(const or_stream* rs, or_inter* o) {
  double cost = 2.0 * draw_at(rs, 1) - 1.0;
  double phi = 2.0 * PI * draw_at(rs, 2);
  double s2 = 1.0 - cost * cost;
  double sint = sqrt(s2 > 0.0 ? s2 : 0.0);
  o->var = cost;
  o->trials = 0;
  o->parent_alive = 0;
  o->n_sec = 2;
  o->sec_species[0] = o->sec_species[1] = OR_GAMMA;
  o->sec_E[0] = o->sec_E[1] = ME;
  o->sec_dir[0][0] = sint * cos(phi);
  o->sec_dir[0][1] = sint * sin(phi);
  o->sec_dir[0][2] = cost;
  for (int i = 0; i < 3; ++i) o->sec_dir[1][i] = -o->sec_dir[0][i];
}

/* ------------------------------------------------------------------ */
/* Transport                                                           */
/* ------------------------------------------------------------------ */
typedef struct {
  int species;
  double E;
  double pos[3], dir[3];
  int slab;
  uint32_t event;
  uint64_t id;
  uint32_t step;
  uint32_t birth;   /* breadth-first iteration in which step 0 is taken */
} or_track;

typedef struct {
  or_track* v;
  size_t n, cap, head;  /* head: FIFO read position */
} or_stack;

static int stack_push(or_stack* s, const or_track* t) {
  if (s->n == s->cap) {
    size_t nc = s->cap ? 2 * s->cap : 1024;
    or_track* nv = (or_track*)realloc(s->v, nc * sizeof(or_track));
    if (!nv) return -1;
    s->v = nv;
    s->cap = nc;
  }
  s->v[s->n++] = *t;
  return 0;
}

typedef struct {
  or_ctx* c;
  uint32_t key[2];
  uint32_t row;
  double* edep;          /* this event's row */
  or_ledger* led;
  or_step_rec* log;
  uint64_t log_cap;
  uint64_t* log_n;
  uint64_t* profile;
  uint32_t profile_cap;
  uint32_t* profile_len;
  or_stack* st;
  int err;
  or_primary* exits;     /* outgoing tracks (NULL: not recorded)          */
  uint64_t exits_cap;
  uint64_t* exits_n;
} or_event;

static void deposit(or_event* ev, int slab, double e, or_step_rec* rec) {
  ev->edep[slab] += e;
  ev->led->edep += e;
  rec->edep += e;
}

/* push (or deposit, below the tracking cut) secondary k of parent p */
static void emit(or_event* ev, const or_track* p, uint32_t k, int species, double E,
                 const double dir[3], or_step_rec* rec) {
  or_ctx* c = ev->c;
  if (species != OR_POSITRON && E < c->ecut) {
    deposit(ev, p->slab, E, rec);
    return;
  }
  or_track t;
  t.species = species;
  t.E = E;
  for (int i = 0; i < 3; ++i) {
    t.pos[i] = p->pos[i];
    t.dir[i] = dir[i];
  }
  t.slab = p->slab;
  t.event = p->event;
  t.id = or_child_id(ev->key, p->id, p->step, k);
  t.step = 0;
  t.birth = p->birth + p->step + 1;
  ev->led->n_created[species] += 1;
  if (stack_push(ev->st, &t)) ev->err = -2;
}

static void apply(or_event* ev, or_track* tr, const or_inter* o, or_step_rec* rec) {
  for (int k = 0; k < o->n_sec; ++k)
    emit(ev, tr, (uint32_t)k, o->sec_species[k], o->sec_E[k], o->sec_dir[k], rec);
  if (o->parent_alive) {
    tr->E = o->parent_E;
    for (int i = 0; i < 3; ++i) tr->dir[i] = o->parent_dir[i];
  } else {
    tr->E = 0.0;
    tr->slab = -1;
  }
}

/* distance along a straight line or helix (u_z is constant) to the z
 * planes of the current slab */
static double dist_z(const or_ctx* c, const or_track* t) {
  if (t->dir[2] > 0.0) return (c->z[t->slab + 1] - t->pos[2]) / t->dir[2];
  if (t->dir[2] < 0.0) return (c->z[t->slab] - t->pos[2]) / t->dir[2];
  return INFINITY;
}
/* straight-line distance to the transverse walls x = +-H, y = +-H */
static double dist_wall(const or_ctx* c, const or_track* t) {
  double h = c->s.half_xy_mm, s = INFINITY;
  for (int i = 0; i < 2; ++i) {
    double d = INFINITY;
    if (t->dir[i] > 0.0) d = (h - t->pos[i]) / t->dir[i];
    else if (t->dir[i] < 0.0) d = (-h - t->pos[i]) / t->dir[i];
    if (d < s) s = d;
  }
  return s;
}
/* ---- box geometry ---- */
static uint32_t vol_material(const or_ctx* c, int v) {
  if (!c->nbox) return c->slab_mat[v];
  return (uint32_t)v < c->nbox ? c->bmat[v] : c->wmat;
}
static int in_axis(double p, double lo, double hi, double u) {
  return (p > lo && p < hi) || (p == lo && u >= 0.0) || (p == hi && u < 0.0);
}
static int in_box(const double* lo, const double* hi, const double p[3], const double u[3]) {
  return in_axis(p[0], lo[0], hi[0], u[0]) && in_axis(p[1], lo[1], hi[1], u[1]) &&
         in_axis(p[2], lo[2], hi[2], u[2]);
}
static int box_locate(const or_ctx* c, const double p[3], const double u[3]) {
  for (uint32_t b = 0; b < c->nbox; ++b)
    if (in_box(c->blo + 3 * b, c->bhi + 3 * b, p, u)) return (int)b;
  return in_box(c->wlo, c->whi, p, u) ? (int)c->nbox : -1;
}
/* leaving a box from inside: nearest exit face (first axis on ties) */
static double ray_exit(const double* lo, const double* hi, const double p[3], const double u[3],
                       int* ax, double* face) {
  double s = INFINITY;
  for (int k = 0; k < 3; ++k) {
    double d = INFINITY, f = 0.0;
    if (u[k] > 0.0) { d = (hi[k] - p[k]) / u[k]; f = hi[k]; }
    else if (u[k] < 0.0) { d = (lo[k] - p[k]) / u[k]; f = lo[k]; }
    if (d < s) { s = d; *ax = k; *face = f; }
  }
  return s;
}
/* entering a box from outside (slab method): the entry distance, or
 * infinity if the ray misses it, grazes an edge or moves away */
static double ray_entry(const double* lo, const double* hi, const double p[3], const double u[3],
                        int* ax, double* face) {
  double tn = -INFINITY, tf = INFINITY;
  int a = -1;
  double f = 0.0;
  for (int k = 0; k < 3; ++k) {
    if (u[k] == 0.0) {
      if (!(p[k] >= lo[k] && p[k] < hi[k])) return INFINITY;
      continue;
    }
    double t1 = (lo[k] - p[k]) / u[k], t2 = (hi[k] - p[k]) / u[k];
    double near = t1 < t2 ? t1 : t2, far = t1 < t2 ? t2 : t1;
    if (near > tn) { tn = near; a = k; f = u[k] > 0.0 ? lo[k] : hi[k]; }
    if (far < tf) tf = far;
  }
  if (a < 0 || !(tn < tf) || !(tf > 0.0)) return INFINITY;
  *ax = a;
  *face = f;
  return tn > 0.0 ? tn : 0.0;
}
/* distance to the next boundary from volume v: a box's own faces, or from
 * the world the nearer of its exit and the first box entered (boxes win
 * ties) */
static double box_distance(const or_ctx* c, int v, const double p[3], const double u[3],
                           int* ax, double* face) {
  if ((uint32_t)v < c->nbox) return ray_exit(c->blo + 3 * v, c->bhi + 3 * v, p, u, ax, face);
  double s = ray_exit(c->wlo, c->whi, p, u, ax, face);
  for (uint32_t b = 0; b < c->nbox; ++b) {
    int a = 0;
    double f = 0.0;
    double d = ray_entry(c->blo + 3 * b, c->bhi + 3 * b, p, u, &a, &f);
    if (d <= s) { s = d; *ax = a; *face = f; }
  }
  return s;
}

static void move_straight(or_track* t, double s) {
  for (int i = 0; i < 3; ++i) t->pos[i] += s * t->dir[i];
}
/* exact helix in B = Bz z-hat; curvature from the pre-step momentum */
static void move_helix(or_track* t, double kappa, double s) {
  double phi = kappa * s;
  double sp = sin(phi), cp = cos(phi), h = sin(0.5 * phi);
  double omc = 2.0 * h * h;
  double ux = t->dir[0], uy = t->dir[1];
  t->pos[0] += (ux * sp + uy * omc) / kappa;
  t->pos[1] += (uy * sp - ux * omc) / kappa;
  t->pos[2] += t->dir[2] * s;
  t->dir[0] = ux * cp + uy * sp;
  t->dir[1] = -ux * sp + uy * cp;
}
/* ---- charged tracks in a box geometry with a field ----
 * Reading (section 2.3 asks for propagation in the field with the boundary
 * found along the curved path): the step follows the exact helix of
 * move_helix, and a box face is reached where the helix meets its plane.
 * With psi = |kappa| s the angle turned, the transverse motion is the
 * circle x = xc + r sin(psi - beta), y = yc + sg r cos(psi - beta) (sg the
 * sign of kappa, r = u_perp / |kappa|), so a plane x = X or y = Y is met at
 * angles given by asin or acos; z = z0 + uz s is linear. */
typedef struct {
  double x0, y0, z0, uz, ak, r, xc, yc, beta;
  int sg;
} or_helix;

static or_helix helix_of(const double p[3], const double u[3], double kappa) {
  or_helix h;
  h.x0 = p[0];
  h.y0 = p[1];
  h.z0 = p[2];
  h.uz = u[2];
  h.ak = fabs(kappa);
  h.sg = kappa > 0.0 ? 1 : -1;
  double up = sqrt(u[0] * u[0] + u[1] * u[1]);
  h.r = up / h.ak;
  h.xc = p[0] + u[1] / kappa;
  h.yc = p[1] - u[0] / kappa;
  /* x - xc = (u_x sin phi - u_y cos phi) / kappa with phi = kappa s */
  h.beta = h.sg * atan2(u[1], u[0]);
  return h;
}

/* the point after path s (the same formulas as move_helix) */
static void helix_at(const or_helix* h, const double u[3], double kappa, double s, double out[3]) {
  double phi = kappa * s;
  double sp = sin(phi), hh = sin(0.5 * phi), omc = 2.0 * hh * hh;
  out[0] = h->x0 + (u[0] * sp + u[1] * omc) / kappa;
  out[1] = h->y0 + (u[1] * sp - u[0] * omc) / kappa;
  out[2] = h->z0 + u[2] * s;
}

/* angle psi in [0, 2 pi) from the start to the angle theta of the circle
 * (theta = psi - beta); within 1e-9 of a full turn counts as 0 (the start
 * itself, up to rounding) */
static double helix_turn_to(const or_helix* h, double theta) {
  double d = fmod(theta + h->beta, 2.0 * PI);
  if (d < 0.0) d += 2.0 * PI;
  if (d > 2.0 * PI - 1e-9) d = 0.0;
  return d;
}

/* first angle psi >= 0 at which the helix crosses the plane (axis 0: x = v,
 * axis 1: y = v) moving up (+1) or down (-1) that axis; -1 if never */
static double helix_plane_psi(const or_helix* h, int axis, double v, int dirn) {
  if (!(h->r > 0.0)) return -1.0;
  double theta;
  if (axis == 0) {
    double w = (v - h->xc) / h->r;
    if (w < -1.0 || w > 1.0) return -1.0;
    double a = asin(w);             /* the branch with cos(theta) >= 0: x increasing */
    theta = dirn > 0 ? a : PI - a;
  } else {
    double w = h->sg * (v - h->yc) / h->r;
    if (w < -1.0 || w > 1.0) return -1.0;
    double a = acos(w);             /* y increasing where sg sin(theta) < 0 */
    theta = dirn > 0 ? -h->sg * a : h->sg * a;
  }
  return helix_turn_to(h, theta);
}

/* Leaving the box [lo, hi] from inside along the helix: the path length to
 * the first face crossed outward (the first axis on ties, as ray_exit),
 * infinity if the helix never leaves it. */
static double helix_exit(const or_helix* h, const double* lo, const double* hi, int* ax, double* face) {
  double s = INFINITY;
  for (int k = 0; k < 3; ++k) {
    double d = INFINITY, f = 0.0;
    if (k < 2) {
      double a = helix_plane_psi(h, k, hi[k], +1);
      double b = helix_plane_psi(h, k, lo[k], -1);
      if (a >= 0.0 && (b < 0.0 || a <= b)) {
        d = a / h->ak;
        f = hi[k];
      } else if (b >= 0.0) {
        d = b / h->ak;
        f = lo[k];
      }
    } else if (h->uz > 0.0) {
      d = (hi[2] - h->z0) / h->uz;
      f = hi[2];
    } else if (h->uz < 0.0) {
      d = (lo[2] - h->z0) / h->uz;
      f = lo[2];
    }
    if (d < 0.0) d = 0.0;
    if (d < s) {
      s = d;
      *ax = k;
      *face = f;
    }
  }
  return s;
}

/* Entering the box [lo, hi] from outside: the smallest path length s in
 * [0, smax] at which the helix crosses one of its face planes inward at a
 * point within the other two bounds (x and y planes are met once per turn
 * in each direction); infinity if none. */
static double helix_entry(const or_helix* h, const double u[3], double kappa, const double* lo,
                          const double* hi, double smax, int* ax, double* face) {
  double best = INFINITY;
  for (int k = 0; k < 3; ++k)
    for (int side = 0; side < 2; ++side) {
      double v = side ? hi[k] : lo[k];
      int dirn = side ? -1 : +1; /* entering through lo moving up, through hi moving down */
      double s0, period;
      if (k < 2) {
        double psi = helix_plane_psi(h, k, v, dirn);
        if (psi < 0.0) continue;
        s0 = psi / h->ak;
        period = 2.0 * PI / h->ak;
      } else {
        if (h->uz == 0.0 || (h->uz > 0.0) != (dirn > 0)) continue;
        s0 = (v - h->z0) / h->uz;
        if (s0 < 0.0) continue;
        period = INFINITY;
      }
      for (double sc = s0; sc <= smax && sc < best; sc += period) {
        double q[3];
        helix_at(h, u, kappa, sc, q);
        q[k] = v;
        int inside = 1;
        for (int j = 0; j < 3; ++j)
          if (j != k && !(q[j] >= lo[j] && q[j] <= hi[j])) inside = 0;
        if (inside) {
          best = sc;
          *ax = k;
          *face = v;
          break;
        }
        if (!(period < INFINITY)) break;
      }
    }
  return best;
}

/* path length along the helix to the next boundary from volume v, searched
 * up to smax (infinity: none within smax): a box's own faces, or from the
 * world the nearer of its exit and the first box entered (boxes win ties,
 * the last such box in index order) */
static double helix_distance(const or_ctx* c, int v, const double p[3], const double u[3], double kappa,
                             double smax, int* ax, double* face) {
  or_helix h = helix_of(p, u, kappa);
  double s;
  if ((uint32_t)v < c->nbox) {
    s = helix_exit(&h, c->blo + 3 * v, c->bhi + 3 * v, ax, face);
  } else {
    s = helix_exit(&h, c->wlo, c->whi, ax, face);
    /* a circle in a plane (u_z = 0) meets what it meets within one turn */
    double lim = smax < s ? smax : s;
    if (h.uz == 0.0 && 2.0 * PI / h.ak < lim) lim = 2.0 * PI / h.ak;
    for (uint32_t b = 0; b < c->nbox; ++b) {
      int a = 0;
      double f = 0.0;
      double d = helix_entry(&h, u, kappa, c->blo + 3 * b, c->bhi + 3 * b, lim, &a, &f);
      if (d <= s) {
        s = d;
        *ax = a;
        *face = f;
      }
    }
  }
  return s <= smax ? s : INFINITY;
}

/* a track leaving the stack: its state at the exit point, in the primary
 * record layout (so that it can be handed back as input) */
static void record_exit(or_event* ev, const or_track* t) {
  if (!ev->exits_n) return;
  uint64_t i = (*ev->exits_n)++;
  if (i >= ev->exits_cap) return;
  or_primary* x = &ev->exits[i];
  x->event = ev->row;
  x->species = (uint32_t)t->species;
  x->ekin_MeV = t->E;
  for (int k = 0; k < 3; ++k) {
    x->pos_mm[k] = t->pos[k];
    x->dir[k] = t->dir[k];
  }
}

/* put the track on the plane it reached (the upper one if up) and enter
 * the next slab; a track that reaches the first or last plane leaves the
 * stack.  On an inner plane the direction decides: a track deflected back
 * (multiple scattering at the step's end) stays in its slab. */
static void cross_z(or_event* ev, or_track* t, int up) {
  or_ctx* c = ev->c;
  t->pos[2] = up ? c->z[t->slab + 1] : c->z[t->slab];
  int next = up ? t->slab + 1 : t->slab - 1;
  int outer = next < 0 || next >= (int)c->n_slabs;
  if (outer || (up ? t->dir[2] > 0.0 : t->dir[2] < 0.0)) t->slab = next;
  if (t->slab < 0 || t->slab >= (int)c->n_slabs) {
    record_exit(ev, t);
    ev->led->escaped[t->species] += t->E;
    t->E = 0.0;
    t->slab = -1;
  }
}
static void escape(or_event* ev, or_track* t) {
  record_exit(ev, t);
  ev->led->escaped[t->species] += t->E;
  t->E = 0.0;
  t->slab = -1;
}
/* box geometry: put the track on the face it reached and find the volume
 * it moves into; reaching the world's surface leaves the geometry */
static void box_cross(or_event* ev, or_track* t, int ax, double face) {
  const or_ctx* c = ev->c;
  t->pos[ax] = face;
  int v = (face == c->wlo[ax] || face == c->whi[ax]) ? -1 : box_locate(c, t->pos, t->dir);
  if (v < 0) escape(ev, t);
  else t->slab = v;
}

static void gamma_step(or_event* ev, or_track* t, or_step_rec* rec) {
  or_ctx* c = ev->c;
  uint32_t mask = c->s.process_mask;
  if (t->E < c->ecut) {
    deposit(ev, t->slab, t->E, rec);
    t->E = 0.0;
    t->slab = -1;
    rec->limiter = OR_L_SUBCUT;
    return;
  }
  uint32_t m = vol_material(c, t->slab);
  double E = t->E;
  double sc = (mask & OR_P_COMPTON) ? xs_lookup(c, m, T_COMPT, E, 0.0) : 0.0;
  double sp = (mask & OR_P_PHOT) ? xs_lookup(c, m, T_PHOT, E, 0.0) : 0.0;
  double sv = (mask & OR_P_CONV) ? xs_lookup(c, m, T_CONV, E, 2.0 * ME) : 0.0;
  double sig = sc + sp + sv;
  int ax = 0;
  double face = 0.0, sz, sw = INFINITY;
  if (c->nbox) {
    sz = box_distance(c, t->slab, t->pos, t->dir, &ax, &face);
  } else {
    sz = dist_z(c, t);
    sw = dist_wall(c, t);
  }
  double sgeom = sz <= sw ? sz : sw;
  or_stream rs = {{ev->key[0], ev->key[1]}, t->id, t->step, 0};
  double u0 = draw(&rs);
  double sphys = sig > 0.0 ? -log(u0) / sig : INFINITY;
  if (sgeom <= sphys) {
    move_straight(t, sgeom);
    rec->step_len = sgeom;
    if (sz <= sw) {
      rec->limiter = OR_L_ZPLANE;
      if (c->nbox) box_cross(ev, t, ax, face);
      else cross_z(ev, t, t->dir[2] > 0.0);
    } else {
      rec->limiter = OR_L_WALL;
      escape(ev, t);
    }
    return;
  }
  move_straight(t, sphys);
  rec->step_len = sphys;
  rec->limiter = OR_L_DISCRETE;
  double r = draw(&rs) * sig;
  or_inter o;
  if (r < sc) {
    rec->process = OR_X_COMPTON;
    sample_compton(E, t->dir, &rs, &o);
  } else if (r < sc + sp) {
    rec->process = OR_X_PHOT;
    sample_photo(E, t->dir, &o);
  } else {
    rec->process = OR_X_CONV;
    sample_pair(pick_element(c, m, 0, E, &rs), E, t->dir, &rs, &o);
    ev->led->n_pair += 1;
  }
  apply(ev, t, &o, rec);
}

/* energy lost by a charged track of kinetic energy T over path s */
static double cont_loss(const or_ctx* c, const double* Rtab, double T, double S,
                        double R, double s) {
  double L;
  if (s >= R) L = T;
  else if (s < c->s.lin_loss_limit * R) L = s * S;
  else L = T - inv_range(c, Rtab, R - s);
  if (T - L < c->ecut) L = T;
  return L;
}

typedef struct {
  int n;
  uint32_t tab[3];
  double th[3];
  int code[3];
} or_proclist;

static or_proclist lepton_procs(const or_ctx* c, int positron) {
  or_proclist p;
  if (!positron) {
    p.n = 2;
    p.tab[0] = T_MOLLER; p.th[0] = 2.0 * c->tcut; p.code[0] = OR_X_MOLLER;
    p.tab[1] = T_BREM;   p.th[1] = c->kcut;       p.code[1] = OR_X_BREM;
  } else {
    p.n = 3;
    p.tab[0] = T_BHABHA; p.th[0] = c->tcut; p.code[0] = OR_X_BHABHA;
    p.tab[1] = T_BREM;   p.th[1] = c->kcut; p.code[1] = OR_X_BREM;
    p.tab[2] = T_ANNIH;  p.th[2] = 0.0;     p.code[2] = OR_X_ANNIH;
  }
  return p;
}

/* total discrete cross section, right-continuous at thresholds (E >= th) */
static double sigtot_upper(const or_ctx* c, uint32_t m, const or_proclist* p, double E) {
  double s = 0.0;
  for (int i = 0; i < p->n; ++i)
    if (E >= p->th[i]) s += plain_lookup(c, m, p->tab[i], E);
  return s;
}

/* maximum of the piecewise log-linear total cross section on [a, b]:
 * endpoints, interior grid nodes, interior thresholds (from above) */
static double sigma_bound(const or_ctx* c, uint32_t m, const or_proclist* p, double a,
                          double b) {
  double best = sigtot_upper(c, m, p, a);
  double v = sigtot_upper(c, m, p, b);
  if (v > best) best = v;
  double xa = (log(a) - c->lnemin) / c->dlog, xb = (log(b) - c->lnemin) / c->dlog;
  int jlo = (int)floor(xa), jhi = (int)ceil(xb);
  if (jlo < 0) jlo = 0;
  if (jhi > (int)c->nb) jhi = (int)c->nb;
  for (int j = jlo; j <= jhi; ++j) {
    double Ej = node_energy(c, j);
    if (!(Ej > a && Ej < b)) continue;
    double s = 0.0;
    for (int i = 0; i < p->n; ++i)
      if (Ej >= p->th[i]) s += tab_ptr(c, m, p->tab[i])[j];
    if (s > best) best = s;
  }
  for (int i = 0; i < p->n; ++i) {
    double th = p->th[i];
    if (th > a && th < b) {
      double s = sigtot_upper(c, m, p, th);
      if (s > best) best = s;
    }
  }
  return best;
}

/* ------------------------------------------------------------------ */
/* Along-step processes of e-/e+ (optional)                            */
/* ------------------------------------------------------------------ */
/* their draws sit far above any sampler's, so switching them on leaves the
 * other draws of a step where they are */
enum { OR_DRAW_MSC = 1u << 16, OR_DRAW_FLUCT = (1u << 16) + 8u, OR_FLUCT_TRIALS = 16 };

/* Highland's width of the projected angle after a path s (PDG RPP,
 * multiple scattering through small angles), unit charge; zero where the
 * logarithmic correction would make it negative */
static double highland(double T, double s, double x0) {
  double p = sqrt(T * (T + 2.0 * ME));
  double beta = p / (T + ME);
  double r = s / x0;
  double corr = 1.0 + 0.038 * log(r / (beta * beta));
  if (!(corr > 0.0)) return 0.0;
  return 13.6 / (beta * p) * sqrt(r) * corr;
}

/* Gaussian multiple scattering: the plane angles are independent normal
 * with width theta_0, so the space angle is theta_0 sqrt(-2 ln u1) and the
 * azimuth 2 pi u2 (capped at pi) */
static void msc_deflect(double theta0, const or_stream* as, double dir[3]) {
  double u1 = draw_at(as, OR_DRAW_MSC), u2 = draw_at(as, OR_DRAW_MSC + 1);
  if (!(theta0 > 0.0)) return;
  double th = theta0 * sqrt(-2.0 * log(u1));
  if (th > PI) th = PI;
  double out[3];
  rotate_to(dir, sin(th), cos(th), 2.0 * PI * u2, out);
  for (int i = 0; i < 3; ++i) dir[i] = out[i];
}

/* variance of the restricted loss over a path s: the second moment of the
 * sub-cut delta-ray spectrum for the spin-0 Bethe cross section,
 * n_el s (2 pi r_e^2 m_e / beta^2) (W_up - beta^2 W_up^2 / (2 W_max)),
 * W_max = T/2 (e-) or T (e+), W_up = min(cut, W_max) */
static double fluct_var(const or_mat* m, double cut, double T, double s, int positron) {
  double g = T / ME + 1.0, b2 = 1.0 - 1.0 / (g * g);
  double wmax = positron ? T : 0.5 * T;
  double wup = cut < wmax ? cut : wmax;
  return m->n_el * s * 2.0 * PI * RE * RE * ME / b2 * (wup - b2 * wup * wup / (2.0 * wmax));
}

/* loss drawn from the gamma distribution with the given mean and variance:
 * Marsaglia and Tsang's method (2000) with shape k (raised by one and the
 * result scaled by u^(1/k) when k < 1), at most OR_FLUCT_TRIALS trials of
 * three draws each (after them: the mode d of the raised shape) */
static double gamma_loss(double mean, double var, const or_stream* fs) {
  double k = mean * mean / var, theta = var / mean;
  double kk = k < 1.0 ? k + 1.0 : k;
  double d = kk - 1.0 / 3.0, cc = 1.0 / sqrt(9.0 * d);
  double x = d;
  for (uint32_t i = 0; i < OR_FLUCT_TRIALS; ++i) {
    double u1 = draw_at(fs, OR_DRAW_FLUCT + 3 * i), u2 = draw_at(fs, OR_DRAW_FLUCT + 3 * i + 1);
    double u3 = draw_at(fs, OR_DRAW_FLUCT + 3 * i + 2);
    double z = sqrt(-2.0 * log(u1)) * cos(2.0 * PI * u2);
    double v = 1.0 + cc * z;
    if (v <= 0.0) continue;
    v = v * v * v;
    if (log(u3) < 0.5 * z * z + d - d * v + d * log(v)) {
      x = d * v;
      break;
    }
  }
  if (k < 1.0) x *= pow(draw_at(fs, OR_DRAW_FLUCT + 3 * OR_FLUCT_TRIALS), 1.0 / k);
  return x * theta;
}

static void lepton_step(or_event* ev, or_track* t, or_step_rec* rec) {
  or_ctx* c = ev->c;
  int positron = (t->species == OR_POSITRON);
  uint32_t mask = c->s.process_mask;
  int cont = (mask & OR_P_CONT) != 0;
  int fluct = cont && (mask & OR_P_FLUCT) != 0;
  int msc = (mask & OR_P_MSC) != 0;
  or_stream rs = {{ev->key[0], ev->key[1]}, t->id, t->step, 0};
  or_inter o;
  double T = t->E;

  /* below the tracking cut: deposit; a positron then annihilates at rest */
  if (T < c->ecut) {
    deposit(ev, t->slab, T, rec);
    rec->limiter = OR_L_SUBCUT;
    t->E = 0.0;
    if (positron) {
      rec->process = OR_X_ANNIH_REST;
      annih_at_rest(&rs, &o);
      ev->led->n_annih += 1;
      apply(ev, t, &o, rec);
    }
    t->slab = -1;
    return;
  }

  int field = (c->s.bz_tesla != 0.0);
  int ax = 0;
  double face = 0.0;
  uint32_t m = vol_material(c, t->slab);
  const double* Rtab = tab_ptr(c, m, positron ? T_R_EP : T_R_EM);
  double S = 0.0, R = INFINITY, scont = INFINITY;
  if (cont) {
    S = plain_lookup(c, m, positron ? T_S_EP : T_S_EM, T);
    R = plain_lookup(c, m, positron ? T_R_EP : T_R_EM, T);
    double rho = c->s.final_range_mm, al = c->s.dr_over_range;
    scont = (R <= rho) ? R : al * R + rho * (1.0 - al) * (2.0 - rho / R);
  }
  double sgeom, sw = INFINITY, dw = INFINITY;
  int zlimited;
  if (c->nbox && field) {
    /* along the helix, searched up to the continuous-loss limit (beyond it
     * the boundary cannot limit the step) */
    double kappa = (positron ? 1.0 : -1.0) * KB * c->s.bz_tesla / sqrt(T * (T + 2.0 * ME));
    sgeom = helix_distance(c, t->slab, t->pos, t->dir, kappa, scont, &ax, &face);
    zlimited = 1;
    if (!(sgeom < INFINITY) && !(scont < INFINITY)) {
      /* nothing limits the step (no continuous loss, a circle that meets no
       * boundary): one turn, without a crossing */
      sgeom = 2.0 * PI / fabs(kappa);
      zlimited = 0;
    }
  } else if (field) {
    double sz = dist_z(c, t);
    double ax = fabs(t->pos[0]), ay = fabs(t->pos[1]);
    dw = c->s.half_xy_mm - (ax > ay ? ax : ay);
    if (dw < OR_SAFETY_EPS) {
      rec->limiter = OR_L_ESCAPE_SAFETY;
      escape(ev, t);
      return;
    }
    sgeom = sz <= dw ? sz : dw;
    zlimited = (sz <= dw);
  } else {
    double sz = c->nbox ? box_distance(c, t->slab, t->pos, t->dir, &ax, &face) : dist_z(c, t);
    if (!c->nbox) sw = dist_wall(c, t);
    sgeom = sz <= sw ? sz : sw;
    zlimited = (sz <= sw);
  }
  double smax = scont <= sgeom ? scont : sgeom;

  /* lowest energy reachable over [0, smax] and the thinning bound */
  double elo = T;
  if (cont) {
    elo = T - cont_loss(c, Rtab, T, S, R, smax);
    double lin = c->s.lin_loss_limit * R;
    if (smax >= lin) {
      double e2 = T - lin * S;
      if (e2 < elo) elo = e2;
    }
  }
  /* with fluctuations any energy down to the cut is reachable */
  double a = (elo > c->ecut && !fluct) ? elo : c->ecut;
  or_proclist pl = lepton_procs(c, positron);
  double bound = sigma_bound(c, m, &pl, a, T);

  double u0 = draw(&rs);
  double sphys = bound > 0.0 ? -log(u0) / bound : INFINITY;
  int lim;
  double s;
  if (sphys < smax) {
    s = sphys;
    lim = OR_L_DISCRETE;
  } else if (sgeom <= scont) {
    s = sgeom;
    lim = zlimited ? OR_L_ZPLANE : (field ? OR_L_SAFETY : OR_L_WALL);
  } else {
    s = scont;
    lim = OR_L_CONT;
  }

  /* propagate */
  if (field) {
    double p = sqrt(T * (T + 2.0 * ME));
    double q = positron ? 1.0 : -1.0;
    double kappa = q * KB * c->s.bz_tesla / p;
    move_helix(t, kappa, s);
  } else {
    move_straight(t, s);
  }
  rec->step_len = s;
  ev->led->charged_len += s;

  /* continuous loss in the slab the step was taken in */
  double dE = cont ? cont_loss(c, Rtab, T, S, R, s) : 0.0;
  if (fluct && dE > 0.0 && dE < T) {
    double var = fluct_var(&c->mat[m], c->tcut, T, s, positron);
    if (var > 0.0) {
      dE = gamma_loss(dE, var, &rs);
      if (dE > T) dE = T;
    }
  }
  deposit(ev, t->slab, dE, rec);
  double Tp = T - dE;
  t->E = Tp;
  rec->limiter = (uint32_t)lim;

  if (Tp == 0.0) {
    rec->limiter = OR_L_STOPPED;
    if (positron) {
      rec->process = OR_X_ANNIH_REST;
      annih_at_rest(&rs, &o);
      ev->led->n_annih += 1;
      apply(ev, t, &o, rec);
    }
    t->slab = -1;
    return;
  }
  /* the plane reached is fixed before any deflection */
  int up = t->dir[2] > 0.0;
  if (msc && s > 0.0) msc_deflect(highland(T, s, c->mat[m].x0), &rs, t->dir);
  if (lim == OR_L_ZPLANE) {
    if (c->nbox) box_cross(ev, t, ax, face);
    else cross_z(ev, t, up);
    return;
  }
  if (lim == OR_L_WALL) {
    escape(ev, t);
    return;
  }
  if (lim != OR_L_DISCRETE) return;

  /* discrete candidate at the post-step energy: accept or null */
  double r = draw(&rs) * bound;
  double cum = 0.0;
  int chosen = -1;
  for (int i = 0; i < pl.n; ++i) {
    cum += xs_lookup(c, m, pl.tab[i], Tp, pl.th[i]);
    if (r < cum) {
      chosen = i;
      break;
    }
  }
  if (chosen < 0) {
    rec->process = OR_X_NULL;
    ev->led->n_null += 1;
    return;
  }
  rec->process = (uint32_t)pl.code[chosen];
  switch (pl.code[chosen]) {
    case OR_X_MOLLER: sample_moller(Tp, c->tcut, t->dir, &rs, &o); break;
    case OR_X_BHABHA: sample_bhabha(Tp, c->tcut, t->dir, &rs, &o); break;
    case OR_X_BREM: sample_brem(pick_element(c, m, 1, Tp, &rs), Tp, c->kcut, t->dir, &rs, &o); break;
    default:
      sample_annih(Tp, t->dir, &rs, &o);
      ev->led->n_annih += 1;
      break;
  }
  apply(ev, t, &o, rec);
}

/* one step of track t: dispatch, then step counter, log and watchdog */
static void step_track(or_event* ev, or_track* t) {
  or_step_rec rec;
  memset(&rec, 0, sizeof rec);
  rec.event = t->event;
  rec.species = (uint32_t)t->species;
  rec.id = t->id;
  rec.step = t->step;
  rec.e_before = t->E;
  if (ev->profile) {
    uint64_t it = (uint64_t)t->birth + t->step;
    if (it < ev->profile_cap) ev->profile[it * 3 + (uint64_t)t->species] += 1;
    if (it + 1 > *ev->profile_len) *ev->profile_len = (uint32_t)(it + 1);
  }
  if (t->species == OR_GAMMA) gamma_step(ev, t, &rec);
  else lepton_step(ev, t, &rec);
  t->step += 1;
  ev->led->n_steps += 1;
  if (t->slab >= 0 && t->step >= ev->c->s.max_steps_per_track) {
    ev->led->killed += t->E;
    t->E = 0.0;
    t->slab = -1;
  }
  rec.slab_after = t->slab;
  rec.e_after = t->E;
  for (int i = 0; i < 3; ++i) rec.pos_after[i] = t->pos[i];
  if (ev->log) {
    if (*ev->log_n < ev->log_cap) ev->log[*ev->log_n] = rec;
  }
  if (ev->log_n) *ev->log_n += 1;
}

/* slab containing z; a point on a plane belongs to the slab it enters */
static int locate(const or_ctx* c, double z, double uz) {
  int k = -1;
  for (uint32_t i = 0; i < c->n_slabs; ++i)
    if (z >= c->z[i] && z < c->z[i + 1]) k = (int)i;
  if (z == c->z[c->n_slabs]) k = (int)c->n_slabs - 1;
  if (k > 0 && z == c->z[k] && uz < 0.0) k -= 1;
  return k;
}

/* ------------------------------------------------------------------ */
/* API                                                                 */
/* ------------------------------------------------------------------ */
/* tables and physics constants (everything but the geometry) */
static int create_common(const or_setup* s, or_ctx** out) {
  if (!s || !out || s->n_materials == 0 || s->n_bins < 2) return -1;
  or_ctx* c = (or_ctx*)calloc(1, sizeof(or_ctx));
  if (!c) return -2;
  c->s = *s;
  c->n_mat = s->n_materials;
  c->nb = s->n_bins;
  c->mat = (or_mat*)malloc(sizeof(or_mat) * s->n_materials);
  c->el = (or_mat*)calloc((size_t)s->n_materials * OR_MAX_EL, sizeof(or_mat));
  c->n_el = (uint32_t*)calloc(s->n_materials, sizeof(uint32_t));
  c->tab = (double*)calloc((size_t)s->n_materials * OR_N_TABLES * (s->n_bins + 1), sizeof(double));
  c->eltab = (double*)calloc((size_t)s->n_materials * OR_MAX_EL * 2 * (s->n_bins + 1), sizeof(double));
  if (!c->mat || !c->el || !c->n_el || !c->tab || !c->eltab) {
    or_destroy(c);
    return -2;
  }
  c->s.z_mm = NULL;
  c->s.material = NULL;
  c->s.materials = NULL;
  for (uint32_t i = 0; i < s->n_materials; ++i)
    derive_material_el(&s->materials[i], &c->mat[i], &c->el[(size_t)i * OR_MAX_EL], &c->n_el[i]);
  c->lnemin = log(s->emin_MeV);
  c->dlog = (log(s->emax_MeV) - log(s->emin_MeV)) / s->n_bins;
  c->ecut = s->emin_MeV;
  c->tcut = s->electron_cut_MeV;
  c->kcut = s->gamma_cut_MeV;
  build_tables(c);
  *out = c;
  return 0;
}

int or_create(const or_setup* s, or_ctx** out) {
  if (!s || !out || s->n_slabs == 0) return -1;
  for (uint32_t i = 0; i < s->n_slabs; ++i) {
    if (!(s->z_mm[i + 1] > s->z_mm[i])) return -1;
    if (s->material[i] >= s->n_materials) return -1;
  }
  or_ctx* c;
  int rc = create_common(s, &c);
  if (rc) return rc;
  c->n_slabs = s->n_slabs;
  c->n_cols = s->n_slabs;
  c->z = (double*)malloc(sizeof(double) * (s->n_slabs + 1));
  c->slab_mat = (uint32_t*)malloc(sizeof(uint32_t) * s->n_slabs);
  if (!c->z || !c->slab_mat) {
    or_destroy(c);
    return -2;
  }
  memcpy(c->z, s->z_mm, sizeof(double) * (s->n_slabs + 1));
  memcpy(c->slab_mat, s->material, sizeof(uint32_t) * s->n_slabs);
  c->s.z_mm = c->z;
  c->s.material = c->slab_mat;
  *out = c;
  return 0;
}

int or_create_boxes(const or_setup* s, const or_boxes* b, or_ctx** out) {
  if (!s || !b || !out || b->n_boxes == 0 || !b->lo || !b->hi || !b->material) return -1;
  if (b->world_material >= s->n_materials) return -1;
  for (int k = 0; k < 3; ++k)
    if (!(b->world_lo[k] < b->world_hi[k])) return -1;
  for (uint32_t i = 0; i < b->n_boxes; ++i) {
    const double *lo = b->lo + 3 * i, *hi = b->hi + 3 * i;
    if (b->material[i] >= s->n_materials) return -1;
    for (int k = 0; k < 3; ++k)
      if (!(lo[k] < hi[k]) || lo[k] < b->world_lo[k] || hi[k] > b->world_hi[k]) return -1;
  }
  /* no two boxes share interior points */
  for (uint32_t i = 0; i < b->n_boxes; ++i)
    for (uint32_t j = i + 1; j < b->n_boxes; ++j) {
      int apart = 0;
      for (int k = 0; k < 3; ++k)
        if (b->hi[3 * i + k] <= b->lo[3 * j + k] || b->hi[3 * j + k] <= b->lo[3 * i + k]) apart = 1;
      if (!apart) return -1;
    }
  or_ctx* c;
  int rc = create_common(s, &c);
  if (rc) return rc;
  c->nbox = b->n_boxes;
  c->n_cols = b->n_boxes + 1;
  c->blo = (double*)malloc(sizeof(double) * 3 * b->n_boxes);
  c->bhi = (double*)malloc(sizeof(double) * 3 * b->n_boxes);
  c->bmat = (uint32_t*)malloc(sizeof(uint32_t) * b->n_boxes);
  if (!c->blo || !c->bhi || !c->bmat) {
    or_destroy(c);
    return -2;
  }
  memcpy(c->blo, b->lo, sizeof(double) * 3 * b->n_boxes);
  memcpy(c->bhi, b->hi, sizeof(double) * 3 * b->n_boxes);
  memcpy(c->bmat, b->material, sizeof(uint32_t) * b->n_boxes);
  for (int k = 0; k < 3; ++k) {
    c->wlo[k] = b->world_lo[k];
    c->whi[k] = b->world_hi[k];
  }
  c->wmat = b->world_material;
  *out = c;
  return 0;
}

int or_geo_locate(const or_ctx* c, const double p[3], const double u[3]) {
  if (!c || !c->nbox) return -1;
  return box_locate(c, p, u);
}

double or_geo_distance(const or_ctx* c, int v, const double p[3], const double u[3], int* axis,
                       double* face) {
  if (!c || !c->nbox || v < 0 || (uint32_t)v > c->nbox || !axis || !face) return NAN;
  *axis = -1;
  *face = NAN;
  return box_distance(c, v, p, u, axis, face);
}
double or_geo_helix_distance(const or_ctx* c, int v, const double p[3], const double u[3], double kappa,
                             double smax, int* axis, double* face) {
  if (!c || !c->nbox || v < 0 || (uint32_t)v > c->nbox || !axis || !face || kappa == 0.0) return NAN;
  *axis = -1;
  *face = NAN;
  return helix_distance(c, v, p, u, kappa, smax, axis, face);
}
void or_destroy(or_ctx* c) {
  if (!c) return;
  free(c->z);
  free(c->slab_mat);
  free(c->blo);
  free(c->bhi);
  free(c->bmat);
  free(c->mat);
  free(c->el);
  free(c->n_el);
  free(c->tab);
  free(c->eltab);
  free(c);
}

int or_run(or_ctx* c, const or_primary* prim, uint64_t n_prim, uint32_t n_events,
           const uint32_t* event_keys, double* edep, or_ledger* ledger,
           or_step_rec* log, uint64_t log_cap, uint64_t* log_n, uint64_t* profile,
           uint32_t profile_cap, uint32_t* profile_len, int stack_order) {
  return or_run_exits(c, prim, n_prim, n_events, event_keys, edep, ledger, log, log_cap, log_n, profile,
                      profile_cap, profile_len, stack_order, NULL, 0, NULL);
}

int or_run_exits(or_ctx* c, const or_primary* prim, uint64_t n_prim, uint32_t n_events,
                 const uint32_t* event_keys, double* edep, or_ledger* ledger,
                 or_step_rec* log, uint64_t log_cap, uint64_t* log_n, uint64_t* profile,
                 uint32_t profile_cap, uint32_t* profile_len, int stack_order,
                 or_primary* exits, uint64_t exits_cap, uint64_t* exits_n) {
  if (!c || (!prim && n_prim) || !edep || !ledger) return -1;
  uint64_t dummy_n = 0;
  uint32_t dummy_len = 0;
  if (!log_n) log_n = &dummy_n;
  if (!profile_len) profile_len = &dummy_len;
  /* validate everything before transporting anything */
  for (uint64_t i = 0; i < n_prim; ++i) {
    const or_primary* p = &prim[i];
    double n2 = p->dir[0] * p->dir[0] + p->dir[1] * p->dir[1] + p->dir[2] * p->dir[2];
    if (p->event >= n_events || p->species > OR_POSITRON || !(p->ekin_MeV > 0.0) || !(n2 > 0.0))
      return -1;
    if (c->nbox) {
      if (box_locate(c, p->pos_mm, p->dir) < 0) return -1;
    } else if (!(p->pos_mm[2] >= c->z[0] && p->pos_mm[2] <= c->z[c->n_slabs]) ||
               !(fabs(p->pos_mm[0]) <= c->s.half_xy_mm) || !(fabs(p->pos_mm[1]) <= c->s.half_xy_mm)) {
      return -1;
    }
  }
  or_stack st = {NULL, 0, 0, 0};
  uint64_t* count = (uint64_t*)calloc(n_events ? n_events : 1, sizeof(uint64_t));
  uint64_t* first = (uint64_t*)calloc((size_t)n_events + 1, sizeof(uint64_t));
  uint64_t* order = (uint64_t*)malloc((n_prim ? n_prim : 1) * sizeof(uint64_t));
  if (!count || !first || !order) {
    free(count); free(first); free(order);
    return -2;
  }
  /* stable grouping of the primaries by event (counting sort) */
  for (uint64_t i = 0; i < n_prim; ++i) first[prim[i].event + 1] += 1;
  for (uint32_t e = 0; e < n_events; ++e) first[e + 1] += first[e];
  for (uint64_t i = 0; i < n_prim; ++i) order[first[prim[i].event] + count[prim[i].event]++] = i;
  memset(count, 0, sizeof(uint64_t) * (n_events ? n_events : 1));
  int err = 0;
  for (uint32_t e = 0; e < n_events && !err; ++e) {
    or_event ev;
    memset(&ev, 0, sizeof ev);
    ev.c = c;
    ev.key[0] = c->s.seed;
    ev.key[1] = event_keys ? event_keys[e] : e;
    ev.row = e;
    ev.edep = edep + (size_t)e * c->n_cols;
    ev.led = &ledger[e];
    ev.log = log;
    ev.log_cap = log_cap;
    ev.log_n = log_n;
    ev.profile = profile;
    ev.profile_cap = profile_cap;
    ev.profile_len = profile_len;
    ev.exits = exits;
    ev.exits_cap = exits_cap;
    ev.exits_n = exits_n;
    ev.st = &st;
    st.n = 0;
    st.head = 0;
    /* primaries of this event: id = running index within the event */
    for (uint64_t q = first[e]; q < first[e + 1]; ++q) {
      const or_primary* p = &prim[order[q]];
      or_track t;
      t.species = (int)p->species;
      t.E = p->ekin_MeV;
      double n = sqrt(p->dir[0] * p->dir[0] + p->dir[1] * p->dir[1] + p->dir[2] * p->dir[2]);
      for (int k = 0; k < 3; ++k) {
        t.pos[k] = p->pos_mm[k];
        t.dir[k] = p->dir[k] / n;
      }
      t.slab = c->nbox ? box_locate(c, t.pos, t.dir) : locate(c, t.pos[2], t.dir[2]);
      t.event = e;
      t.id = count[e]++;
      t.step = 0;
      t.birth = 0;
      if (stack_push(&st, &t)) err = -2;
    }
    while (!err && st.n > st.head) {
      or_track t;
      if (stack_order == 0) {
        t = st.v[--st.n];
      } else {
        t = st.v[st.head++];
      }
      while (t.slab >= 0) step_track(&ev, &t);
      if (ev.err) err = ev.err;
      if (stack_order != 0 && st.head == st.n) st.head = st.n = 0;
    }
  }
  free(st.v);
  free(count);
  free(first);
  free(order);
  return err;
}

uint64_t or_table_count(const or_ctx* c) {
  return (uint64_t)c->n_mat * OR_N_TABLES * (c->nb + 1);
}

int or_export_tables(const or_ctx* c, double* out, uint64_t n) {
  uint64_t need = or_table_count(c);
  if (n < need) return -1;
  memcpy(out, c->tab, need * sizeof(double));
  return 0;
}

double or_table_lookup(const or_ctx* c, uint32_t m, uint32_t t, double E) {
  return plain_lookup(c, m, t, E);
}

double or_inverse_range(const or_ctx* c, uint32_t m, uint32_t species, double r) {
  return inv_range(c, tab_ptr(c, m, species == OR_POSITRON ? T_R_EP : T_R_EM), r);
}

double or_sigma_bound(const or_ctx* c, uint32_t m, uint32_t species, double a, double b) {
  or_proclist pl = lepton_procs(c, species == OR_POSITRON);
  return sigma_bound(c, m, &pl, a, b);
}

double or_sigma_total(const or_ctx* c, uint32_t m, uint32_t species, double E) {
  or_proclist pl = lepton_procs(c, species == OR_POSITRON);
  return sigtot_upper(c, m, &pl, E);
}

double or_formula(int which, const or_material* in, double cut, double E, double arg2) {
  or_mat m;
  derive_material(in, &m);
  switch (which) {
    case OR_F_SIGMA_KN: return xs_compton(E);
    case OR_F_SIGMA_PE: return xs_photo(&m, E);
    case OR_F_SIGMA_PAIR: return xs_pair(&m, E);
    case OR_F_DSDE_PAIR: return pair_pref(&m) * pair_F(&m, E, arg2);
    case OR_F_SIGMA_BREM: return xs_brem(&m, E, cut);
    case OR_F_DSDK_BREM: return pair_pref(&m) * brem_brace(&m, E, arg2) / arg2;
    case OR_F_SBREM: return sbrem(&m, E, cut);
    case OR_F_SIGMA_MOLLER: return xs_moller(E, cut);
    case OR_F_DSDE_MOLLER: return dsde_moller(E, arg2);
    case OR_F_SIGMA_BHABHA: return xs_bhabha(E, cut);
    case OR_F_DSDE_BHABHA: return dsde_bhabha(E, arg2);
    case OR_F_SION_E: return sion(&m, E, cut, 0);
    case OR_F_SION_P: return sion(&m, E, cut, 1);
    case OR_F_SIGMA_ANNIH: return xs_annih(E);
    case OR_F_DSDE_COMPTON: return dsde_compton(E, arg2);
    case OR_F_PAIR_FMAX: return pair_Fmax(&m, E);
    case OR_F_PAIR_F: return pair_F(&m, E, arg2);
    case OR_F_BREM_BOUND: return brem_bound(&m, E, cut);
    case OR_F_BREM_F: return brem_brace(&m, E, arg2);
    case OR_F_X0: return m.x0;
    case OR_F_HIGHLAND: return highland(E, arg2, m.x0);
    case OR_F_FLUCT_VAR_E: return fluct_var(&m, cut, E, arg2, 0);
    case OR_F_FLUCT_VAR_P: return fluct_var(&m, cut, E, arg2, 1);
    default: return NAN;
  }
}

int or_sample(const or_ctx* c, int which, uint32_t material, double E, const double dir[3],
              const uint32_t key[2], uint64_t id, uint32_t step, double* out) {
  if (!c || material >= c->n_mat || !out) return -1;
  or_stream rs = {{key[0], key[1]}, id, step, 2};
  double u[3] = {dir[0], dir[1], dir[2]};
  normalise(u);
  or_inter o;
  memset(&o, 0, sizeof o);
  const or_mat* el0 = &c->el[(size_t)material * OR_MAX_EL];
  const or_mat* m = el0;
  switch (which) {
    case 0: sample_compton(E, u, &rs, &o); break;
    case 1:
      if (E <= 2.0 * ME) return -1;
      m = pick_element(c, material, 0, E, &rs);
      sample_pair(m, E, u, &rs, &o);
      break;
    case 2:
      if (E <= c->kcut) return -1;
      m = pick_element(c, material, 1, E, &rs);
      sample_brem(m, E, c->kcut, u, &rs, &o);
      break;
    case 3:
      if (E <= 2.0 * c->tcut) return -1;
      sample_moller(E, c->tcut, u, &rs, &o);
      break;
    case 4:
      if (E <= c->tcut) return -1;
      sample_bhabha(E, c->tcut, u, &rs, &o);
      break;
    case 5: sample_annih(E, u, &rs, &o); break;
    default: return -1;
  }
  for (int i = 0; i < 16; ++i) out[i] = 0.0;
  out[0] = o.var;
  out[1] = o.trials;
  out[2] = o.parent_alive ? o.parent_E : -1.0;
  for (int i = 0; i < 3; ++i) out[3 + i] = o.parent_dir[i];
  out[6] = o.n_sec > 0 ? o.sec_E[0] : -1.0;
  for (int i = 0; i < 3; ++i) out[7 + i] = o.sec_dir[0][i];
  out[10] = o.n_sec > 1 ? o.sec_E[1] : -1.0;
  for (int i = 0; i < 3; ++i) out[11 + i] = o.sec_dir[1][i];
  out[15] = (double)(m - el0);
  return 0;
}

int or_sample_along(const or_ctx* c, int which, uint32_t material, double T, double s, double mean,
                    const double dir[3], const uint32_t key[2], uint64_t id, uint32_t step, double* out) {
  if (!c || material >= c->n_mat || !out || !(T > 0.0) || !(s >= 0.0)) return -1;
  or_stream rs = {{key[0], key[1]}, id, step, 0};
  const or_mat* m = &c->mat[material];
  for (int i = 0; i < 4; ++i) out[i] = 0.0;
  if (which == 0) {
    double u[3] = {dir[0], dir[1], dir[2]};
    normalise(u);
    out[0] = highland(T, s, m->x0);
    msc_deflect(out[0], &rs, u);
    for (int i = 0; i < 3; ++i) out[1 + i] = u[i];
    return 0;
  }
  if (which == 1 || which == 2) {
    if (!(mean > 0.0)) return -1;
    out[1] = fluct_var(m, c->tcut, T, s, which == 2);
    out[0] = out[1] > 0.0 ? gamma_loss(mean, out[1], &rs) : mean;
    return 0;
  }
  return -1;
}
