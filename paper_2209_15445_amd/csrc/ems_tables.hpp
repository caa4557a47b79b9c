// ems_tables.hpp -- host-built log-energy tables and their device layout.
//
// The paper copies its physics data to the GPU once, at initialisation
// (section 2.2).  Here the host builds, per material, 13 tables on the grid
// E_j = E_min exp(j D), j = 0..n_bins, interpolated linearly in ln E; the step
// kernel stages them into LDS.
#pragma once
#include <stdint.h>

#include <vector>

#include "ems_models.hpp"

namespace ems {

// table ids (the first 11 are the exported ones)
enum : int {
  tCompt = 0, tPhot = 1, tConv = 2, tSem = 3, tRem = 4, tMoller = 5, tBrem = 6,
  tSep = 7, tRep = 8, tBhabha = 9, tAnnih = 10,
  tPMem = 11,  // running max over nodes <= E_j of the e- discrete total
  tPMep = 12,  // same for e+
  kNumTables = 13, kNumExport = 11,
  // device layout only (derived when the tables are packed): the e- and e+
  // discrete totals at the nodes, summed over the processes in the order
  // and arithmetic type of the step code
  tSumEm = 13, tSumEp = 14, kNumDevTables = 15
};

struct MaterialIn {
  double Z, A, rho, I_eV;
  uint32_t n_el;  // 0: the single element (Z, A); else a compound of n_el elements
  double el_Z[kMaxElements], el_A[kMaxElements], el_atoms[kMaxElements];
};

struct MatFull {
  double Z, nat, nel, I, plasma;
  MatRT rt;
};

// A material as a whole (electron density, I, plasma energy; the screening
// constants of its first element) and its elements, each with its own atom
// density and screening constants.
struct MatSet {
  MatFull bulk;
  uint32_t n;
  MatFull el[kMaxElements];
};

MatSet derive_material(const MaterialIn& in);

struct TableParams {
  uint32_t n_bins;
  double emin, emax;
  double gamma_cut, electron_cut;
  uint32_t process_mask;
};

// tables[(m * kNumTables + t) * (n_bins + 1) + j]; per-element partial pair
// (w = 0) and bremsstrahlung (w = 1) totals el[((m * kMaxElements + i) * 2 +
// w) * nodes + j] (zero beyond a material's elements) and the elements'
// screening constants elc[(m * kMaxElements + i) * 2 + {0: c136, 1: gshift}]
struct TableSet {
  uint32_t n_mat = 0, nodes = 0;
  double lnemin = 0, dlog = 0;
  std::vector<double> v, el, elc;
  std::vector<MatRT> rt;
  double at(uint32_t m, int t, uint32_t j) const { return v[((size_t)m * kNumTables + t) * nodes + j]; }
};

TableSet build_tables(const TableParams& p, const std::vector<MaterialIn>& mats);

// host-side cross sections (per atom / per electron), exposed for tests
double kn_sigma(double E);
double photo_sigma(const MatFull& m, double E);
double pair_sigma(const MatFull& m, double E);
double brem_sigma(const MatFull& m, double T, double kc);
double brem_loss(const MatFull& m, double T, double kc);
double moller_sigma(double T, double tcut);
double bhabha_sigma(double T, double tcut);
double ion_loss(const MatFull& m, double T, double tcut, bool positron);
double heitler_sigma(double T);

}  // namespace ems
