/*
 * ems_oracle.h -- plain, slow, single-threaded FP64 CPU oracle for the
 * electromagnetic-shower transport loop of "Offloading electromagnetic shower
 * transport to GPUs" (AdePT, ACAT 2021).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  The GPU product path
 * never links, loads or calls it, and this code shares nothing (headers,
 * helpers, tables, constants) with the GPU library.
 *
 * What it computes: for each event, every track is transported to completion
 * one step at a time, depth first, secondaries kept on a stack -- the CPU model
 * the paper describes in its "Stepping workflow" section (one thread follows
 * one track, secondaries are pushed on a stack, events are independent).
 * The paper delegates physics to G4HepEm (section 2.2) and gives no formulas;
 * the physics below is a set of textbook models: Klein-Nishina Compton,
 * Heitler K-shell photo-effect, Bethe-Heitler pair production with
 * Thomas-Fermi screening, screened 1/k bremsstrahlung, Moller/Bhabha
 * ionisation with restricted Berger-Seltzer loss, Heitler two-photon
 * annihilation; optionally Highland-width multiple scattering and gamma-law
 * loss fluctuations; compounds by Bragg additivity with a sampled target
 * element.  Geometry is a slab stack or a set of boxes navigated by brute
 * force.  Every random number is addressed by
 * (seed, event key, track id, step, draw index) through Philox4x32-10, so a
 * breadth-first GPU loop that uses the same addressing reaches the same
 * per-track histories.
 *
 * Units: MeV, mm, tesla.  All arithmetic in IEEE double, built with
 * -O2 -ffp-contract=off (no fused multiply-add, no fast-math).
 */
#ifndef EMS_ORACLE_H
#define EMS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_GAMMA = 0, OR_ELECTRON = 1, OR_POSITRON = 2 };

/* process mask bits */
enum {
  OR_P_COMPTON = 1u << 0, OR_P_PHOT = 1u << 1, OR_P_CONV = 1u << 2,
  OR_P_EIONI = 1u << 3,   /* Moller (e-) / Bhabha (e+) delta rays      */
  OR_P_EBREM = 1u << 4,   /* discrete bremsstrahlung above the cut     */
  OR_P_ANNIH = 1u << 5,   /* e+ annihilation in flight                 */
  OR_P_CONT = 1u << 6,    /* continuous (restricted) energy loss       */
  OR_P_ALL = 0x7fu,
  /* optional along-step processes of e-/e+ (not in OR_P_ALL):            */
  OR_P_MSC = 1u << 7,     /* multiple Coulomb scattering: Gaussian
                             deflection with the Highland width at the end
                             of every charged step                        */
  OR_P_FLUCT = 1u << 8    /* fluctuations of the restricted loss: gamma
                             distribution with the step's mean loss and the
                             Bethe second moment of the sub-cut delta rays
                             (needs OR_P_CONT)                            */
};

/* limiter codes written to the step log */
enum {
  OR_L_ZPLANE = 0,   /* step ended on a z plane (slab change or escape)   */
  OR_L_WALL = 1,     /* straight step ended on a transverse wall: escape  */
  OR_L_SAFETY = 2,   /* helix step limited by the transverse safety       */
  OR_L_CONT = 3,     /* charged step limited by the step function         */
  OR_L_DISCRETE = 4, /* discrete interaction point reached                */
  OR_L_STOPPED = 5,  /* charged track ranged out inside the step          */
  OR_L_SUBCUT = 6,   /* track below the tracking cut at step start        */
  OR_L_ESCAPE_SAFETY = 7 /* helix track closer than 1e-6 mm to a wall     */
};
/* process codes written to the step log */
enum {
  OR_X_NONE = 0, OR_X_COMPTON = 1, OR_X_PHOT = 2, OR_X_CONV = 3,
  OR_X_MOLLER = 4, OR_X_BHABHA = 5, OR_X_BREM = 6, OR_X_ANNIH = 7,
  OR_X_ANNIH_REST = 8, OR_X_NULL = 9
};

/* A material: one element (n_elements = 0: Z, A_g_mol) or a compound of
 * 1..4 elements with el_atoms atoms of element i per formula unit (Z and
 * A_g_mol are then not used); density and mean excitation energy are the
 * material's.  In a compound, per-atom cross sections (photo-effect, pair,
 * bremsstrahlung and its sub-cut loss) add up over the elements weighted by
 * their atom densities, per-electron ones (Compton, Moller, Bhabha,
 * annihilation, ionisation loss) use the total electron density, and a pair
 * or bremsstrahlung interaction draws its target element from the partial
 * cross sections with one extra random number (single-element materials
 * draw none). */
typedef struct {
  double Z, A_g_mol, density_g_cm3, I_eV;
  uint32_t n_elements;
  double el_Z[4], el_A[4], el_atoms[4];
} or_material;

typedef struct {
  /* geometry: a stack of slabs along z, slab k spans [z[k], z[k+1]) */
  uint32_t n_slabs;
  const double* z_mm;          /* n_slabs + 1 increasing planes          */
  const uint32_t* material;    /* n_slabs material indices               */
  uint32_t n_materials;
  const or_material* materials;
  double half_xy_mm;           /* transverse extent is [-H, H]^2         */
  /* physics / stepping configuration */
  double bz_tesla;
  double gamma_cut_MeV, electron_cut_MeV;
  uint32_t n_bins;
  double emin_MeV, emax_MeV;
  double dr_over_range, final_range_mm, lin_loss_limit;
  uint32_t process_mask;
  uint32_t max_steps_per_track;
  uint32_t seed;
} or_setup;

typedef struct {
  uint32_t event;      /* tally row                                     */
  uint32_t species;    /* OR_GAMMA / OR_ELECTRON / OR_POSITRON          */
  double ekin_MeV;     /* kinetic energy (total energy for a photon)    */
  double pos_mm[3];
  double dir[3];       /* need not be normalised                        */
} or_primary;

typedef struct {
  double edep;          /* sum of this event's deposits over slabs       */
  double escaped[3];    /* kinetic energy leaving the stack, per species */
  double killed;        /* kinetic energy of tracks stopped by watchdog  */
  double charged_len;   /* total e-/e+ path length (mm)                  */
  uint64_t n_steps;
  uint64_t n_created[3];/* secondaries pushed, per species                */
  uint64_t n_null;      /* rejected (null) discrete candidates           */
  uint32_t n_pair, n_annih;
} or_ledger;

typedef struct {
  uint32_t event, species;
  uint64_t id;
  uint32_t step;        /* step index n of this step (before increment)  */
  int32_t slab_after;   /* -1 once the track has left the stack          */
  uint32_t limiter, process;
  double e_before, e_after;
  double pos_after[3];
  double step_len;
  double edep;          /* energy deposited during this step             */
} or_step_rec;

typedef struct or_ctx or_ctx;

/* Builds the cross-section / stopping-power / range tables. 0 = OK. */
int or_create(const or_setup* s, or_ctx** out);

/*
 * Box geometry (instead of the slab stack): n_boxes non-overlapping
 * axis-aligned boxes [lo, hi] inside a world box, whose remaining volume is
 * made of world_material; leaving the world box leaves the geometry.
 * Volume v < n_boxes is box v, volume n_boxes the world; deposits are
 * scored per volume (n_boxes + 1 columns).  A point on a face belongs to
 * the box it moves into (per axis: lo < p < hi, or p = lo moving with
 * u >= 0, or p = hi moving with u < 0).  Navigation is brute force over all
 * boxes.  No magnetic field.  The slab fields of s are not used.
 */
typedef struct {
  uint32_t n_boxes;
  const double* lo;           /* n_boxes x 3 (x, y, z), mm               */
  const double* hi;           /* n_boxes x 3, lo < hi                     */
  const uint32_t* material;   /* n_boxes material indices                 */
  double world_lo[3], world_hi[3];
  uint32_t world_material;
} or_boxes;
int or_create_boxes(const or_setup* s, const or_boxes* b, or_ctx** out);
/* volume containing point p moving along u (-1: outside the world) */
int or_geo_locate(const or_ctx* c, const double p[3], const double u[3]);
/* distance from p in volume v along u to the next boundary, and the
 * crossed face (axis, coordinate) */
double or_geo_distance(const or_ctx* c, int v, const double p[3], const double u[3],
                       int* axis, double* face);
/* The same along the helix of curvature kappa (1/mm, signed as in the
 * transport: q 0.299792458 Bz / p) about z: path length to the next
 * boundary searched up to smax (infinity when none is met within it), with
 * the face reached. */
double or_geo_helix_distance(const or_ctx* c, int v, const double p[3], const double u[3], double kappa,
                             double smax, int* axis, double* face);
void or_destroy(or_ctx* c);

/*
 * Transports all primaries to completion.
 *  n_events     tally rows; edep is [n_events][n_slabs] and is ADDED to.
 *  event_keys   RNG event key per row (NULL: key = row index).
 *  ledger       n_events entries, ADDED to (caller zeroes).
 *  log          optional step log (NULL to skip); *log_n returns the number
 *               of steps taken even if it exceeds log_cap.
 *  profile      optional live-track count per breadth-first iteration,
 *               [profile_cap][3], ADDED to; *profile_len returns the number
 *               of iterations (may exceed profile_cap).
 *  stack_order  0 = LIFO (depth first), 1 = FIFO.
 * Returns 0 on success, <0 on invalid input.
 */
int or_run(or_ctx* c, const or_primary* prim, uint64_t n_prim,
           uint32_t n_events, const uint32_t* event_keys,
           double* edep, or_ledger* ledger,
           or_step_rec* log, uint64_t log_cap, uint64_t* log_n,
           uint64_t* profile, uint32_t profile_cap, uint32_t* profile_len,
           int stack_order);

/* As or_run, and records every track leaving the stack (through the first
 * or last plane, a transverse wall, or the field-safety margin) in
 * exits[*exits_n] with its event row, species, kinetic energy, exit point
 * and direction; *exits_n counts all exits (records beyond exits_cap are
 * dropped).  exits_n NULL: nothing recorded. */
int or_run_exits(or_ctx* c, const or_primary* prim, uint64_t n_prim,
                 uint32_t n_events, const uint32_t* event_keys,
                 double* edep, or_ledger* ledger,
                 or_step_rec* log, uint64_t log_cap, uint64_t* log_n,
                 uint64_t* profile, uint32_t profile_cap, uint32_t* profile_len,
                 int stack_order, or_primary* exits, uint64_t exits_cap, uint64_t* exits_n);

/* Table export: [n_materials][OR_N_TABLES][n_bins+1]. */
enum { OR_N_TABLES = 11 };
uint64_t or_table_count(const or_ctx* c);
int or_export_tables(const or_ctx* c, double* out, uint64_t n);
/* Interpolated table value for material m, table t at energy E. */
double or_table_lookup(const or_ctx* c, uint32_t m, uint32_t t, double E);
/* Inverse range of species (1 e-, 2 e+) in material m. */
double or_inverse_range(const or_ctx* c, uint32_t m, uint32_t species, double r);

/* Null-collision bound of an e- (species 1) or e+ (2) step in material m
 * whose energy spans [a, b]: the largest value of the interpolated discrete
 * total cross section (1/mm) on the interval, each process counted from its
 * threshold on (right-continuous). */
double or_sigma_bound(const or_ctx* c, uint32_t m, uint32_t species, double a, double b);
/* That discrete total at energy E (the same right-continuous convention). */
double or_sigma_total(const or_ctx* c, uint32_t m, uint32_t species, double E);

/* Direct formula evaluation (no tables) for pins. */
enum {
  OR_F_SIGMA_KN = 0,      /* per-electron Klein-Nishina sigma (mm^2)      */
  OR_F_SIGMA_PE = 1,      /* per-atom photoelectric sigma                 */
  OR_F_SIGMA_PAIR = 2,    /* per-atom pair sigma (quadrature)             */
  OR_F_DSDE_PAIR = 3,     /* d sigma / d eps (arg2 = eps)                 */
  OR_F_SIGMA_BREM = 4,    /* per-atom sigma above k_c (quadrature)        */
  OR_F_DSDK_BREM = 5,     /* d sigma / d k (arg2 = k)                     */
  OR_F_SBREM = 6,         /* restricted radiative loss MeV/mm             */
  OR_F_SIGMA_MOLLER = 7,  /* per-electron Moller sigma above cut          */
  OR_F_DSDE_MOLLER = 8,   /* d sigma / d eps (arg2 = eps)                 */
  OR_F_SIGMA_BHABHA = 9,
  OR_F_DSDE_BHABHA = 10,
  OR_F_SION_E = 11,       /* restricted collision loss e- MeV/mm, arg2=cut*/
  OR_F_SION_P = 12,       /* restricted collision loss e+ MeV/mm, arg2=cut*/
  OR_F_SIGMA_ANNIH = 13,  /* per-electron Heitler sigma                   */
  OR_F_DSDE_COMPTON = 14, /* d sigma / d eps (arg2 = eps)                 */
  OR_F_PAIR_FMAX = 15,    /* rejection bound of the pair sampler          */
  OR_F_PAIR_F = 16,       /* rejection function of the pair sampler       */
  OR_F_BREM_BOUND = 17,   /* rejection bound of the brems sampler         */
  OR_F_BREM_F = 18,       /* rejection function (brace) at arg2 = k       */
  OR_F_X0 = 19,           /* radiation length (mm), Tsai's form           */
  OR_F_HIGHLAND = 20,     /* theta_0 (rad) of e-/e+ with kinetic energy E
                             after a path arg2 (mm)                       */
  OR_F_FLUCT_VAR_E = 21,  /* loss variance (MeV^2) of an e- over a path
                             arg2 with delta-ray cut `cut`                */
  OR_F_FLUCT_VAR_P = 22   /* the same for an e+                           */
};
double or_formula(int which, const or_material* m, double cut, double E,
                  double arg2);

/* Philox4x32-10 block. */
void or_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Uniform U_i of the draw stream of (key, track id, step). */
double or_uniform(const uint32_t key[2], uint64_t id, uint32_t step,
                  uint32_t i);
/* Child id of secondary k created at step n of track id. */
uint64_t or_child_id(const uint32_t key[2], uint64_t id, uint32_t step,
                     uint32_t k);

/*
 * Runs one interaction sampler on its own draw stream starting at draw
 * index 2 (the index a sampler starts from inside a step).
 * which: 0 Compton (E = photon energy), 1 pair, 2 brems, 3 Moller,
 *        4 Bhabha, 5 annihilation in flight.
 * out (<= 16 doubles): [0] = sampled fraction (eps / k / T_delta ...),
 * [1] = number of trials, then energies and unit directions of the
 * surviving parent and up to two secondaries (see ems_oracle.c), and
 * [15] = index of the target element (pair, brems; else 0).
 */
int or_sample(const or_ctx* c, int which, uint32_t material, double E,
              const double dir[3], const uint32_t key[2], uint64_t id,
              uint32_t step, double* out);

/*
 * Runs one along-step sampler on the draws a charged step of (key, id,
 * step) uses for it.  which 0: multiple scattering of a track of kinetic
 * energy T after a path s, out[0] = theta_0, out[1..3] = new direction;
 * which 1 (e-) / 2 (e+): loss fluctuation, out[0] = the loss sampled
 * around the mean loss `mean` over the path s from kinetic energy T
 * (not clamped to T), out[1] = its variance.
 */
int or_sample_along(const or_ctx* c, int which, uint32_t material, double T,
                    double s, double mean, const double dir[3],
                    const uint32_t key[2], uint64_t id, uint32_t step,
                    double* out);

#ifdef __cplusplus
}
#endif
#endif
