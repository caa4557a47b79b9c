// ems_device.hpp -- device-side data layout shared by the kernels and the
// host runtime: SoA track queues, the loop-control block, kernel arguments.
#pragma once
#include "ems_step.hpp"

namespace ems {

// One species queue buffer, structure of arrays: position and energy in
// FP64, 64-bit id, direction in the arithmetic type R, then event row, RNG
// event key, and step count and volume packed in one word (n << b | volume,
// b = 12 for the slab stack, more for a large box geometry; all ones marks a
// dead slot).  76 bytes per track in the FP64 form, 64 in the mixed form.
// The six buffers (2 x 3 species) are consecutive blocks of cap *
// track_bytes.
constexpr uint32_t kSlabBits = 12, kSlabMask = (1u << kSlabBits) - 1;
constexpr uint32_t kMaxSlabs = kSlabMask;                 // slab indices 0..4094
constexpr uint32_t kMaxBoxes = 1u << 24;
constexpr uint32_t kMaxStepsPerTrack = (1u << 20) - 1;    // step counts fit 20 bits
constexpr uint32_t kDeadRecord = 0xFFFFFFFFu;
template <class R>
struct Queue {
  double *x, *y, *z, *E;
  uint64_t* id;
  R *ux, *uy, *uz;
  uint32_t *ev, *key, *ns;
};
template <class R>
constexpr size_t track_bytes() {
  return 4 * 8 + 8 + 3 * sizeof(R) + 3 * 4;
}

template <class R>
EMS_HD Queue<R> queue_view(char* base, uint64_t cap, uint32_t buf, uint32_t sp) {
  char* b = base + (size_t)(buf * 3u + sp) * cap * track_bytes<R>();
  Queue<R> q;
  q.x = reinterpret_cast<double*>(b);
  q.y = q.x + cap;
  q.z = q.y + cap;
  q.E = q.z + cap;
  q.id = reinterpret_cast<uint64_t*>(q.E + cap);
  q.ux = reinterpret_cast<R*>(q.id + cap);
  q.uy = q.ux + cap;
  q.uz = q.uy + cap;
  q.ev = reinterpret_cast<uint32_t*>(q.uz + cap);
  q.key = q.ev + cap;
  q.ns = q.key + cap;
  return q;
}

// Loop control, written by the last block of each step launch.
//
// Each next-queue buffer of capacity cap has two regions: survivors and
// carried tracks of that species fill it from the bottom (home region), new
// secondaries from the top (position cap-1-s for secondary slot s).  The
// secondaries of species q may use at most cap - n_cur[q] slots, which leaves
// room for every survivor, so a step whose secondaries do not fit is simply
// not taken: the track is carried unchanged and stepped again later (its
// random numbers depend only on its id and step count).
struct Ctl {
  uint32_t cur;           // index of the current buffer (0/1)
  uint32_t n_home[3];     // current queues: tracks in the home region
  uint32_t n_sec[3];      // current queues: tracks in the secondary region
  uint32_t next_home[3];  // append counters of the next queues
  uint32_t next_sec[3];
  uint32_t blocks_done;   // completion ticket of the running launch
  uint32_t iteration;
  uint32_t live;          // tracks in the current queues (after the swap)
  uint32_t error;         // kErr* bits
  uint32_t peak[3];
  uint32_t commits;       // steps taken in the running launch
  uint32_t carried;       // live tracks carried unstepped in the running launch
  uint32_t cursor[2];     // next queue index handed out (photon, e-/e+ launch)
  unsigned long long steps[3], created[3], deferred, log_n;
  unsigned long long visits[3];  // track records loaded (one per visit)
  unsigned long long made_by[2];  // secondary records written (photon, e-/e+ launches)
  // Live records: the extents n_home + n_sec may include dead slots (unused
  // ends of wave-private append chunks); n_real counts the live tracks of
  // the current queues, next_real those written to the next queues.
  uint32_t n_real[3];
  uint32_t next_real[3];
  unsigned long long exit_n;  // outgoing tracks recorded (may exceed the capacity)
  // Short electrons (KArgs::short_E): extent and live records of the
  // current short buffer, append counters of the next one, the spill
  // buffer's extent (tracks the short launch hands to this iteration's
  // e-/e+ launch) and the short launch's cursor.
  uint32_t n_short, n_short_real, next_short, next_short_real, n_spill, cursor_s;
  unsigned long long steps_s;  // e- steps taken by the short launches
};
enum : uint32_t { kErrOverflow = 1u, kErrStall = 2u, kErrCorrupt = 4u };

// Track prepared on the host for injection (slab located, direction unit,
// RNG event key of its row).
struct InjRec {
  double x, y, z, ux, uy, uz, E;
  uint64_t id;
  uint32_t ev, sp;
  int32_t slab;
  uint32_t key;
};

// Outgoing track, laid out as a primary record of the public header.
struct ExitRec {
  uint32_t event, species;
  double ekin, pos[3], dir[3];
};

// Per-event ledger as laid out in the public header.
struct LedgerDev {
  double edep, escaped[3], killed, charged_len;
  unsigned long long n_steps, n_created[3], n_null;
  uint32_t n_pair, n_annih;
};

struct StepRec {
  uint32_t event, species;
  uint64_t id;
  uint32_t step;
  int32_t slab_after;
  uint32_t limiter, process;
  double e_before, e_after, pos[3], step_len, edep;
};

enum : uint32_t { kFlagSteplog = 1u, kFlagFullLedger = 2u, kFlagProfile = 4u, kFlagEventLive = 8u, kFlagTiming = 16u };

struct KArgs {
  char* qbase;         // six queue buffers, see queue_view
  Ctl* ctl;
  double* edep;        // [rows][n_slabs]
  LedgerDev* ledger;   // [rows]
  const void* tab_g;   // photon table block [mat][3][nodes] (double or float)
  const void* tab_l;   // lepton table block [mat][10][nodes]
  const double* zplane;
  const uint32_t* slab_mat;
  const MatRT* mat;
  const double* el_c;   // element screening constants [mat][4][2]
  const void* el_tab;   // partial pair / brems totals [mat][4][2][nodes] (double or float)
  StepRec* log;
  uint32_t* profile;   // [profile_cap][3]
  int32_t* live_ev;    // [rows] live tracks per event (kFlagEventLive)
  uint64_t cap;        // tracks per species per buffer
  uint32_t max_events;  // tally rows
  uint64_t log_cap;
  uint32_t profile_cap;
  uint32_t flags;
  uint32_t n_mat;
  uint32_t lds_g, lds_l;      // dynamic LDS of the photon / lepton kernels
  uint32_t steps_per_visit;   // steps a thread may take per launch
  uint32_t refill_below;      // batch commit/refill when at most this many lanes still step
  uint32_t interact_min;      // e-/e+: sample a batch's interactions once this many wait
  uint32_t photon_steps_per_visit, photon_refill_below;  // the photon kernel's own two
  uint32_t precision;  // 0: FP64 kernels, 1: mixed kernels
  uint32_t waves_g, waves_l;  // waves of the photon and of the e-/e+ launch
  ExitRec* exits;             // outgoing tracks (exit_cap records)
  uint64_t exit_cap;
  uint32_t geo;               // geometry kind: 0 slab stack, 1 boxes
  uint32_t feat_g, feat_l;    // optional parts (kF* bits) of the photon and e-/e+ kernels launched
  uint32_t vol_bits;          // low bits of the packed word that hold the volume
  StepEnv<double> env;  // scalars; its pointers are set per block
  // Short electrons: e- secondaries below short_E (0: none) are appended to
  // a buffer of their own (two of cap_s records, current and next) and take
  // their first step in a launch of their own at the start of the next
  // iteration; a track whose first step selects an interaction goes to the
  // spill buffer (cap_p records) for the e-/e+ launch of that iteration.
  char* sbase;                // the two short buffers, then the spill buffer
  uint64_t cap_s, cap_p;
  double short_E;
  uint32_t waves_s;           // waves of the short launch
};

// short buffer b (0/1) and the spill buffer (b = 2), laid out as queues
template <class R>
EMS_HD Queue<R> short_view(const KArgs& a, uint32_t b) {
  char* base = a.sbase + (size_t)b * a.cap_s * track_bytes<R>();
  return queue_view<R>(base, b == 2 ? a.cap_p : a.cap_s, 0, 0);
}

}  // namespace ems
