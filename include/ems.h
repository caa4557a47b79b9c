/*
 * ems.h -- C ABI of the MI355X (gfx950) electromagnetic-shower transport
 * library.
 *
 * The library implements the per-step, track-parallel transport loop of
 * "Offloading electromagnetic shower transport to GPUs" (AdePT, ACAT 2021):
 * one step is taken for the whole population of e-, e+ and gamma tracks at a
 * time, secondaries are appended in parallel to per-species "next" arrays that
 * are swapped with the "current" arrays after every step, and the species of a
 * track is implied by the array it is in (section 3, "Stepping workflow").
 * Physics follows section 2.2 (run-time functions taking scalar arguments plus
 * an abstracted counter-based RNG), the charged propagation follows section
 * 2.3 (constant field; here an exact helix), and per-event hit arrays are
 * returned to the host as in section 4 ("Geant4 integration").
 *
 * Conventions shared by every entry point:
 *  - Every call returns ems_status: 0 on success, a negative code on error;
 *    nothing throws or aborts.  ems_last_error() gives a thread-local text.
 *  - "host" pointers are ordinary CPU memory read or written before the call
 *    returns; "device" pointers are HIP device memory owned by the caller.
 *  - Units: MeV, mm, tesla.  Species codes: EMS_GAMMA, EMS_ELECTRON,
 *    EMS_POSITRON.
 *  - A context is single-threaded: calls on one ems_ctx must not overlap.
 *  - After a HIP error the context is failed: every later call except
 *    ems_destroy returns EMS_E_STATE.
 */
#ifndef EMS_H
#define EMS_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EMS_ABI_VERSION 8u

typedef int32_t ems_status;
enum {
  EMS_OK = 0,
  EMS_E_INVALID = -1,   /* bad argument; nothing was changed               */
  EMS_E_CAPACITY = -2,  /* workspace or queue capacity exceeded            */
  EMS_E_DEVICE = -3,    /* a HIP runtime call failed                        */
  EMS_E_STATE = -4,     /* context failed earlier, or call out of order     */
  EMS_E_BUSY = -5,
  EMS_E_TIMEOUT = -6,
  EMS_E_VERSION = -7    /* abi_version does not match EMS_ABI_VERSION       */
};
enum { EMS_GAMMA = 0, EMS_ELECTRON = 1, EMS_POSITRON = 2 };
enum { EMS_FP64 = 0, EMS_MIXED = 1 };

/* process_mask bits */
enum {
  EMS_P_COMPTON = 1u << 0, EMS_P_PHOT = 1u << 1, EMS_P_CONV = 1u << 2,
  EMS_P_EIONI = 1u << 3,   /* Moller / Bhabha delta rays above the cut     */
  EMS_P_EBREM = 1u << 4,   /* bremsstrahlung photons above the cut         */
  EMS_P_ANNIH = 1u << 5,   /* positron annihilation in flight               */
  EMS_P_CONT = 1u << 6,    /* continuous restricted energy loss             */
  EMS_P_ALL = 0x7fu,
  /* Optional along-step processes of e-/e+ (not in EMS_P_ALL), the rest of
   * the electromagnetic physics the paper's G4HepEm covers (section 2.2):  */
  EMS_P_MSC = 1u << 7,     /* multiple Coulomb scattering: at the end of each
                              charged step of length s the direction turns by
                              a space angle theta_0 sqrt(-2 ln u1), azimuth
                              2 pi u2, theta_0 Highland's width for s / X0
                              (X0 after Tsai, 1/X0 summed over elements); a
                              track turned back on an inner plane stays in
                              its slab, one reaching the first or last plane
                              or a wall leaves the stack                     */
  EMS_P_FLUCT = 1u << 8    /* restricted-loss fluctuations (with EMS_P_CONT):
                              the step's loss is drawn from a gamma law with
                              its mean loss and the Bethe second moment of
                              the sub-cut delta rays (Marsaglia-Tsang, at most
                              16 trials), capped at the kinetic energy       */
};
/* flags bits */
enum {
  EMS_F_STEPLOG = 1u << 0,     /* record every step (tests; slow)           */
  EMS_F_FULL_LEDGER = 1u << 1, /* per-event step/secondary/null counts and
                                  charged path length (one more atomic per
                                  step); energy terms are always kept       */
  EMS_F_PROFILE = 1u << 2,     /* live tracks per species per iteration     */
  EMS_F_EVENT_LIVE = 1u << 3,  /* per-event live-track counters (set by the
                                  offload server to detect finished events) */
  EMS_F_KERNEL_TIMING = 1u << 4, /* a HIP event after every launch: per-kernel
                                  device time in ems_run_stats.kernel_ms;
                                  the chunk's kernels are then launched
                                  directly, not replayed from a graph      */
  EMS_F_NO_GRAPH = 1u << 5,     /* launch each chunk's kernels directly
                                  instead of replaying a captured hipGraph
                                  of steps_per_launch iterations (always
                                  direct on the null stream)               */
  EMS_F_FULL_KERNELS = 1u << 6  /* launch the kernels built with every
                                  optional part (field, multiple scattering,
                                  fluctuations, compound targets, per-step
                                  records) instead of the smallest variant
                                  that covers the configuration; the
                                  results are the same (tests)             */
};

/* A material: a single element (n_elements = 0: Z, A_g_mol), or a compound
 * of 1..4 elements with el_atoms[i] atoms of element (el_Z[i], el_A[i]) per
 * formula unit (Z and A_g_mol are then ignored), such as the lead tungstate
 * absorber of the paper's validation calorimeter (section 2.2).  Density and
 * mean excitation energy are the material's.  In a compound the per-atom
 * cross sections (photo-effect, pair, bremsstrahlung and its sub-cut loss)
 * add up over the elements at their atom densities, the per-electron ones
 * (Compton, Moller, Bhabha, annihilation, ionisation loss) use the total
 * electron density, and pair production and bremsstrahlung draw their target
 * element from the partial cross sections with one extra random number of
 * the interaction (single-element materials draw none). */
typedef struct {
  double Z, A_g_mol, density_g_cm3, I_eV;
  uint32_t n_elements;           /* 0: single element; 1 .. 4: compound      */
  double el_Z[4], el_A[4], el_atoms[4];
} ems_material;

/* Geometry, one of two kinds.
 *
 * Slab stack along z (the paper's 50-layer sampling calorimeter, section
 * 2.2; n_boxes = 0): slab k spans [z_mm[k], z_mm[k+1]) and is made of
 * material[k]; deposits are scored per slab (n_slabs columns).
 *
 * Boxes (n_boxes > 0; n_slabs = 0 and the slab fields unused): box v spans
 * [box_lo[v], box_hi[v]] (x, y, z) and is made of box_material[v]; boxes may
 * touch but not overlap and lie inside the world box [world_lo, world_hi],
 * whose remaining volume is world_material; a track reaching the world's
 * surface leaves the geometry.  A point on a face belongs to the box it
 * moves into (per axis lo < p < hi, or p = lo moving with u >= 0, or p = hi
 * moving with u < 0).  Navigation walks a bounding-volume hierarchy built at
 * ems_create, the acceleration structure of the paper's geometry work
 * (section 2.1), whose results equal a walk over all boxes.  Deposits are
 * scored per volume: n_boxes + 1 columns, the world last.  In a field
 * (bz_tesla != 0) charged tracks follow the exact helix about z and reach a
 * box face where the helix meets its plane (section 2.3: the boundary along
 * the curved path), searched up to the continuous-loss step limit; from the
 * world volume the hierarchy supplies the boxes the arc's bounding box
 * overlaps.  The volume index shares a 32-bit word with the
 * track's step count: max_steps_per_track must stay below 2^(32 - b), b the
 * bits of n_boxes + 2 (at least 12). */
typedef struct {
  uint32_t n_slabs;              /* 1 .. 4095 (0 with boxes)                */
  const double* z_mm;            /* host, n_slabs + 1 strictly increasing   */
  const uint32_t* material;      /* host, n_slabs indices < n_materials     */
  uint32_t n_materials;          /* 1 .. 4                                  */
  const ems_material* materials; /* host                                    */
  double half_xy_mm;             /* transverse extent [-H, H]^2, H > 0      */
  uint32_t n_boxes;              /* 0: slab stack; 1 .. 2^24: boxes          */
  const double* box_lo;          /* host, n_boxes x 3, mm                   */
  const double* box_hi;          /* host, n_boxes x 3, lo < hi              */
  const uint32_t* box_material;  /* host, n_boxes indices < n_materials     */
  double world_lo[3], world_hi[3];
  uint32_t world_material;
} ems_geometry;

typedef struct {
  uint32_t abi_version;          /* EMS_ABI_VERSION                          */
  uint32_t precision;            /* EMS_FP64 or EMS_MIXED                    */
  double bz_tesla;               /* uniform field along +z                   */
  double gamma_cut_MeV;          /* bremsstrahlung production threshold      */
  double electron_cut_MeV;       /* delta-ray production threshold           */
  uint32_t n_bins;               /* log-energy bins (nodes = n_bins + 1)     */
  double emin_MeV, emax_MeV;     /* table range; emin is the tracking cut    */
  double dr_over_range;          /* step-function alpha                      */
  double final_range_mm;         /* step-function rho                        */
  double lin_loss_limit;         /* linear-loss limit (fraction of range)    */
  uint32_t process_mask;         /* EMS_P_* bits                             */
  uint32_t flags;                /* EMS_F_* bits                             */
  uint32_t max_steps_per_track;  /* watchdog, 1 .. 2^20 - 1                  */
  uint32_t seed;                 /* Philox key word 0                        */
  uint32_t max_events;           /* tally rows (>= 1)                        */
  uint64_t track_capacity;       /* tracks per species per queue, 64..2^28 */
  uint32_t steps_per_launch;     /* iterations enqueued between status reads */
  uint32_t launch_blocks;        /* step-kernel grid (0 = library default)   */
  uint64_t steplog_capacity;     /* records kept when EMS_F_STEPLOG is set   */
  uint32_t profile_capacity;     /* iterations kept when EMS_F_PROFILE       */
  uint32_t steps_per_visit;      /* steps one thread may take of one track per
                                    launch, through interactions its track
                                    survives (results do not depend on it);
                                    1 here and in photon_steps_per_visit =
                                    strictly one step of the whole
                                    population per iteration               */
  uint32_t refill_below;         /* a wave commits the visits that ended and
                                    refills those lanes once at most this
                                    many of its 64 lanes are still stepping
                                    (0..63; results do not depend on it)    */
  uint32_t interact_min;         /* e-/e+ kernel: a batch samples the
                                    interactions its lanes selected only when
                                    at least this many are waiting, or when
                                    the queue is used up; until then those
                                    lanes keep their tracks and wait (0..64;
                                    0 = every batch; results do not depend
                                    on it)                                  */
  uint32_t photon_steps_per_visit; /* steps_per_visit and refill_below of
                                      the photon kernel (1..1024, 0..63); the
                                      two above then apply to the e-/e+
                                      kernel.  Results do not depend on them */
  uint32_t photon_refill_below;
  uint64_t exit_capacity;        /* outgoing-track records kept per run
                                    (0 = none; see ems_read_exits)          */
  double short_electron_MeV;     /* e- secondaries below this kinetic energy
                                    take their first step in a launch of
                                    their own at the start of the next
                                    iteration (most range out there); 0 =
                                    off.  Adds two buffers of half the
                                    track capacity and one of 5/8 of it.
                                    Results do not depend on it             */
} ems_config;

/* One primary track (64 bytes). event is the tally row (< max_events); the
 * track id is the running index of the primary within its row. */
typedef struct {
  uint32_t event, species;
  double ekin_MeV;               /* kinetic energy; photon: total energy     */
  double pos_mm[3];              /* inside the geometry (on a plane or face:
                                    the volume the direction enters)         */
  double dir[3];                 /* non-zero; normalised by the library      */
} ems_primary;

/* Per-event energy ledger.  Exactly (to rounding):
 *   sum of primary kinetic energies = edep + sum(escaped) + killed
 *                                     + 2 m_e (n_pair - n_annih)            */
typedef struct {
  double edep;                   /* sum of the row's slab deposits          */
  double escaped[3];             /* kinetic energy leaving the stack        */
  double killed;                 /* kinetic energy removed by the watchdog  */
  double charged_len;            /* e-/e+ path length (EMS_F_FULL_LEDGER)   */
  uint64_t n_steps;              /* (EMS_F_FULL_LEDGER)                     */
  uint64_t n_created[3];         /* pushed secondaries (EMS_F_FULL_LEDGER)  */
  uint64_t n_null;               /* null collisions (EMS_F_FULL_LEDGER)     */
  uint32_t n_pair, n_annih;
} ems_ledger;

/* One step of one track (EMS_F_STEPLOG), 88 bytes. */
typedef struct {
  uint32_t event, species;
  uint64_t id;
  uint32_t step;                 /* step index before the increment         */
  int32_t slab_after;            /* -1 once the track has ended             */
  uint32_t limiter, process;
  double e_before, e_after;
  double pos_after[3];
  double step_len;
  double edep;                   /* deposited during this step              */
} ems_step_record;

typedef struct {
  uint64_t iterations;           /* breadth-first steps of the population   */
  uint64_t steps[3];             /* track steps per species                 */
  uint64_t created[3];           /* secondaries pushed per species          */
  uint64_t deferred;             /* track-steps postponed for capacity      */
  uint64_t launches;             /* step-kernel launches                    */
  uint32_t peak_live[3];         /* largest queue per species               */
  uint32_t steplog_overflow;     /* records dropped beyond the capacity     */
  double run_ms;                 /* host wall time of the last ems_run      */
  double step_kernel_ms;         /* device time of the step launches, from
                                    HIP events around each chain of launches
                                    on the bound stream (gaps included)     */
  uint64_t visits[3];            /* track records loaded per species (one
                                    per visit of a thread to a track)       */
  uint64_t made_by[2];           /* secondary records written by the photon
                                    launches and by the e-/e+ launches      */
  double kernel_ms[3];           /* with EMS_F_KERNEL_TIMING: device time of
                                    the photon, the e-/e+ and the short-
                                    electron launches, event to event on
                                    the bound stream                        */
  uint64_t graph_launches;       /* chunks replayed from a captured hipGraph */
  uint64_t short_steps;          /* e- steps (within steps[1]) taken by the
                                    short-electron launches                 */
} ems_run_stats;

typedef struct ems_ctx ems_ctx;

/* Measurement (section 5, where the paper profiles its kernels against the
 * device's limits): the device's FP64 atomic-add throughput on a tally-like
 * scatter:
 * n_ops adds of 1.0 by the instruction the deposit tallies use, each to a
 * cell drawn uniformly (fixed hash of the op index) from the n_cells
 * doubles at d_cells (device, zeroed here, left holding the counts).  The
 * adds run on hip_stream (NULL: the null stream) between two HIP events;
 * *ms receives their elapsed time.  A ceiling for the tallies' atomic rate,
 * against which bench.py reports the kernels' achieved rate.
 * EMS_E_INVALID for null pointers or zero sizes. */
ems_status ems_probe_atomics(void* d_cells, uint64_t n_cells, uint64_t n_ops, void* hip_stream, double* ms);

/* Initialisation (section 2.2: physics data built once and transferred to
 * the GPU; section 3: per-species track arrays).  Device workspace needed
 * for (cfg, geo), in bytes (host output): loop-control block, tables,
 * geometry, tallies and the two track queues per species.  EMS_E_INVALID
 * for an invalid configuration or geometry. */
ems_status ems_workspace_bytes(const ems_config* cfg, const ems_geometry* geo,
                               uint64_t* bytes);

/* Initialisation (section 2.2 for the physics tables, section 2.1 for the
 * geometry, section 3 for the track arrays): builds the tables on the host,
 * uploads tables and geometry into the caller's device workspace (d_workspace, >= ems_workspace_bytes, 256-byte
 * aligned) and binds the caller's HIP stream (hipStream_t; NULL = the null
 * stream).  Workspace and stream must outlive the context; the context
 * owns only host memory, two pinned staging buffers and HIP events.
 * Tallies start at zero and event key of row r is r.  EMS_E_INVALID for bad
 * arguments, EMS_E_CAPACITY when bytes < ems_workspace_bytes, EMS_E_DEVICE
 * on a HIP error; *out is untouched on error. */
ems_status ems_create(const ems_config* cfg, const ems_geometry* geo,
                      void* d_workspace, uint64_t bytes, void* hip_stream,
                      ems_ctx** out);

/* Bytes of the library's static device workspace: one copy per GPU the
 * library runs on, held from the loading of the library until the process
 * ends. */
#define EMS_STATIC_WORKSPACE_BYTES (64ull << 20)

/* For callers that cannot allocate (code under graph capture, tight serving
 * loops, harnesses that forbid allocation): ems_create without a caller
 * workspace.  The context runs in the library's static workspace of the
 * current device (EMS_STATIC_WORKSPACE_BYTES) and binds hip_stream (NULL =
 * the null stream).  Neither this call nor any later call on the context
 * allocates device memory or pinned host memory (no hipMalloc, hipFree,
 * hipHostMalloc, graphs or events): host staging is ordinary memory and
 * every chunk of iterations is launched directly.  Inputs (primaries) and
 * outputs (deposits, ledgers, exits) are passed as with ems_create; every
 * other entry point works on the context as on one from ems_create.
 * ems_create clears the control block, the tallies and the queues (the
 * array keeps the contents of the previous context on that GPU).  One
 * context at a time may hold a GPU's static workspace: two contexts on one
 * GPU would race on it, so a second call before ems_destroy of the first
 * returns EMS_E_BUSY.  EMS_E_CAPACITY when the configuration needs more than
 * EMS_STATIC_WORKSPACE_BYTES (the message names the bytes needed; a smaller
 * track_capacity or max_events fits); EMS_E_INVALID for a bad configuration
 * or for the flags EMS_F_KERNEL_TIMING and EMS_F_EVENT_LIVE (they need
 * events and pinned memory); EMS_E_DEVICE on a HIP error. *out is untouched
 * on error. */
ems_status ems_create_static(const ems_config* cfg, const ems_geometry* geo,
                             void* hip_stream, ems_ctx** out);

/* Counter-based random numbers (section 2.2: the physics functions take an
 * abstracted random-number engine): sets the RNG event key of tally rows
 * [first_row, first_row + n) for the
 * primaries enqueued from now on (each track carries its key). Results of a
 * row depend only on (seed, key, its primaries), never on the row. Host
 * only: no device work, no synchronisation. */
ems_status ems_set_event_keys(ems_ctx* ctx, uint32_t first_row, uint32_t n,
                              const uint32_t* host_keys);

/* Particles in (section 4: the tracks handed to the GPU library; section
 * 3: they enter the species' current arrays).  Validates and copies n
 * primaries (host, 64-byte records, read before return) into the current
 * queues.  All or
 * nothing: EMS_E_INVALID (NaN or <= 0 energy, zero direction, position
 * outside the stack, bad species, event >= max_events) or EMS_E_CAPACITY
 * leaves the context unchanged.  Asynchronous on the bound stream. */
ems_status ems_enqueue(ems_ctx* ctx, const ems_primary* host, uint64_t n);
/* Particles in (section 4), already resident in device memory: as
 * ems_enqueue for n primaries held by the caller in one device allocation
 * (64-byte records, read by work queued on the bound stream: keep them
 * unchanged until that stream has passed this call).  The checks,
 * normalisation, volume location and per-row track ids (the running index
 * of each primary within its row, in input order) are computed on the
 * device and give the tracks ems_enqueue would give for the same records.
 * All or nothing: EMS_E_INVALID for an invalid primary (as ems_enqueue) or
 * a pointer that is not n records inside one device allocation;
 * EMS_E_CAPACITY as ems_enqueue.  The primaries of a batch (between two
 * ems_reset_tallies) come either from host or from device memory:
 * EMS_E_STATE for a mix.  Returns after the check pass has drained the
 * bound stream; staging and injection stay queued there. */
ems_status ems_enqueue_device(ems_ctx* ctx, const ems_primary* d_primaries, uint64_t n);

/* The stepping loop (section 3): every live track takes its steps, the
 * secondaries are appended to the next arrays, the arrays are swapped,
 * until no track is left; physics of section 2.2, field propagation of
 * section 2.3.  Returns after the bound stream has drained.  EMS_E_CAPACITY if the queues cannot make
 * progress; EMS_E_DEVICE on a HIP error. */
ems_status ems_run(ems_ctx* ctx);

/* Hits out (section 4: per-event hit arrays copied to the host).  Copies
 * the FP64 deposits of rows [first, first+n) to host_out[n][n_slabs]
 * (row-major, caller-owned); EMS_E_INVALID for rows out of range. */
ems_status ems_read_edep(ems_ctx* ctx, uint32_t first, uint32_t n, double* host_out);
/* Hits out (section 4), kept in device memory: copies the FP64 deposits
 * of rows [first, first+n) to d_out[n][n_slabs] (row-major, caller-owned
 * device memory, one allocation), asynchronously on the bound stream: the
 * caller orders its own reads of d_out after that stream.  EMS_E_INVALID
 * for rows out of range or an output that is not n rows inside one device
 * allocation. */
ems_status ems_read_edep_device(ems_ctx* ctx, uint32_t first, uint32_t n, double* d_out);
/* Hits out (section 4), with the energy accounting of killed tracks that
 * section 2.3 requires: copies the ledgers of rows [first, first+n) to
 * host_out[n]; EMS_E_INVALID for rows out of range. */
ems_status ems_read_ledger(ems_ctx* ctx, uint32_t first, uint32_t n, ems_ledger* host_out);
/* Between batches (section 4: one synchronous batch after another): zeroes
 * deposits, ledgers, the step log, the profile and per-row track-id
 * counters (asynchronous on the bound stream). */
ems_status ems_reset_tallies(ems_ctx* ctx);
/* Tracks that left the stack since the last ems_reset_tallies (the paper's
 * hybrid contract, section 4: particles in, hits and outgoing particles
 * out): one record per track in the primary layout -- event row, species,
 * kinetic energy, exit point (on the first or last plane, on a transverse
 * wall, or within the 1e-6 mm field-safety margin of one) and direction --
 * so that records can be enqueued elsewhere as primaries.  Copies
 * min(cap, *n_total, exit_capacity) records in no particular order;
 * *n_total counts every exit, including those beyond exit_capacity. */
ems_status ems_read_exits(ems_ctx* ctx, ems_primary* host_out, uint64_t cap, uint64_t* n_total);

/* Step-by-step record of the stepping loop (section 3; tests, with
 * EMS_F_STEPLOG): copies up to cap step records (host_out) and returns the
 * number of steps taken in *n (may exceed cap; records beyond the
 * configured capacity are dropped). */
ems_status ems_read_steplog(ems_ctx* ctx, ems_step_record* host_out, uint64_t cap,
                            uint64_t* n);
/* Population per iteration of the stepping loop (section 3; with
 * EMS_F_PROFILE; section 5 discusses how the live population sets the
 * device's occupancy): live tracks per species per iteration of the last
 * run, host_out[cap][3]; *n = iterations run. */
ems_status ems_read_profile(ems_ctx* ctx, uint32_t* host_out, uint32_t cap, uint32_t* n);
/* Counts and timings of the last run (section 5: kernel time, steps and
 * launches of the stepping loop); host copy, no device work. */
ems_status ems_stats(ems_ctx* ctx, ems_run_stats* out);
/* Waits for the bound stream and frees the context's host memory, pinned
 * buffers and events; workspace and stream stay the caller's.  NULL is
 * accepted. */
ems_status ems_destroy(ems_ctx* ctx);
/* Thread-local text of the last error of the calling thread. */
const char* ems_last_error(void);
/* EMS_ABI_VERSION of the built library. */
uint32_t ems_abi_version(void);

/* Physics data as transferred to the GPU (section 2.2): copies the tables
 * this context uploaded back from its device workspace, in the layout of
 * ems_host_tables ([n_materials][11][n_bins + 1]: Compton, photo, pair
 * (1/mm), S e- (MeV/mm), R e- (mm), Moller, brems, S e+, R e+, Bhabha,
 * annihilation), widened to FP64 in the mixed form, so the device copy can
 * be compared with an independent implementation.  n_doubles is the size
 * of host_out; EMS_E_INVALID when it is too small; synchronises the bound
 * stream. */
ems_status ems_export_tables(ems_ctx* ctx, double* host_out, uint64_t n_doubles);

/* ---------------------------------------------------------------------
 * Offload server: a device-resident continuous-batching loop in front of one
 * context, like the paper's hybrid workflow (section 4: particles of a
 * region are handed to the GPU library, hits come back per event) with the
 * staggered injection its analysis section proposes (section 5: new
 * primaries injected while earlier showers are still developing).
 *
 * Producers (any number of host threads) submit requests: the EM tracks of
 * one event.  A driver thread owned by the server admits requests in order
 * while a tally slot is free and the estimated track-buffer bytes of the
 * admitted requests stay within admit_cap_bytes, injects them between chunks
 * of steps_per_launch iterations, detects completed events from per-event
 * live-track counters, and hands their per-slab deposits and ledger back.
 * A result depends only on (seed, event_key, tracks): the same request gives
 * the same deposits alone or in any mix (up to FP64 atomic summation order).
 * --------------------------------------------------------------------- */
typedef struct ems_server ems_server;

typedef struct {
  uint64_t submitted, completed, in_flight, queued;
  uint64_t admitted_bytes, admit_cap_bytes, peak_admitted_bytes;
  uint64_t primaries_completed;
  uint64_t chunks;              /* chunks of iterations launched            */
  double p50_ms, p99_ms, mean_ms, max_ms;  /* submit -> result latency      */
  double wall_s;                /* since creation or the last stats reset   */
  double primaries_per_s;       /* completed primaries / wall_s             */
  uint64_t exits_dropped;       /* outgoing tracks beyond the per-poll
                                   exit_capacity (lost to their requests)   */
} ems_server_info;

/* Continuous batching in front of the stepping loop (section 4: particles
 * of a region handed over, hits back per event; section 5: staggered
 * injection).  cfg->max_events is the number of tally slots (events in
 * flight);
 * EMS_F_STEPLOG and EMS_F_PROFILE are not available in a server.  The
 * server runs its context with EMS_F_EVENT_LIVE set: the workspace must hold
 * ems_workspace_bytes of cfg with that flag (it adds the row lists and the
 * result staging area); EMS_E_CAPACITY otherwise.  Stream as for
 * ems_create; it is used by the driver thread only.  admit_cap_bytes bounds
 * the estimated track-buffer bytes of admitted requests (estimate: 2 x
 * record bytes x (tracks + 0.1 per MeV of request energy + 1)); a request
 * larger than the cap is admitted alone. */
ems_status ems_server_create(const ems_config* cfg, const ems_geometry* geo, void* d_workspace,
                             uint64_t bytes, void* hip_stream, uint64_t admit_cap_bytes,
                             ems_server** out);
/* Particles in (section 4), thread-safe.  Copies n (1..65536) tracks
 * (host, read before return; their event field is ignored);
 * EMS_E_INVALID as for ems_enqueue; EMS_E_BUSY when 2^20 requests wait. */
ems_status ems_server_submit(ems_server* s, const ems_primary* tracks, uint32_t n,
                             uint32_t event_key, uint64_t* ticket);
/* Particles in (section 4) with their arrival time (section 5 measures the
 * time from hand-over to hits): as ems_server_submit, but the request's
 * latency in ems_server_info counts from arrival_ns, a time on the
 * monotonic clock (CLOCK_MONOTONIC, in ns; Python: time.monotonic_ns()),
 * such as the arrival a load schedule planned, so that a producer running
 * late does not hide its delay.  0, or a time later than the call, counts
 * from the call. */
ems_status ems_server_submit_at(ems_server* s, const ems_primary* tracks, uint32_t n,
                                uint32_t event_key, uint64_t arrival_ns, uint64_t* ticket);
/* Hits out per event (section 4), thread-safe.  Waits up to timeout_us
 * (< 0: forever) for the ticket and
 * copies its deposits (edep_out[n_slabs], may be NULL) and ledger (may be
 * NULL); the ticket is released.  EMS_E_TIMEOUT, EMS_E_INVALID (unknown
 * ticket), EMS_E_STATE (the device loop failed). */
/* Hits and particles out (section 4: the GPU region returns its outgoing
 * particles).  As ems_server_wait, and also copies the request's outgoing
 * tracks (with
 * cfg->exit_capacity > 0: the capacity of exits gathered per poll) into
 * exits_out (event field = 0; *n_exits = all of the request's exits, at
 * most exits_cap copied). */
ems_status ems_server_wait_exits(ems_server* s, uint64_t ticket, int64_t timeout_us, double* edep_out,
                                 ems_ledger* ledger_out, ems_primary* exits_out, uint64_t exits_cap,
                                 uint64_t* n_exits);
ems_status ems_server_wait(ems_server* s, uint64_t ticket, int64_t timeout_us,
                           double* edep_out, ems_ledger* ledger_out);
/* Thread-safe, non-blocking (section 4): *done = 1 when the ticket's
 * result is ready; EMS_E_INVALID for an unknown ticket. */
ems_status ems_server_poll(ems_server* s, uint64_t ticket, int* done);
/* Blocks until every request submitted before the call has completed (the
 * paper's Flush, section 4). */
ems_status ems_server_flush(ems_server* s);
/* Latency and throughput of the offload loop (section 5: the batch-size
 * and idle-time effects the paper measures); thread-safe. */
ems_status ems_server_stats(ems_server* s, ems_server_info* out);
/* Restarts the latency and throughput statistics (thread-safe). */
ems_status ems_server_reset_stats(ems_server* s);
/* Stops the driver thread (pending requests are dropped) and frees the
 * server; workspace and stream remain the caller's. */
ems_status ems_server_destroy(ems_server* s);

/* Measurement of the server (section 5: the time from hand-over to hits, and
 * throughput, under load from many host threads) with native producer
 * threads, so that the load is not limited by the caller's runtime.
 * Producer p (n_producers threads) takes requests [first[p], first[p+1]) of
 * reqs in order (first: n_producers + 1 non-decreasing offsets).  A request with arrival_ns = 0 is submitted when fewer than
 * `window` (>= 1) of the producer's requests are outstanding (closed loop;
 * latency from the submission).  A request with arrival_ns != 0 (monotonic
 * clock, ns) is submitted at that time, the producer sleeping until then,
 * through ems_server_submit_at (latency from the arrival, also when the
 * producer runs late); its completions are collected after the last
 * submission.  Results are waited for and discarded.  *max_lag_ms (may be
 * NULL) receives the largest delay of a submission behind its arrival,
 * *last_submit_ns (may be NULL) the monotonic time of the last submission.
 * Returns the first error of any producer (its remaining requests are
 * skipped); EMS_E_INVALID for bad arguments. */
typedef struct {
  const ems_primary* tracks;     /* host, n_tracks records, read during the call */
  uint32_t n_tracks;
  uint32_t event_key;
  uint64_t arrival_ns;           /* 0: closed loop                          */
} ems_load_request;
ems_status ems_server_drive(ems_server* s, const ems_load_request* reqs, const uint64_t* first,
                            uint32_t n_producers, uint32_t window, double* max_lag_ms,
                            uint64_t* last_submit_ns);

/* Physics data (section 2.2), host only (no device needed): the tables the
 * library would upload, layout
 * [n_materials][11][n_bins+1] with tables in the order: Compton, photo, pair
 * (1/mm), S e- (MeV/mm), R e- (mm), Moller, brems, S e+, R e+, Bhabha,
 * annihilation.  Used to compare the library's tables with an independent
 * implementation. */
ems_status ems_host_tables(const ems_config* cfg, const ems_geometry* geo, double* host_out,
                           uint64_t n_doubles);

/* Test hook, never used by ems_run (section 3's loop on the host): runs the
 * library's per-track step code on the host, breadth-first over a queue, for CPU-side checking before any
 * GPU is used.  Arguments as for a run: primaries (host), n_events rows,
 * optional keys (NULL: key = row), edep [n_events][n_slabs] and ledger
 * [n_events] are overwritten, optional step log. */
ems_status ems_debug_host_transport(const ems_config* cfg, const ems_geometry* geo,
                                   const ems_primary* prim, uint64_t n, uint32_t n_events,
                                   const uint32_t* keys, double* edep, ems_ledger* ledger,
                                   ems_step_record* log, uint64_t log_cap, uint64_t* log_n);

#ifdef __cplusplus
}
#endif
#endif
