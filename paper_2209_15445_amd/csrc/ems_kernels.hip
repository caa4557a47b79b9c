// ems_kernels.hip -- gfx950 kernels of the transport loop.
//
// The paper steps the whole track population once per iteration with one
// kernel per species in three streams, appending secondaries to per-species
// "next" index arrays with an atomic counter and swapping current/next after
// each step (section 3).  On MI355X:
//  - one launch per iteration for photons and one for e-/e+ (a concatenated
//    index space [e- | e+]), in stream order, so the light photon kernel is
//    not held to the lepton kernel's register budget and each stages only
//    its own tables in LDS;
//  - the queues hold the tracks themselves (SoA, coalesced); survivors are
//    rewritten compactly each iteration, so slots are reused by construction;
//  - a thread keeps stepping its track (a "visit") until a step creates
//    secondaries or ends the track, so the many boundary crossings of photons
//    in the thin slabs do not each cost a queue round trip; every step still
//    draws from its own (id, step) stream, so histories are unchanged;
//  - appends are aggregated per wave (ballot + popcount prefix, one atomic
//    per wave and species);
//  - secondaries are reserved against a per-species limit that always leaves
//    room for every survivor; a track whose secondaries do not fit is carried
//    from before that step, so a full queue defers work instead of losing it;
//  - the last block of the e-/e+ launch swaps the queues, so a chain of
//    launches needs no host round trip.
#include <hip/hip_runtime.h>

#include "ems_device.hpp"

namespace ems {

namespace {

constexpr int kBlock = 256;
// lanes waiting in the world volume that make a wave compute their boundary
// distances together (box geometries)
#ifndef EMS_WORLD_BATCH
#define EMS_WORLD_BATCH 16
#endif
constexpr uint32_t kWorldBatch = EMS_WORLD_BATCH;
// s_waitcnt immediate for "all vector memory operations done" (vmcnt 0,
// expcnt and lgkmcnt at their maxima: not waited on)
constexpr int kWaitVmem = 0x0F70;

// Reserve `count` (0..3) consecutive slots per lane in an append counter with
// one atomic per wave; returns this lane's first slot.  Every lane of the wave
// must pass the same counter.
__device__ inline uint32_t wave_reserve(uint32_t* counter, uint32_t count) {
  const uint64_t b0 = __ballot(count & 1u);
  const uint64_t b1 = __ballot((count >> 1) & 1u);
  const uint32_t total = (uint32_t)(__popcll(b0) + 2 * __popcll(b1));
  if (total == 0) return 0;
  const uint64_t lt = __lanemask_lt();
  const uint32_t prefix = (uint32_t)(__popcll(b0 & lt) + 2 * __popcll(b1 & lt));
  const int leader = __ffsll((unsigned long long)(b0 | b1)) - 1;
  uint32_t base = 0;
  if ((int)__lane_id() == leader) base = atomicAdd(counter, total);
  base = __shfl(base, leader);
  return base + prefix;
}

// Next queue index for every lane with `want`: taken from the wave's own
// range [lo, hi), which is refilled EMS_CURSOR_CHUNK indices at a time from
// the launch's global cursor, so a wave pays one global atomic per chunk
// instead of one per refill.  Every index below the cursor's final value is
// handed out exactly once (ranges are disjoint and none is dropped).
#ifndef EMS_CURSOR_CHUNK
#define EMS_CURSOR_CHUNK 64
#endif
static_assert(EMS_CURSOR_CHUNK <= 1 || EMS_CURSOR_CHUNK >= 64, "a chunk must cover a whole wave's request");
__device__ inline uint32_t take_next(uint32_t* cursor, bool want, uint32_t& lo, uint32_t& hi) {
  if (EMS_CURSOR_CHUNK <= 1) return wave_reserve(cursor, want ? 1u : 0u);
  const uint64_t m = __ballot(want);
  const uint32_t n = (uint32_t)__popcll(m);
  const uint32_t rank = (uint32_t)__popcll(m & __lanemask_lt());
  const uint32_t avail = hi - lo;
  uint32_t i = lo + rank;
  if (n > avail) {
    // the rest of the old range, then a fresh chunk (n <= 64 <= chunk size)
    uint32_t base = 0;
    const int leader = __ffsll((unsigned long long)m) - 1;
    if ((int)__lane_id() == leader) base = atomicAdd(cursor, (uint32_t)EMS_CURSOR_CHUNK);
    base = __shfl(base, leader);
    if (rank >= avail) i = base + (rank - avail);
    lo = base + (n - avail);
    hi = base + EMS_CURSOR_CHUNK;
  } else {
    lo += n;
  }
  return i;
}

// Append slots in wave-private chunks.  A wave holds a range [lo, hi) of an
// append counter and refills it `chunk` slots at a time (one global atomic
// per chunk instead of one per batch: thousands of waves appending to the
// same few counters otherwise serialise on them).  take_slots reserves cnt
// (0..3) slots per lane and returns the lane's first position x in the
// wave's request; its k-th slot is slot_of(tk, x + k).  Unused ends of the
// ranges are marked dead when the wave exits.  chunk = 1 is exact
// reservation (no unused slots).
struct Take {
  uint32_t lo, avail, base;
};
__device__ inline uint32_t take_slots(uint32_t* counter, uint32_t cnt, uint32_t chunk, uint32_t& lo, uint32_t& hi,
                                      Take& tk) {
  const uint64_t b0 = __ballot(cnt & 1u);
  const uint64_t b1 = __ballot((cnt >> 1) & 1u);
  const uint32_t total = (uint32_t)(__popcll(b0) + 2 * __popcll(b1));
  const uint64_t lt = __lanemask_lt();
  const uint32_t prefix = (uint32_t)(__popcll(b0 & lt) + 2 * __popcll(b1 & lt));
  tk.lo = lo;
  tk.avail = hi - lo;
  tk.base = 0;
  if (total > tk.avail) {
    const uint32_t need = total - tk.avail;
    const uint32_t grab = need > chunk ? need : chunk;
    const int leader = __ffsll((unsigned long long)(b0 | b1)) - 1;
    uint32_t base = 0;
    if ((int)__lane_id() == leader) base = atomicAdd(counter, grab);
    base = __builtin_amdgcn_readfirstlane(__shfl(base, leader));
    tk.base = base;
    lo = base + need;
    hi = base + grab;
  } else {
    lo += total;
  }
  return prefix;
}
__device__ inline uint32_t slot_of(const Take& tk, uint32_t x) {
  return x < tk.avail ? tk.lo + x : tk.base + (x - tk.avail);
}

// Per-iteration append plan of species q (the same in both launches of an
// iteration, computed from the current queue sizes).  The chunk is the
// largest power of two up to EMS_APPEND_CHUNK for which all waves together
// leave unused at most a quarter of the current population and of the free
// room (so small populations append exactly); the secondary limit leaves
// room for every survivor plus the unused chunk ends of the home region.
#ifndef EMS_APPEND_CHUNK
#define EMS_APPEND_CHUNK 256
#endif
struct Plan {
  uint32_t lim[3], chunk[3];
  uint32_t lim_s, chunk_s;  // appends to the next short buffer
};
// The current short electrons (ns) may all survive their first step into
// the next e- queue, so they count with the current e- tracks; the short
// launch's waves also append to that queue's home region.  New short
// electrons are e- of the next iteration as well: the e- secondary limit is
// shared, half of it (at most the short buffer's capacity) for the short
// buffer, so that the next iteration's e- and short electrons together
// again leave room for all their survivors.  The short buffer takes the e-
// chunk, bounded so that all waves together leave unused at most a quarter
// of its capacity.
// SHORT: the kernel variant routes short electrons (the plan is the same
// as without when the context has no short buffers).
template <bool SHORT>
__device__ inline Plan append_plan(const KArgs& a, uint32_t n0, uint32_t n1, uint32_t n2, uint32_t ns) {
  Plan p;
  if constexpr (!SHORT) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const uint64_t n = q == 0 ? n0 : (q == 1 ? n1 : n2);
      const uint64_t room = a.cap - n;
      const uint64_t waves = (uint64_t)a.waves_g + a.waves_l;
      const uint64_t budget = (n < room ? n : room) / 4;
      uint32_t chunk = EMS_APPEND_CHUNK;
      while (chunk > 1 && waves * chunk > budget) chunk >>= 1;
      const uint64_t home_waves = q == 0 ? a.waves_g : a.waves_l;
      p.chunk[q] = chunk;
      p.lim[q] = (uint32_t)(room - (chunk > 1 ? home_waves * chunk : 0));  // slack <= room / 4
    }
    p.lim_s = 0;
    p.chunk_s = 1;
    return p;
  }
  const uint64_t waves = (uint64_t)a.waves_g + a.waves_l + (a.cap_s ? a.waves_s : 0u);
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const uint64_t n = q == 0 ? n0 : (q == 1 ? (uint64_t)n1 + ns : n2);
    const uint64_t room = n < a.cap ? a.cap - n : 0;
    const uint64_t budget = (n < room ? n : room) / 4;
    uint32_t chunk = EMS_APPEND_CHUNK;
    while (chunk > 1 && waves * chunk > budget) chunk >>= 1;
    const uint64_t home_waves = q == 0 ? a.waves_g : (q == 1 && a.cap_s ? a.waves_l + a.waves_s : a.waves_l);
    const uint64_t slack = chunk > 1 ? home_waves * chunk : 0;
    p.chunk[q] = chunk;
    p.lim[q] = (uint32_t)(room > slack ? room - slack : 0);
  }
  uint32_t cs = p.chunk[1];
  while (cs > 1 && waves * cs > a.cap_s / 4) cs >>= 1;
  p.chunk_s = cs;
  p.lim_s = 0;
  if (a.cap_s) {
    const uint32_t half = p.lim[1] / 2;
    p.lim_s = (uint64_t)half < a.cap_s ? half : (uint32_t)a.cap_s;
    p.lim[1] -= p.lim_s;
  }
  return p;
}

// the interactions after which the parent track goes on
__device__ inline bool parent_survives(uint32_t process) {
  return process == kXCompton || process == kXMoller || process == kXBhabha || process == kXBrem;
}

// One slot per lane with `want` among the lanes executing this call (also in
// divergent code): one atomic per call for all of them.
__device__ inline unsigned long long active_append(unsigned long long* counter, bool want) {
  const uint64_t m = __ballot(want);
  if (m == 0) return 0;
  const int leader = __ffsll((unsigned long long)m) - 1;
  unsigned long long base = 0;
  if ((int)__lane_id() == leader) base = atomicAdd(counter, (unsigned long long)__popcll(m));
  base = __shfl(base, leader);
  return base + (unsigned long long)__popcll(m & __lanemask_lt());
}

__device__ inline uint32_t wave_sum(uint32_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// sum over the wave of a per-lane count, one atomic by lane 0
__device__ inline void wave_count(unsigned long long* counter, uint32_t v) {
  const uint32_t s = wave_sum(v);
  if (__lane_id() == 0 && s) atomicAdd(counter, (unsigned long long)s);
}
__device__ inline void wave_count(uint32_t* counter, uint32_t v) {
  const uint32_t s = wave_sum(v);
  if (__lane_id() == 0 && s) atomicAdd(counter, s);
}

template <class R>
__device__ inline void store_track(const Queue<R>& q, uint32_t i, const Trk<R>& t, uint32_t vb) {
  q.x[i] = t.x;
  q.y[i] = t.y;
  q.z[i] = t.z;
  q.ux[i] = t.ux;
  q.uy[i] = t.uy;
  q.uz[i] = t.uz;
  q.E[i] = t.E;
  q.id[i] = t.id;
  q.ev[i] = t.ev;
  q.key[i] = t.key;
  q.ns[i] = (t.n << vb) | (uint32_t)t.slab;
}

// position of the idx-th track of a queue with `home` tracks in the bottom
// region (the rest are in the top region, counted downwards)
__device__ inline uint32_t queue_pos(uint32_t idx, uint32_t home, uint64_t cap) {
  return idx < home ? idx : (uint32_t)(cap - 1 - (idx - home));
}

// Tallies of one applied step: FP64 atomic scoring per (event, slab), energy
// ledger, optional per-event counts and step log.
struct DevSink {
  double* edep;
  LedgerDev* ledger;
  Ctl* ctl;
  StepRec* log;
  unsigned long long log_cap;
  uint32_t n_slabs;
  bool full, logging;
  // deposits of consecutive steps into the same (event, slab) add up in the
  // lane and reach the tally with one atomic when the cell changes or the
  // lane finishes (summation order of FP64 atomics is unordered anyway)
  size_t acc_cell;
  double acc_dep;
  ExitRec* exits;
  uint64_t exit_cap;

  __device__ void flush() {
    if (acc_dep != 0.0) atomicAdd(&edep[acc_cell], acc_dep);
    acc_dep = 0.0;
  }

  // F: the kernel's optional parts; the per-step records (exits, full
  // ledger, step log) exist only with kFRecord
  template <int F, class R>
  __device__ void apply(int sp, const Trk<R>& t, const StepOut<R>& o, double e_before) {
    if (o.dep != 0.0) {
      const size_t cell = (size_t)t.ev * n_slabs + o.slab;
      if (cell != acc_cell) {
        flush();
        acc_cell = cell;
      }
      acc_dep += o.dep;
    }
    LedgerDev& L = ledger[t.ev];
    if (o.escaped != 0.0) atomicAdd(&L.escaped[0] + sp, o.escaped);
    if (o.killed != 0.0) atomicAdd(&L.killed, o.killed);
    if (o.pair) atomicAdd(&L.n_pair, (uint32_t)o.pair);
    if (o.annih) atomicAdd(&L.n_annih, (uint32_t)o.annih);
    if constexpr ((F & kFRecord) == 0) return;
    if (exit_cap) {
      // the track left the stack: its state at the exit point
      const bool out = o.escaped != 0.0;
      const unsigned long long i = active_append(&ctl->exit_n, out);
      if (out && i < exit_cap) {
        ExitRec& x = exits[i];
        x.event = t.ev;
        x.species = (uint32_t)sp;
        x.ekin = o.escaped;
        x.pos[0] = t.x;
        x.pos[1] = t.y;
        x.pos[2] = t.z;
        x.dir[0] = t.ux;
        x.dir[1] = t.uy;
        x.dir[2] = t.uz;
      }
    }
    if (full) {
      atomicAdd(&L.n_steps, 1ull);
      if (o.clen != 0.0) atomicAdd(&L.charged_len, o.clen);
      if (o.null) atomicAdd(&L.n_null, 1ull);
      if (o.nsec > 0) atomicAdd(&L.n_created[0] + o.sec[0].sp, 1ull);
      if (o.nsec > 1) atomicAdd(&L.n_created[0] + o.sec[1].sp, 1ull);
    }
    if (logging) {
      const unsigned long long ls = atomicAdd(&ctl->log_n, 1ull);
      if (ls < log_cap) {
        StepRec& r = log[ls];
        r.event = t.ev;
        r.species = (uint32_t)sp;
        r.id = t.id;
        r.step = t.n - 1;
        r.slab_after = t.slab;
        r.limiter = o.limiter;
        r.process = o.process;
        r.e_before = e_before;
        r.e_after = t.E;
        r.pos[0] = t.x;
        r.pos[1] = t.y;
        r.pos[2] = t.z;
        r.step_len = o.step_len;
        r.edep = o.dep;
      }
    }
  }
};

// Stage a table block, the slab planes, slab materials and material
// constants in LDS; returns the environment pointing there.
template <class R, int GEO>
__device__ StepEnv<R> stage(const KArgs& a, char* lds_bytes, bool photons) {
  const uint32_t nt = photons ? kGammaTables : kLeptonTables;
  const uint32_t ntab = a.n_mat * nt * a.env.nodes;
  const R* src = static_cast<const R*>(photons ? a.tab_g : a.tab_l);
  R* lds = reinterpret_cast<R*>(lds_bytes);
  for (uint32_t i = threadIdx.x; i < ntab; i += kBlock) lds[i] = src[i];
  double* zp = reinterpret_cast<double*>(lds_bytes + (ntab * sizeof(R) + 7) / 8 * 8);
  // a box geometry reads its volume materials from global memory
  const uint32_t nz = GEO == 1 ? 0u : a.env.n_slabs + 1, nsm = GEO == 1 ? 0u : a.env.n_slabs;
  for (uint32_t i = threadIdx.x; i < nz; i += kBlock) zp[i] = a.zplane[i];
  MatRT* mr = reinterpret_cast<MatRT*>(zp + nz);
  if (threadIdx.x < a.n_mat) mr[threadIdx.x] = a.mat[threadIdx.x];
  uint32_t* sm = reinterpret_cast<uint32_t*>(mr + a.n_mat);
  for (uint32_t i = threadIdx.x; i < nsm; i += kBlock) sm[i] = a.slab_mat[i];
  __syncthreads();
  StepEnv<R> env = retype<R>(a.env);
  env.tg = photons ? lds : nullptr;
  env.tl = photons ? nullptr : lds;
  env.zplane = GEO == 1 ? nullptr : zp;
  env.mat = mr;
  env.elc = a.el_c;
  env.elt = static_cast<const R*>(a.el_tab);
  env.slab_mat = GEO == 1 ? a.slab_mat : sm;
  return env;
}

}  // namespace

// One iteration for the photons (PHOTONS) or for the e-/e+ (otherwise).
//
// Batched lane refill: the lanes of a wave keep stepping their tracks while
// more than refill_below (photons: photon_refill_below) of them are still
// inside a visit.  Then the lanes whose visit ended commit together
// (secondaries, survivors, carried tracks: a few atomics for the whole
// batch) and empty lanes take the next tracks of the queue from a
// per-launch cursor.  Lanes thus stay busy instead of waiting for the
// wave's longest visit, without paying one atomic per track.  The order in
// which tracks are visited does not change any result.

// Minimum resident waves per SIMD the register allocation must allow, per
// kernel, arithmetic type and geometry kind.
#ifndef EMS_WAVES_F64_PHOTON
#define EMS_WAVES_F64_PHOTON 2
#endif
#ifndef EMS_WAVES_F64_LEPTON
#define EMS_WAVES_F64_LEPTON 2
#endif
#ifndef EMS_WAVES_F32_PHOTON
#define EMS_WAVES_F32_PHOTON 3  // fits in 168 registers; at 169 it would drop to 2 waves, 22% slower
#endif
#ifndef EMS_WAVES_F32_LEPTON
#define EMS_WAVES_F32_LEPTON 3  // 168 registers, a few spills: 8% faster than 2 waves of 205
#endif
// Box geometries: photon steps wait on dependent loads of box records; with
// the world volume's boundary distances computed for many lanes at once,
// the photon kernels gain more from running without register spills (FP64
// at 2 waves: 168 VGPRs and 132 spilled at 3; towers photon launch 2.85 ms
// instead of 3.44 ms; FP32 at 3: 2.58 ms instead of 2.90 ms at 4).  More
// waves made the e-/e+ kernels slower; the FP32 one runs at 2 rather than 3
// (towers e-/e+ launch 1.98 ms instead of 2.11 ms; photons at 2: slower).
#ifndef EMS_WAVES_BOX_F64_PHOTON
#define EMS_WAVES_BOX_F64_PHOTON 2
#endif
#ifndef EMS_WAVES_BOX_F64_LEPTON
#define EMS_WAVES_BOX_F64_LEPTON EMS_WAVES_F64_LEPTON
#endif
#ifndef EMS_WAVES_BOX_F32_PHOTON
#define EMS_WAVES_BOX_F32_PHOTON 3
#endif
#ifndef EMS_WAVES_BOX_F32_LEPTON
#define EMS_WAVES_BOX_F32_LEPTON 2
#endif
// The FP32 e-/e+ slab kernels with optional parts (every such variant has
// the field part) need more registers: at 3 waves they spill 100-176 bytes
// per lane, at 2 they spill none.  With 2: the mixed species in a field
// +4.3%, PbWO4 +3.5%, scattering and fluctuations +4.2%, the offload server
// +6.6% (mixed form); the beam's kernel (no optional parts) keeps 3.
#ifndef EMS_WAVES_F32_LEPTON_FIELD
#define EMS_WAVES_F32_LEPTON_FIELD 2
#endif
template <bool PHOTONS, class R, int GEO, int F = 0>
constexpr int visit_waves() {
  if (!PHOTONS && GEO == 0 && sizeof(R) == 4 && (F & kFField) != 0) return EMS_WAVES_F32_LEPTON_FIELD;
  if (GEO == 1)
    return sizeof(R) == 8 ? (PHOTONS ? EMS_WAVES_BOX_F64_PHOTON : EMS_WAVES_BOX_F64_LEPTON)
                          : (PHOTONS ? EMS_WAVES_BOX_F32_PHOTON : EMS_WAVES_BOX_F32_LEPTON);
  return sizeof(R) == 8 ? (PHOTONS ? EMS_WAVES_F64_PHOTON : EMS_WAVES_F64_LEPTON)
                        : (PHOTONS ? EMS_WAVES_F32_PHOTON : EMS_WAVES_F32_LEPTON);
}
template <bool PHOTONS, class R, int GEO, int F>
__global__ __launch_bounds__(kBlock, (visit_waves<PHOTONS, R, GEO, F>())) void k_visit(KArgs a) {
  extern __shared__ double lds_words[];
  char* lds = reinterpret_cast<char*>(lds_words);
  Ctl* ctl = a.ctl;
  const uint32_t cur = ctl->cur;
  const uint32_t h0 = ctl->n_home[0], h1 = ctl->n_home[1], h2 = ctl->n_home[2];
  const uint32_t n0 = h0 + ctl->n_sec[0], n1 = h1 + ctl->n_sec[1], n2 = h2 + ctl->n_sec[2];
  constexpr bool kShort = (F & kFShort) != 0;
  const uint32_t ns = kShort ? ctl->n_short : 0u;
  // the e-/e+ launch also takes the tracks the short launch spilled
  const uint32_t np_raw = (PHOTONS || !(F & kFShort)) ? 0u : ctl->n_spill;
  const uint32_t np = (uint64_t)np_raw < a.cap_p ? np_raw : (uint32_t)a.cap_p;
  const uint32_t nmine = PHOTONS ? n0 : n1 + n2 + np;
  const uint32_t need = (nmine + kBlock - 1) / kBlock;
  const bool work = blockIdx.x < need && ctl->error == 0;
  constexpr int KIND = PHOTONS ? 0 : 1;

  if (work) {
    const StepEnv<R> env = stage<R, GEO>(a, lds, PHOTONS);
    const uint32_t nxt = cur ^ 1u;
    const int max_visit = (int)(PHOTONS ? a.photon_steps_per_visit : a.steps_per_visit);
    const uint32_t refill_below = PHOTONS ? a.photon_refill_below : a.refill_below;
    // secondary slots per species that leave room for all survivors
    const Plan plan = append_plan<kShort>(a, n0, n1, n2, ns);
    const uint32_t lim0 = plan.lim[0], lim1 = plan.lim[1], lim2 = plan.lim[2];
    // wave-private append ranges (uniform): secondaries and home, per
    // species, and the next short buffer
    uint32_t slo[3] = {0, 0, 0}, shi[3] = {0, 0, 0}, hlo[3] = {0, 0, 0}, hhi[3] = {0, 0, 0};
    uint32_t sslo = 0, sshi = 0;
    // short-electron routing: compiled into the kFShort variants only
    const bool shorts = kShort && a.cap_s != 0;
    DevSink sink{a.edep, a.ledger, ctl, a.log, a.log_cap, a.env.n_slabs,
                 (a.flags & kFlagFullLedger) != 0, (a.flags & kFlagSteplog) != 0, 0, 0.0,
                 a.exits, a.exit_cap};
    uint32_t* cursor = &ctl->cursor[PHOTONS ? 0 : 1];
    const bool track_live = (F & kFRecord) && (a.flags & kFlagEventLive) != 0;

    bool has = false;   // lane holds a track (inside a visit or waiting to commit)
    bool fin = false;   // its visit ended; outputs wait for the batch commit
    bool held = false;  // the visit's last step is not yet applied to the tallies
    bool drained = false;
    uint32_t chunk_lo = 0, chunk_hi = 0;  // queue indices held by this wave (uniform)
    int sp = PHOTONS ? 0 : 1;
    Trk<R> t, before;
    VisitState<R> vs;
    StepOut<R> o;
    o.nsec = 0;
    uint32_t visits_e = 0, visits_p = 0, steps_e = 0, steps_p = 0, carried_n = 0;
    uint32_t made0 = 0, made1 = 0, made2 = 0, made_s = 0;
    uint32_t kept_a = 0, kept_b = 0;  // home records written (own species; e+)
    // Box geometries: a step that starts in the world volume needs the
    // nearest box along the track, a walk of the hierarchy that costs the
    // whole wave as much as many ordinary steps however few lanes take it.
    // Such lanes wait (world_wait), also across batches, until kWorldBatch
    // of them do or no other lane steps; then the wave computes their
    // distances together (world_ready, world_pre) and they take their steps
    // with them.
    bool world_ready = false;
    GeoPre world_pre{0.0, Face{0, 0.0, 0, -1}};
    // (charged tracks in a field search their boundary along the helix
    // within their own step limit: they take no straight-line distance)
    const bool world_batch = PHOTONS || !((F & kFField) && env.bz != 0.0);
    for (;;) {
      bool world_wait = false;
      if constexpr (GEO == 1)
        world_wait = world_batch && has && !fin && !world_ready && (uint32_t)t.slab == env.nav.n_boxes;
      uint32_t stepping = (uint32_t)__popcll(__ballot(has && !fin && !world_wait));
      if constexpr (GEO == 1) {
        const uint32_t nw = (uint32_t)__popcll(__ballot(world_wait));
        if (nw && (nw >= kWorldBatch || stepping == 0)) {
          if (world_wait) {
            const double p[3] = {t.x, t.y, t.z}, u[3] = {(double)t.ux, (double)t.uy, (double)t.uz};
            world_pre.s = box_distance(env.nav, t.slab, p, u, world_pre.fc);
            world_ready = true;
            world_wait = false;
          }
          stepping += nw;
        }
      }
      // batch point: few lanes still stepping (or none, once the queue is drained)
      if (stepping <= (drained ? 0u : refill_below)) {
        // (0) e-/e+: while the queue still has tracks, interactions are
        // sampled only once at least interact_min lanes wait for one (each
        // sampler costs the wave one pass however few lanes use it); until
        // then those lanes are parked: they keep their tracks and take no
        // part in this batch.  A wave whose lanes are all parked samples
        // them, so every wave ends (interact_min <= 64).
        const uint32_t npend = PHOTONS ? 0u : (uint32_t)__popcll(__ballot(fin && o.pending));
        const bool parked = !PHOTONS && !drained && npend < a.interact_min && fin && o.pending;
        const bool done = fin && !parked;  // visits this batch finishes
        // (1) prefetch the records of the tracks that the lanes free after
        // this batch will take; the loads are in flight during (2)
        // a parent that survives its interaction keeps its lane and goes on
        // stepping in this launch while it has steps left
        const bool will_continue = done && o.pending && parent_survives(o.process) && vs.steps < max_visit;
        const bool want = (!has || (done && !will_continue)) && !drained;
        bool got = false;
        int nsp = PHOTONS ? 0 : 1;
        uint32_t nw = kDeadRecord;
        Trk<R> nt;
        if (__ballot(want) != 0) {
          const uint32_t i = take_next(cursor, want, chunk_lo, chunk_hi);
          got = want && i < nmine;
          drained = __ballot(want && i >= nmine) != 0;
          if (got) {
            uint32_t idx = i, home = PHOTONS ? h0 : h1;
            if (!PHOTONS && i >= n1) {
              nsp = 2;
              idx = i - n1;
              home = h2;
            }
            const bool spilled = !PHOTONS && (F & kFShort) && i >= n1 + n2;  // an e- from the spill buffer
            if (spilled) nsp = 1;
            const uint32_t pos = spilled ? i - n1 - n2 : queue_pos(idx, home, a.cap);
            const Queue<R> src = spilled ? short_view<R>(a, 2u) : queue_view<R>(a.qbase, a.cap, cur, (uint32_t)nsp);
            nw = src.ns[pos];
            nt.ev = src.ev[pos];
            nt.key = src.key[pos];
            nt.x = src.x[pos];
            nt.y = src.y[pos];
            nt.z = src.z[pos];
            nt.ux = src.ux[pos];
            nt.uy = src.uy[pos];
            nt.uz = src.uz[pos];
            nt.E = src.E[pos];
            nt.id = src.id[pos];
          }
        }
        // (2) the interactions selected by the lanes' last steps, sampled
        // together (one pass through each sampler the wave needs)
        if (done && o.pending) interact<KIND, F>(env, t, o);
        // (3) the prefetched records have arrived; waiting here, before any
        // store of this batch is issued, keeps later uses of their fields
        // from waiting on those stores (vector memory completes in order)
        __builtin_amdgcn_s_waitcnt(kWaitVmem);
        bool take = got && nw != kDeadRecord;  // dead: refused secondary or unused chunk end
        nt.slab = (int32_t)(nw & ((1u << a.vol_bits) - 1u));
        nt.n = nw >> a.vol_bits;
        // a record that would index outside the tallies or the slab stack
        // is reported, never used
        if (take && (nt.slab >= (int32_t)a.env.n_slabs || nt.ev >= a.max_events)) {
          atomicOr(&ctl->error, kErrCorrupt);
          take = false;
        }
        // (4) commit the finished visits: reserve first, then write
        if (__ballot(done) != 0) {
          // secondaries into the top regions (a step commits only if all of
          // its secondaries fit), then survivors or carried tracks
          // e- secondaries below short_E go to the next short buffer
          const bool s0 = shorts && done && o.nsec > 0 && o.sec[0].sp == kElectron && o.sec[0].E < a.short_E;
          const bool s1 = shorts && done && o.nsec > 1 && o.sec[1].sp == kElectron && o.sec[1].E < a.short_E;
          uint32_t d[3];
#pragma unroll
          for (int q = 0; q < 3; ++q)
            d[q] = (done && o.nsec > 0 && o.sec[0].sp == q && !s0 ? 1u : 0u) +
                   (done && o.nsec > 1 && o.sec[1].sp == q && !s1 ? 1u : 0u);
          const uint32_t ds = (s0 ? 1u : 0u) + (s1 ? 1u : 0u);
          uint32_t slot[3];
          Take tk[3];
          bool fits = true;
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            slot[q] = take_slots(&ctl->next_sec[q], d[q], plan.chunk[q], slo[q], shi[q], tk[q]);
            const uint32_t lim = q == 0 ? lim0 : (q == 1 ? lim1 : lim2);
            if (d[q] && slot_of(tk[q], slot[q] + d[q] - 1) >= lim) fits = false;
            if (d[q] > 1 && slot_of(tk[q], slot[q]) >= lim) fits = false;
          }
          uint32_t slot_s = 0;
          Take tks{0, 0, 0};
          if (shorts) {
            slot_s = take_slots(&ctl->next_short, ds, plan.chunk_s, sslo, sshi, tks);
            if (ds && slot_of(tks, slot_s + ds - 1) >= plan.lim_s) fits = false;
            if (ds > 1 && slot_of(tks, slot_s) >= plan.lim_s) fits = false;
          }
          const bool pending = done && o.nsec > 0;
          const bool commit = pending && fits;
          const bool apply_now = commit || (done && held && o.nsec == 0);
          const bool carry = pending && !commit;  // back to the state before the last step
          const bool alive = done && (carry ? before.slab >= 0 : t.slab >= 0);
          const bool cont = alive && !carry && will_continue;  // stays in the lane
          const bool keep = alive && !cont;                    // written to the next queue
          // home slots (one counter per call: a wave may hold e- and e+)
          uint32_t hs = 0;
#pragma unroll
          for (int q = PHOTONS ? 0 : 1; q < (PHOTONS ? 1 : 3); ++q) {
            const bool mine = keep && sp == q;
            Take th;
            const uint32_t hx = take_slots(&ctl->next_home[q], mine ? 1u : 0u, plan.chunk[q], hlo[q], hhi[q], th);
            if (mine) hs = slot_of(th, hx);
          }
          if (apply_now) {
            sink.apply<F>(sp, t, o, before.E);
            if (sp == 2) ++steps_p;
            else ++steps_e;
            made0 += d[0];
            made1 += d[1];
            made2 += d[2];
            made_s += ds;
          }
          if (carry) ++carried_n;
          if (done && track_live) {
            // net change of the event's live tracks: the visited track ends
            // or stays, committed secondaries join
            const int delta = (alive ? 1 : 0) + (commit ? (int)(d[0] + d[1] + d[2] + ds) : 0) - 1;
            if (delta != 0) atomicAdd(&a.live_ev[t.ev], delta);
          }
#pragma unroll
          for (int q = 0; q < 3; ++q) {
            if (!d[q]) continue;
            const uint32_t lim = q == 0 ? lim0 : (q == 1 ? lim1 : lim2);
            const Queue<R> dq = queue_view<R>(a.qbase, a.cap, nxt, (uint32_t)q);
            uint32_t x = slot[q];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
              if (!(k < o.nsec && o.sec[k].sp == q)) continue;
              const uint32_t sl = slot_of(tk[q], x);
              if (sl < lim) {
                const uint32_t ps = (uint32_t)(a.cap - 1 - sl);
                if (commit) {
                  Trk<R> c;
                  c.x = t.x;
                  c.y = t.y;
                  c.z = t.z;
                  c.ux = o.sec[k].ux;
                  c.uy = o.sec[k].uy;
                  c.uz = o.sec[k].uz;
                  c.E = o.sec[k].E;
                  c.id = o.sec[k].id;
                  c.ev = t.ev;
                  c.key = t.key;
                  c.n = 0;
                  c.slab = o.slab;
                  store_track(dq, ps, c, a.vol_bits);
                } else {
                  dq.ns[ps] = kDeadRecord;  // refused: the next iteration skips this slot
                }
              }
              ++x;
            }
          }
          if (ds) {
            const Queue<R> sq = short_view<R>(a, nxt);
            uint32_t x = slot_s;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
              if (!(k == 0 ? s0 : s1)) continue;
              const uint32_t sl = slot_of(tks, x);
              if (sl < plan.lim_s) {
                if (commit) {
                  Trk<R> c;
                  c.x = t.x;
                  c.y = t.y;
                  c.z = t.z;
                  c.ux = o.sec[k].ux;
                  c.uy = o.sec[k].uy;
                  c.uz = o.sec[k].uz;
                  c.E = o.sec[k].E;
                  c.id = o.sec[k].id;
                  c.ev = t.ev;
                  c.key = t.key;
                  c.n = 0;
                  c.slab = o.slab;
                  store_track(sq, sl, c, a.vol_bits);
                } else {
                  sq.ns[sl] = kDeadRecord;
                }
              }
              ++x;
            }
          }
          if (keep) {
            const Queue<R> dq = queue_view<R>(a.qbase, a.cap, nxt, (uint32_t)sp);
            if (hs >= a.cap) {
              atomicOr(&ctl->error, kErrOverflow);
            } else {
              if (carry) store_track(dq, hs, before, a.vol_bits);
              else store_track(dq, hs, t, a.vol_bits);
              if (sp == 2) ++kept_b;
              else ++kept_a;
            }
          }
          if (done) {
            has = cont;
            fin = false;
            held = false;
            o.nsec = 0;
            o.pending = false;
          }
          // a continuing photon has a new energy and direction
          if (PHOTONS && cont) photon_begin(env, t, vs.pc);
        }
        // (5) the freed lanes take their prefetched tracks
        if (take) {
          t.x = nt.x;
          t.y = nt.y;
          t.z = nt.z;
          t.ux = nt.ux;
          t.uy = nt.uy;
          t.uz = nt.uz;
          t.E = nt.E;
          t.id = nt.id;
          t.ev = nt.ev;
          t.key = nt.key;
          t.n = nt.n;
          t.slab = nt.slab;
          sp = nsp;
          has = true;
          visit_begin<KIND>(env, sp, t, vs);
          world_ready = false;
          if (sp == 2) ++visits_p;
          else ++visits_e;
        }
        if (__ballot(has) == 0) {
          if (drained) break;
          continue;
        }
        // tracks just taken that start in the world wait for a world pass
        if constexpr (GEO == 1)
          world_wait = world_batch && has && !fin && !world_ready && (uint32_t)t.slab == env.nav.n_boxes;
      }

      // one step of every lane inside a visit
      if (has && !fin && !world_wait) {
        before = t;
        const double e0 = t.E;
        fin = visit_step<KIND, R, GEO, F>(env, sp, vs, t, o, max_visit, world_ready ? &world_pre : nullptr);
        world_ready = false;
        held = o.pending;
        if (!held) {
          sink.apply<F>(sp, t, o, e0);
          if (sp == 2) ++steps_p;
          else ++steps_e;
        }
      }
    }

    sink.flush();
    // unused ends of the wave's append ranges hold no track
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const Queue<R> dq = queue_view<R>(a.qbase, a.cap, nxt, (uint32_t)q);
      const uint32_t lim = q == 0 ? lim0 : (q == 1 ? lim1 : lim2);
      const uint32_t send = shi[q] < lim ? shi[q] : lim;
      for (uint32_t x = slo[q] + __lane_id(); x < send; x += 64) dq.ns[a.cap - 1 - x] = kDeadRecord;
      for (uint32_t x = hlo[q] + __lane_id(); x < hhi[q]; x += 64) {
        if (x < a.cap) dq.ns[x] = kDeadRecord;
      }
    }
    if (shorts) {
      const Queue<R> sq = short_view<R>(a, nxt);
      const uint32_t send = sshi < plan.lim_s ? sshi : plan.lim_s;
      for (uint32_t x = sslo + __lane_id(); x < send; x += 64) sq.ns[x] = kDeadRecord;
    }
    // statistics and per-launch progress
    if (PHOTONS) {
      wave_count(&ctl->steps[0], steps_e);
      wave_count(&ctl->visits[0], visits_e);
    } else {
      wave_count(&ctl->steps[1], steps_e);
      wave_count(&ctl->steps[2], steps_p);
      wave_count(&ctl->visits[1], visits_e);
      wave_count(&ctl->visits[2], visits_p);
    }
    wave_count(&ctl->deferred, carried_n);
    wave_count(&ctl->created[0], made0);
    wave_count(&ctl->created[1], made1 + made_s);
    wave_count(&ctl->created[2], made2);
    wave_count(&ctl->made_by[PHOTONS ? 0 : 1], made0 + made1 + made2 + made_s);
    if (shorts) wave_count(&ctl->next_short_real, made_s);
    wave_count(&ctl->next_real[0], made0 + (PHOTONS ? kept_a : 0u));
    wave_count(&ctl->next_real[1], made1 + (PHOTONS ? 0u : kept_a));
    wave_count(&ctl->next_real[2], made2 + kept_b);
    const uint32_t c = wave_sum(steps_e + steps_p), k = wave_sum(carried_n);
    if (__lane_id() == 0) {
      if (c) atomicAdd(&ctl->commits, c);
      if (k) atomicAdd(&ctl->carried, k);
    }
  }

  if (PHOTONS) return;

  // the last block of the e-/e+ launch publishes the next iteration (the
  // photon launch of this iteration finished before this launch started)
  __shared__ uint32_t last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(&ctl->blocks_done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __threadfence();
    const uint32_t r0 = ctl->n_real[0], r1 = ctl->n_real[1] + (kShort ? ctl->n_short_real : 0u), r2 = ctl->n_real[2];
    if (a.flags & kFlagProfile) {
      if (ctl->iteration < a.profile_cap) {
        a.profile[(size_t)ctl->iteration * 3 + 0] = r0;
        a.profile[(size_t)ctl->iteration * 3 + 1] = r1;
        a.profile[(size_t)ctl->iteration * 3 + 2] = r2;
      }
    }
    if (r0 + r1 + r2 > 0) ctl->iteration += 1;
    const uint32_t commits = atomicAdd(&ctl->commits, 0u), carried = atomicAdd(&ctl->carried, 0u);
    if (carried > 0 && commits == 0) ctl->error |= kErrStall;  // nothing can move: queues too small
    const uint32_t srv = kShort ? atomicAdd(&ctl->next_short_real, 0u) : 0u;
    uint32_t live = srv;
    for (int q = 0; q < 3; ++q) live += atomicAdd(&ctl->next_real[q], 0u);
    const Plan plan = append_plan<kShort>(a, n0, n1, n2, ns);
    for (int q = 0; q < 3; ++q) {
      const uint32_t lim = plan.lim[q];
      const uint32_t hv = atomicAdd(&ctl->next_home[q], 0u);
      uint32_t sv = atomicAdd(&ctl->next_sec[q], 0u);
      sv = sv < lim ? sv : lim;
      const uint32_t rv = atomicAdd(&ctl->next_real[q], 0u);
      // with no live track left the dead slots need no visit
      ctl->n_home[q] = live ? hv : 0u;
      ctl->n_sec[q] = live ? sv : 0u;
      ctl->n_real[q] = rv;
      ctl->next_home[q] = 0;
      ctl->next_sec[q] = 0;
      ctl->next_real[q] = 0;
      ctl->peak[q] = rv > ctl->peak[q] ? rv : ctl->peak[q];
    }
    if constexpr (kShort) {
      // the next short buffer becomes the current one
      const uint32_t sv = atomicAdd(&ctl->next_short, 0u);
      ctl->n_short = live ? (sv < plan.lim_s ? sv : plan.lim_s) : 0u;
      ctl->n_short_real = srv;
      ctl->next_short = 0;
      ctl->next_short_real = 0;
      ctl->n_spill = 0;
      ctl->cursor_s = 0;
      ctl->peak[1] = ctl->n_real[1] + srv > ctl->peak[1] ? ctl->n_real[1] + srv : ctl->peak[1];
    }
    ctl->live = live;
    ctl->commits = 0;
    ctl->carried = 0;
    ctl->cursor[0] = 0;
    ctl->cursor[1] = 0;
    ctl->cur = cur ^ 1u;
    ctl->blocks_done = 0;
    __threadfence();
  }
}

// Short electrons.  Most e- secondaries of a shower are slow (Compton and
// photo-electrons, delta rays) and end in their first step, ranged out.
// In the e-/e+ launch each of them costs a lane a record load, one step and
// a commit in a wave whose other lanes follow long tracks; here a launch of
// its own, at the start of the iteration, gives every lane one such track:
// one step, its tallies, and the survivor (if any) appended to the next e-
// queue as any e-/e+ survivor.  A track whose first step selects a discrete
// interaction is handed unchanged to this iteration's e-/e+ launch (spill
// buffer), which takes the same step again and samples the interaction
// there: every step still draws from its own (id, step) stream, so results
// and the iteration of every step are those of the e-/e+ launch.
// (without optional parts the step and a prefetched record fit 3 resident
// waves per SIMD in FP64, 5 in FP32; with them 3 and 4; in box geometries
// 2 and 3)
#ifndef EMS_WAVES_F64_SHORT
#define EMS_WAVES_F64_SHORT 3
#endif
#ifndef EMS_WAVES_F32_SHORT
#define EMS_WAVES_F32_SHORT 5
#endif
template <class R, int GEO, int F>
constexpr int short_waves() {
  if (GEO == 1) return sizeof(R) == 8 ? 2 : 3;  // box navigation needs more registers
  return sizeof(R) == 8 ? (F == 0 ? EMS_WAVES_F64_SHORT : 3) : (F == 0 ? EMS_WAVES_F32_SHORT : 4);
}
template <class R, int GEO, int F>
__global__ __launch_bounds__(kBlock, (short_waves<R, GEO, F>())) void k_short(KArgs a) {
  extern __shared__ double lds_words[];
  char* lds = reinterpret_cast<char*>(lds_words);
  Ctl* ctl = a.ctl;
  const uint32_t cur = ctl->cur;
  const uint32_t ns = ctl->n_short;
  if (blockIdx.x >= (ns + kBlock - 1) / kBlock || ctl->error != 0) return;
  const uint32_t n0 = ctl->n_home[0] + ctl->n_sec[0], n1 = ctl->n_home[1] + ctl->n_sec[1];
  const uint32_t n2 = ctl->n_home[2] + ctl->n_sec[2];
  const StepEnv<R> env = stage<R, GEO>(a, lds, false);
  const Plan plan = append_plan<true>(a, n0, n1, n2, ns);
  DevSink sink{a.edep, a.ledger, ctl, a.log, a.log_cap, a.env.n_slabs,
               (a.flags & kFlagFullLedger) != 0, (a.flags & kFlagSteplog) != 0, 0, 0.0,
               a.exits, a.exit_cap};
  const bool track_live = (F & kFRecord) && (a.flags & kFlagEventLive) != 0;
  const Queue<R> src = short_view<R>(a, cur);
  const Queue<R> spill = short_view<R>(a, 2u);
  const Queue<R> dst = queue_view<R>(a.qbase, a.cap, cur ^ 1u, (uint32_t)kElectron);
  // wave-private append ranges (uniform): next e- home, spill buffer
  uint32_t hlo = 0, hhi = 0, plo = 0, phi = 0;
  // spill appends: all waves' unused chunk ends fit in the spill buffer's
  // room beyond cap_s (at most ns <= cap_s tracks spill)
  uint32_t chunk_p = plan.chunk[1] < 64u ? plan.chunk[1] : 64u;
  while (chunk_p > 1 && (uint64_t)a.waves_s * chunk_p > a.cap_p - a.cap_s) chunk_p >>= 1;
  uint32_t steps = 0, loads = 0, kept = 0;
  // the record of the lane's next track is loaded while the current one
  // steps (the step reads only LDS, so nothing waits for those loads early)
  auto load = [&](uint32_t i, Trk<R>& t, uint32_t& w) {
    w = kDeadRecord;
    if (i < ns) {
      w = src.ns[i];
      t.x = src.x[i];
      t.y = src.y[i];
      t.z = src.z[i];
      t.ux = src.ux[i];
      t.uy = src.uy[i];
      t.uz = src.uz[i];
      t.E = src.E[i];
      t.id = src.id[i];
      t.ev = src.ev[i];
      t.key = src.key[i];
    }
  };
  const uint32_t stride = gridDim.x * kBlock;
  Trk<R> t;
  uint32_t w;
  load(blockIdx.x * kBlock + threadIdx.x, t, w);
  for (uint32_t base = blockIdx.x * kBlock; base < ns; base += stride) {
    Trk<R> tn;
    uint32_t wn;
    load(base + stride + threadIdx.x, tn, wn);
    bool has = w != kDeadRecord;
    t.slab = (int32_t)(w & ((1u << a.vol_bits) - 1u));
    t.n = w >> a.vol_bits;
    if (has && (t.slab >= (int32_t)a.env.n_slabs || t.ev >= a.max_events)) {
      atomicOr(&ctl->error, kErrCorrupt);
      has = false;
    }
    const Trk<R> first = t;
    StepOut<R> o;
    o.nsec = 0;
    bool to_spill = false, alive = false;
    if (has) {
      ++loads;
      clear_out(t, o);
      lepton_step<R, GEO, F>(env, false, t, o);
      if (o.pending) {
        to_spill = true;
      } else {
        watchdog(env, t, o);
        sink.apply<F>(kElectron, t, o, first.E);
        ++steps;
        alive = t.slab >= 0;
        if (track_live && !alive) atomicAdd(&a.live_ev[t.ev], -1);
      }
    }
    Take th, tp;
    const uint32_t hx = take_slots(&ctl->next_home[1], alive ? 1u : 0u, plan.chunk[1], hlo, hhi, th);
    const uint32_t px = take_slots(&ctl->n_spill, to_spill ? 1u : 0u, chunk_p, plo, phi, tp);
    if (alive) {
      const uint32_t hs = slot_of(th, hx);
      if (hs >= a.cap) {
        atomicOr(&ctl->error, kErrOverflow);
      } else {
        store_track(dst, hs, t, a.vol_bits);
        ++kept;
      }
    }
    if (to_spill) {
      const uint32_t ps = slot_of(tp, px);
      if (ps >= a.cap_p) atomicOr(&ctl->error, kErrOverflow);
      else store_track(spill, ps, first, a.vol_bits);
    }
    t = tn;
    w = wn;
  }
  sink.flush();
  for (uint32_t x = hlo + __lane_id(); x < hhi; x += 64) {
    if (x < a.cap) dst.ns[x] = kDeadRecord;
  }
  for (uint32_t x = plo + __lane_id(); x < phi; x += 64) {
    if (x < a.cap_p) spill.ns[x] = kDeadRecord;
  }
  wave_count(&ctl->steps[1], steps);
  wave_count(&ctl->steps_s, steps);
  wave_count(&ctl->visits[1], loads);
  wave_count(&ctl->next_real[1], kept);
  const uint32_t c = wave_sum(steps);
  if (__lane_id() == 0 && c) atomicAdd(&ctl->commits, c);
}

#ifndef EMS_SLAB_F32_TU
// Zero `words` 8-byte words at p and then `ntail` single bytes at tail, with
// plain vector stores (grid-stride).  The library clears its device memory
// with this kernel instead of memset nodes, which a caller capturing the
// stream into a graph could not rely on.
__global__ __launch_bounds__(kBlock) void k_fill_zero(unsigned long long* p, uint64_t words, unsigned char* tail,
                                                      uint32_t ntail) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < words; i += stride) p[i] = 0ull;
  if (blockIdx.x == 0 && threadIdx.x < ntail) tail[threadIdx.x] = 0;
}

// Atomic-throughput probe: FP64 adds of 1.0, the instruction of the deposit
// tallies, to cells drawn by a fixed hash of the op index (grid-stride).
__global__ __launch_bounds__(kBlock) void k_atomic_probe(double* cells, uint64_t n_cells, uint64_t n_ops) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n_ops; i += stride) {
    uint64_t h = i * 0x9E3779B97F4A7C15ull;
    h ^= h >> 29;
    h *= 0xBF58476D1CE4E5B9ull;
    h ^= h >> 32;
    atomicAdd(&cells[h % n_cells], 1.0);
  }
}

// Injection: prepared tracks appended to the home regions of the current
// queues.
template <class R>
__global__ __launch_bounds__(kBlock) void k_inject(KArgs a, const InjRec* rec, uint32_t n) {
  Ctl* ctl = a.ctl;
  const uint32_t cur = ctl->cur;
  for (uint32_t base = blockIdx.x * kBlock; base < n; base += gridDim.x * kBlock) {
    const uint32_t i = base + threadIdx.x;
    const bool active = i < n;
    InjRec r{};
    if (active) r = rec[i];
    for (int qs = 0; qs < 3; ++qs) {
      const uint32_t cnt = (active && (int)r.sp == qs) ? 1u : 0u;
      const uint32_t slot = wave_reserve(&ctl->n_home[qs], cnt);
      const bool fits = cnt && slot + ctl->n_sec[qs] < a.cap;
      wave_count(&ctl->n_real[qs], fits ? 1u : 0u);
      if (!cnt) continue;
      if (!fits) {
        atomicOr(&ctl->error, kErrOverflow);
        continue;
      }
      Trk<R> t;
      t.x = r.x;
      t.y = r.y;
      t.z = r.z;
      t.ux = (R)r.ux;
      t.uy = (R)r.uy;
      t.uz = (R)r.uz;
      t.E = r.E;
      t.id = r.id;
      t.ev = r.ev;
      t.key = r.key;
      t.n = 0;
      t.slab = r.slab;
      store_track(queue_view<R>(a.qbase, a.cap, cur, (uint32_t)qs), slot, t, a.vol_bits);
      if (a.flags & kFlagEventLive) atomicAdd(&a.live_ev[r.ev], 1);
    }
  }
}

// Zero the deposits, ledger and live counter of the listed rows (one block
// per row, grid-stride over the list).
__global__ __launch_bounds__(kBlock) void k_reset_rows(KArgs a, const uint32_t* rows, uint32_t n) {
  for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const uint32_t r = rows[i];
    if (r >= a.max_events) continue;
    double* e = a.edep + (size_t)r * a.env.n_slabs;
    for (uint32_t k = threadIdx.x; k < a.env.n_slabs; k += kBlock) e[k] = 0.0;
    unsigned long long* l = reinterpret_cast<unsigned long long*>(a.ledger + r);
    for (uint32_t k = threadIdx.x; k < sizeof(LedgerDev) / 8; k += kBlock) l[k] = 0ull;
    if (threadIdx.x == 0) a.live_ev[r] = 0;
  }
}

// Copy the deposits and ledger of the listed rows to a compact staging area:
// entry i holds n_slabs doubles, then the row's ledger.
__global__ __launch_bounds__(kBlock) void k_gather_rows(KArgs a, const uint32_t* rows, uint32_t n, char* out) {
  const size_t stride = (size_t)a.env.n_slabs * 8 + sizeof(LedgerDev);
  for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
    const uint32_t r = rows[i];
    if (r >= a.max_events) continue;
    double* o = reinterpret_cast<double*>(out + i * stride);
    const double* e = a.edep + (size_t)r * a.env.n_slabs;
    for (uint32_t k = threadIdx.x; k < a.env.n_slabs; k += kBlock) o[k] = e[k];
    unsigned long long* lo = reinterpret_cast<unsigned long long*>(o + a.env.n_slabs);
    const unsigned long long* li = reinterpret_cast<const unsigned long long*>(a.ledger + r);
    for (uint32_t k = threadIdx.x; k < sizeof(LedgerDev) / 8; k += kBlock) lo[k] = li[k];
  }
}

// live count after injection (one thread)
__global__ void k_census(KArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctl* c = a.ctl;
    uint32_t live = c->n_short_real;
    for (int q = 0; q < 3; ++q) {
      const uint32_t n = c->n_real[q] + (q == 1 ? c->n_short_real : 0u);
      c->peak[q] = n > c->peak[q] ? n : c->peak[q];
      live += c->n_real[q];
    }
    c->live = live;
  }
}

#endif  // EMS_SLAB_F32_TU

// Kernel variants: the optional parts each kernel is built with.  The
// e-/e+ kernel of a slab stack comes without any, with the field and the
// records (mixed-species runs in a field, the offload server) or with all;
// the photon kernels and the box-geometry e-/e+ kernels without any or with
// all.  A context launches the smallest variant that covers its
// configuration (KArgs::feat_g, feat_l).
template <bool PHOTONS, class R, int GEO>
const void* visit_fn(uint32_t feat) {
  if (feat == 0) return reinterpret_cast<const void*>(&k_visit<PHOTONS, R, GEO, 0>);
  if (feat == kFShort) return reinterpret_cast<const void*>(&k_visit<PHOTONS, R, GEO, kFShort>);
  if constexpr (!PHOTONS && GEO == 0) {
    if (feat == (kFField | kFRecord))
      return reinterpret_cast<const void*>(&k_visit<PHOTONS, R, GEO, kFField | kFRecord>);
    if (feat == (kFField | kFRecord | kFShort))
      return reinterpret_cast<const void*>(&k_visit<PHOTONS, R, GEO, kFField | kFRecord | kFShort>);
  }
  if (feat == (kFAll & ~kFShort)) return reinterpret_cast<const void*>(&k_visit<PHOTONS, R, GEO, kFAll & ~kFShort>);
  return reinterpret_cast<const void*>(&k_visit<PHOTONS, R, GEO, kFAll>);
}
// the short launch takes the e-/e+ launch's optional parts (its own work is
// the short path, so the routing bit does not apply to it)
template <class R, int GEO>
const void* short_fn(uint32_t feat) {
  feat &= ~(uint32_t)kFShort;
  if (feat == 0) return reinterpret_cast<const void*>(&k_short<R, GEO, 0>);
  if constexpr (GEO == 0) {
    if (feat == (kFField | kFRecord)) return reinterpret_cast<const void*>(&k_short<R, GEO, kFField | kFRecord>);
  }
  return reinterpret_cast<const void*>(&k_short<R, GEO, kFAll>);
}
template <class R, int GEO>
const void* kernel_of(const KArgs& a, int which) {
  return which == 0 ? visit_fn<true, R, GEO>(a.feat_g)
                    : (which == 1 ? visit_fn<false, R, GEO>(a.feat_l) : short_fn<R, GEO>(a.feat_l));
}
#ifdef EMS_SLAB_F32_TU
const void* kernel_of_slab_f32(const KArgs& a, int which) { return kernel_of<float, 0>(a, which); }
#else
// The mixed-form kernels of the slab stack come from a translation unit of
// their own (ems_kernels_slab_f32.hip), built with another instruction
// scheduler (see build.py).
const void* kernel_of_slab_f32(const KArgs& a, int which);
// which: 0 photon, 1 e-/e+, 2 short-electron launch
const void* kernel_for(const KArgs& a, int which) {
  if (a.geo == 1) return a.precision ? kernel_of<float, 1>(a, which) : kernel_of<double, 1>(a, which);
  return a.precision ? kernel_of_slab_f32(a, which) : kernel_of<double, 0>(a, which);
}
hipError_t launch_kernel(const KArgs& a, int which, uint32_t blocks, hipStream_t s) {
  KArgs arg = a;
  void* args[] = {&arg};
  return hipLaunchKernel(kernel_for(a, which), dim3(blocks), dim3(kBlock), args, which == 0 ? a.lds_g : a.lds_l, s);
}
hipError_t launch_short(const KArgs& a, uint32_t blocks, hipStream_t s) { return launch_kernel(a, 2, blocks, s); }
// one iteration is the short-electron launch, the photon launch and the
// e-/e+ launch
hipError_t launch_visit(const KArgs& a, bool photons, uint32_t blocks, hipStream_t s) {
  return launch_kernel(a, photons ? 0 : 1, blocks, s);
}
hipError_t launch_inject(const KArgs& a, const InjRec* rec, uint32_t n, hipStream_t s) {
  const uint32_t want = (n + kBlock - 1) / kBlock;
  const uint32_t blocks = n == 0 ? 1 : (want < 4096 ? want : 4096);
  if (a.precision) hipLaunchKernelGGL(k_inject<float>, dim3(blocks), dim3(kBlock), 0, s, a, rec, n);
  else hipLaunchKernelGGL(k_inject<double>, dim3(blocks), dim3(kBlock), 0, s, a, rec, n);
  return hipGetLastError();
}
hipError_t launch_reset_rows(const KArgs& a, const uint32_t* rows, uint32_t n, hipStream_t s) {
  const uint32_t blocks = n == 0 ? 1 : (n < 1024 ? n : 1024);
  hipLaunchKernelGGL(k_reset_rows, dim3(blocks), dim3(kBlock), 0, s, a, rows, n);
  return hipGetLastError();
}
hipError_t launch_gather_rows(const KArgs& a, const uint32_t* rows, uint32_t n, char* out, hipStream_t s) {
  const uint32_t blocks = n == 0 ? 1 : (n < 1024 ? n : 1024);
  hipLaunchKernelGGL(k_gather_rows, dim3(blocks), dim3(kBlock), 0, s, a, rows, n, out);
  return hipGetLastError();
}
hipError_t launch_atomic_probe(double* cells, uint64_t n_cells, uint64_t n_ops, hipStream_t s) {
  const uint64_t want = (n_ops + kBlock - 1) / kBlock;
  const uint32_t blocks = (uint32_t)(want < 16384 ? (want ? want : 1) : 16384);
  hipLaunchKernelGGL(k_atomic_probe, dim3(blocks), dim3(kBlock), 0, s, cells, n_cells, n_ops);
  return hipGetLastError();
}
hipError_t launch_fill_zero(void* p, uint64_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  if (reinterpret_cast<uintptr_t>(p) % 8) return hipErrorInvalidValue;
  const uint64_t words = bytes / 8;
  const uint64_t want = (words + kBlock - 1) / kBlock;
  const uint32_t blocks = (uint32_t)(want == 0 ? 1 : (want < 8192 ? want : 8192));
  hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(kBlock), 0, s, static_cast<unsigned long long*>(p), words,
                     static_cast<unsigned char*>(p) + words * 8, (uint32_t)(bytes % 8));
  return hipGetLastError();
}
hipError_t launch_census(const KArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_census, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}
// blocks of each visit kernel that fit on one CU (registers and LDS), for
// the variants the context launches
hipError_t visit_occupancy(const KArgs& a, int* per_cu_g, int* per_cu_l, int* per_cu_s) {
  int* out[3] = {per_cu_g, per_cu_l, per_cu_s};
  for (int w = 0; w < 3; ++w) {
    const void* f = kernel_for(a, w);
    const uint32_t lds = w == 0 ? a.lds_g : a.lds_l;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(out[w], f, kBlock, lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}
#endif  // EMS_SLAB_F32_TU

}  // namespace ems
