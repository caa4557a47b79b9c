// ems_kernels.hip -- gfx950 kernels of the transport loop.
//
// The paper steps the whole track population once per iteration with one
// kernel per species in three streams, appending secondaries to per-species
// "next" index arrays with an atomic counter and swapping current/next after
// each step (section 3).  On MI355X this is one fused launch per iteration:
//  - threads map to a concatenated index space [gamma | e- | e+], so a wave
//    almost always holds one species and no stream synchronisation is needed;
//  - the queues hold the tracks themselves (SoA, coalesced), and survivors
//    are rewritten compactly each step, so slots are reused by construction;
//  - appends are aggregated per wave (ballot + popcount prefix, one atomic
//    per wave and species);
//  - cross-section tables, slab planes and materials are staged in LDS;
//  - secondaries are reserved against a per-species limit that always leaves
//    room for every survivor; a track whose secondaries do not fit is carried
//    unstepped, so a full queue defers work instead of losing it;
//  - the last block to finish swaps the queues, so a chain of launches needs
//    no host round trip.
#include <hip/hip_runtime.h>

#include "ems_device.hpp"

namespace ems {

namespace {

constexpr int kBlock = 256;

__device__ inline uint64_t lanes_below() { return __lanemask_lt(); }

// Reserve `count` (0..3) consecutive slots per lane in an append counter with
// one atomic per wave; returns this lane's first slot.
__device__ inline uint32_t wave_reserve(uint32_t* counter, uint32_t count) {
  const uint64_t b0 = __ballot(count & 1u);
  const uint64_t b1 = __ballot((count >> 1) & 1u);
  const uint32_t total = (uint32_t)(__popcll(b0) + 2 * __popcll(b1));
  if (total == 0) return 0;
  const uint64_t lt = lanes_below();
  const uint32_t prefix = (uint32_t)(__popcll(b0 & lt) + 2 * __popcll(b1 & lt));
  const uint64_t any = b0 | b1;
  const int leader = __ffsll((unsigned long long)any) - 1;
  uint32_t base = 0;
  if ((int)__lane_id() == leader) base = atomicAdd(counter, total);
  base = __shfl(base, leader);
  return base + prefix;
}

// sum over the wave of a per-lane count, one atomic by lane 0
__device__ inline void wave_count(unsigned long long* counter, uint32_t v) {
  uint32_t s = v;
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if (__lane_id() == 0 && s) atomicAdd(counter, (unsigned long long)s);
}

__device__ inline void store_track(const Queue& q, uint32_t i, const Trk& t) {
  q.x[i] = t.x;
  q.y[i] = t.y;
  q.z[i] = t.z;
  q.ux[i] = t.ux;
  q.uy[i] = t.uy;
  q.uz[i] = t.uz;
  q.E[i] = t.E;
  q.id[i] = t.id;
  q.ev[i] = t.ev;
  q.n[i] = t.n;
  q.slab[i] = t.slab;
}

// position of the idx-th track of a queue with `home` tracks in the bottom
// region (the rest are in the top region, counted downwards)
__device__ inline uint32_t queue_pos(uint32_t idx, uint32_t home, uint64_t cap) {
  return idx < home ? idx : (uint32_t)(cap - 1 - (idx - home));
}

__device__ inline void store_dead(const Queue& q, uint32_t i) { q.slab[i] = -1; }

}  // namespace

__global__ __launch_bounds__(kBlock) void k_step(KArgs a) {
  extern __shared__ double lds[];
  Ctl* ctl = a.ctl;
  const uint32_t cur = ctl->cur;
  const uint32_t h0 = ctl->n_home[0], h1 = ctl->n_home[1], h2 = ctl->n_home[2];
  const uint32_t n0 = h0 + ctl->n_sec[0], n1 = h1 + ctl->n_sec[1], n2 = h2 + ctl->n_sec[2];
  const uint32_t ntot = n0 + n1 + n2;
  const uint32_t need = (ntot + kBlock - 1) / kBlock;
  const bool work = blockIdx.x < need && ctl->error == 0;

  if (work) {
    // stage tables, slab planes, slab materials and material constants
    const uint32_t ntab = a.n_mat * kNumTables * a.env.nodes;
    for (uint32_t i = threadIdx.x; i < ntab; i += kBlock) lds[i] = a.tab[i];
    double* zp = lds + ntab;
    for (uint32_t i = threadIdx.x; i <= a.env.n_slabs; i += kBlock) zp[i] = a.zplane[i];
    MatRT* mr = reinterpret_cast<MatRT*>(zp + a.env.n_slabs + 1);
    if (threadIdx.x < a.n_mat) mr[threadIdx.x] = a.mat[threadIdx.x];
    uint32_t* sm = reinterpret_cast<uint32_t*>(mr + a.n_mat);
    for (uint32_t i = threadIdx.x; i < a.env.n_slabs; i += kBlock) sm[i] = a.slab_mat[i];
    __syncthreads();

    StepEnv env = a.env;
    env.tab = lds;
    env.zplane = zp;
    env.mat = mr;
    env.slab_mat = sm;
    const uint32_t nxt = cur ^ 1u;
    const bool full = (a.flags & kFlagFullLedger) != 0;
    const bool logging = (a.flags & kFlagSteplog) != 0;
    // secondary slots per species that leave room for all survivors
    const uint32_t lim0 = (uint32_t)(a.cap - n0), lim1 = (uint32_t)(a.cap - n1), lim2 = (uint32_t)(a.cap - n2);

    for (uint32_t base = blockIdx.x * kBlock; base < ntot; base += gridDim.x * kBlock) {
      const uint32_t i = base + threadIdx.x;
      const bool active = i < ntot;
      int sp = 0;
      uint32_t idx = i, home = h0;
      if (i >= n0 + n1) {
        sp = 2;
        idx = i - n0 - n1;
        home = h2;
      } else if (i >= n0) {
        sp = 1;
        idx = i - n0;
        home = h1;
      }
      const uint32_t pos = queue_pos(idx, home, a.cap);
      const Queue src = queue_view(a.qbase, a.cap, cur, (uint32_t)sp);
      Trk t;
      StepOut o;
      o.nsec = 0;
      o.dep = o.escaped = o.killed = o.clen = 0.0;
      o.pair = o.annih = o.null = 0;
      bool live_in = false;
      double e_before = 0.0;
      if (active) {
        t.slab = src.slab[pos];
        live_in = t.slab >= 0;  // slots of refused secondaries hold slab -1
      }
      if (live_in) {
        t.x = src.x[pos];
        t.y = src.y[pos];
        t.z = src.z[pos];
        t.ux = src.ux[pos];
        t.uy = src.uy[pos];
        t.uz = src.uz[pos];
        t.E = src.E[pos];
        t.id = src.id[pos];
        t.ev = src.ev[pos];
        t.n = src.n[pos];
        t.key = a.keys[t.ev];
        e_before = t.E;
        take_step(env, sp, t, o);
      }

      // reserve secondary slots (top regions); the step commits only if all
      // of this track's secondaries fit
      uint32_t d[3];
#pragma unroll
      for (int q = 0; q < 3; ++q)
        d[q] = (o.nsec > 0 && o.sec[0].sp == q ? 1u : 0u) + (o.nsec > 1 && o.sec[1].sp == q ? 1u : 0u);
      uint32_t slot[3];
      bool commit = live_in;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        slot[q] = wave_reserve(&ctl->next_sec[q], d[q]);
        const uint32_t lim = q == 0 ? lim0 : (q == 1 ? lim1 : lim2);
        if (d[q] && slot[q] + d[q] > lim) commit = false;
      }
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        if (!d[q]) continue;
        const uint32_t lim = q == 0 ? lim0 : (q == 1 ? lim1 : lim2);
        const Queue dq = queue_view(a.qbase, a.cap, nxt, (uint32_t)q);
        uint32_t s = slot[q];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          if (!(k < o.nsec && o.sec[k].sp == q)) continue;
          if (s < lim) {
            const uint32_t p = (uint32_t)(a.cap - 1 - s);
            if (commit) {
              Trk c;
              c.x = t.x;
              c.y = t.y;
              c.z = t.z;
              c.ux = o.sec[k].ux;
              c.uy = o.sec[k].uy;
              c.uz = o.sec[k].uz;
              c.E = o.sec[k].E;
              c.id = o.sec[k].id;
              c.ev = t.ev;
              c.n = 0;
              c.slab = o.slab;
              store_track(dq, p, c);
            } else {
              store_dead(dq, p);
            }
          }
          ++s;
        }
      }

      // home region: survivors of committed steps, or the unstepped track
      const bool carry = live_in && !commit;
      const bool keep = carry || (commit && t.slab >= 0);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const uint32_t hs = wave_reserve(&ctl->next_home[q], (keep && sp == q) ? 1u : 0u);
        if (keep && sp == q) {
          const Queue dq = queue_view(a.qbase, a.cap, nxt, (uint32_t)q);
          if (hs >= a.cap) {
            atomicOr(&ctl->error, kErrOverflow);
          } else if (carry) {
            // the current buffer is untouched during the launch
            dq.x[hs] = src.x[pos];
            dq.y[hs] = src.y[pos];
            dq.z[hs] = src.z[pos];
            dq.ux[hs] = src.ux[pos];
            dq.uy[hs] = src.uy[pos];
            dq.uz[hs] = src.uz[pos];
            dq.E[hs] = src.E[pos];
            dq.id[hs] = src.id[pos];
            dq.ev[hs] = src.ev[pos];
            dq.n[hs] = src.n[pos];
            dq.slab[hs] = src.slab[pos];
          } else {
            store_track(dq, hs, t);
          }
        }
      }

      // tallies of committed steps
      if (commit) {
        if (o.dep != 0.0) atomicAdd(&a.edep[(size_t)t.ev * env.n_slabs + o.slab], o.dep);
        LedgerDev& L = a.ledger[t.ev];
        if (o.escaped != 0.0) atomicAdd(&L.escaped[0] + sp, o.escaped);
        if (o.killed != 0.0) atomicAdd(&L.killed, o.killed);
        if (o.pair) atomicAdd(&L.n_pair, (uint32_t)o.pair);
        if (o.annih) atomicAdd(&L.n_annih, (uint32_t)o.annih);
        if (full) {
          atomicAdd(&L.n_steps, 1ull);
          if (o.clen != 0.0) atomicAdd(&L.charged_len, o.clen);
          if (o.null) atomicAdd(&L.n_null, 1ull);
#pragma unroll
          for (int q = 0; q < 3; ++q)
            if (d[q]) atomicAdd(&L.n_created[q], (unsigned long long)d[q]);
        }
        if (logging) {
          const unsigned long long ls = atomicAdd(&ctl->log_n, 1ull);
          if (ls < a.log_cap) {
            StepRec& r = a.log[ls];
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
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        wave_count(&ctl->steps[s], (commit && sp == s) ? 1u : 0u);
        wave_count(&ctl->created[s], commit ? d[s] : 0u);
      }
      wave_count(&ctl->deferred, carry ? 1u : 0u);
      {
        // per-launch progress counters (32-bit, reset by the last block)
        uint32_t c = commit ? 1u : 0u, k = carry ? 1u : 0u;
        for (int off = 32; off > 0; off >>= 1) {
          c += __shfl_xor(c, off);
          k += __shfl_xor(k, off);
        }
        if (__lane_id() == 0) {
          if (c) atomicAdd(&ctl->commits, c);
          if (k) atomicAdd(&ctl->carried, k);
        }
      }
    }
  }

  // the last block to finish publishes the next iteration
  __shared__ uint32_t last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(&ctl->blocks_done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __threadfence();
    if (a.flags & kFlagProfile) {
      if (ctl->iteration < a.profile_cap) {
        a.profile[(size_t)ctl->iteration * 3 + 0] = n0;
        a.profile[(size_t)ctl->iteration * 3 + 1] = n1;
        a.profile[(size_t)ctl->iteration * 3 + 2] = n2;
      }
    }
    if (ntot > 0) ctl->iteration += 1;
    const uint32_t commits = atomicAdd(&ctl->commits, 0u), carried = atomicAdd(&ctl->carried, 0u);
    if (carried > 0 && commits == 0) ctl->error |= kErrStall;  // nothing can move: queues too small
    uint32_t live = 0;
    for (int q = 0; q < 3; ++q) {
      const uint32_t lim = (uint32_t)(a.cap - (q == 0 ? n0 : (q == 1 ? n1 : n2)));
      const uint32_t hv = atomicAdd(&ctl->next_home[q], 0u);
      uint32_t sv = atomicAdd(&ctl->next_sec[q], 0u);
      sv = sv < lim ? sv : lim;
      ctl->n_home[q] = hv;
      ctl->n_sec[q] = sv;
      ctl->next_home[q] = 0;
      ctl->next_sec[q] = 0;
      ctl->peak[q] = hv + sv > ctl->peak[q] ? hv + sv : ctl->peak[q];
      live += hv + sv;
    }
    ctl->live = live;
    ctl->commits = 0;
    ctl->carried = 0;
    ctl->cur = cur ^ 1u;
    ctl->blocks_done = 0;
    __threadfence();
  }
}

// Injection: prepared tracks appended to the current queues.
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
      if (!cnt) continue;
      if (slot + ctl->n_sec[qs] >= a.cap) {
        atomicOr(&ctl->error, kErrOverflow);
        continue;
      }
      Trk t;
      t.x = r.x;
      t.y = r.y;
      t.z = r.z;
      t.ux = r.ux;
      t.uy = r.uy;
      t.uz = r.uz;
      t.E = r.E;
      t.id = r.id;
      t.ev = r.ev;
      t.n = 0;
      t.slab = r.slab;
      store_track(queue_view(a.qbase, a.cap, cur, (uint32_t)qs), slot, t);
    }
  }
}

hipError_t launch_step(const KArgs& a, uint32_t blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_step, dim3(blocks), dim3(kBlock), a.lds_bytes, s, a);
  return hipGetLastError();
}
hipError_t launch_inject(const KArgs& a, const InjRec* rec, uint32_t n, hipStream_t s) {
  const uint32_t blocks = n == 0 ? 1 : (n + kBlock - 1) / kBlock < 4096 ? (n + kBlock - 1) / kBlock : 4096;
  hipLaunchKernelGGL(k_inject, dim3(blocks), dim3(kBlock), 0, s, a, rec, n);
  return hipGetLastError();
}
// live count after injection (one thread)
__global__ void k_census(KArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctl* c = a.ctl;
    uint32_t live = 0;
    for (int q = 0; q < 3; ++q) {
      const uint32_t n = c->n_home[q] + c->n_sec[q];
      c->peak[q] = n > c->peak[q] ? n : c->peak[q];
      live += n;
    }
    c->live = live;
  }
}
hipError_t launch_census(const KArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_census, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t set_step_lds(uint32_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

}  // namespace ems
