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
//  - the last block to finish swaps the queues and decides how many tracks
//    of each species fit in the next step (the rest are carried unchanged),
//    so a chain of launches needs no host round trip.
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

// How many tracks of each species can be stepped so that every next queue
// can hold the worst case: stepped tracks yield at most (A[q][s]) tracks of
// species q, carried tracks stay where they are.
__device__ void plan_iteration(Ctl* c, uint64_t cap) {
  const int A[3][3] = {{1, 1, 2}, {1, 2, 1}, {1, 0, 1}};
  const uint64_t n[3] = {c->n_cur[0], c->n_cur[1], c->n_cur[2]};
  double f = 1.0;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int64_t grow = (int64_t)(A[q][0] * n[0] + A[q][1] * n[1] + A[q][2] * n[2]) - (int64_t)n[q];
    if (grow > 0) {
      const double fq = (double)(cap - n[q]) / (double)grow;
      f = fq < f ? fq : f;
    }
  }
  uint64_t m[3];
  for (int attempt = 0; attempt < 64; ++attempt) {
#pragma unroll
    for (int s = 0; s < 3; ++s) m[s] = f >= 1.0 ? n[s] : (uint64_t)floor(f * (double)n[s]);
    bool ok = true;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const uint64_t w = (n[q] - m[q]) + A[q][0] * m[0] + A[q][1] * m[1] + A[q][2] * m[2];
      ok = ok && (w <= cap);
    }
    if (ok) break;
    f *= 0.99;
    if (attempt == 63) m[0] = m[1] = m[2] = 0;
  }
  uint64_t live = n[0] + n[1] + n[2];
  if (live > 0 && m[0] + m[1] + m[2] == 0) c->error |= kErrStall;
  for (int s = 0; s < 3; ++s) c->m[s] = (uint32_t)m[s];
  c->deferred += (n[0] - m[0]) + (n[1] - m[1]) + (n[2] - m[2]);
  c->live = (uint32_t)live;
}

}  // namespace

__global__ __launch_bounds__(kBlock) void k_step(KArgs a) {
  extern __shared__ double lds[];
  Ctl* ctl = a.ctl;
  const uint32_t cur = ctl->cur;
  const uint32_t n0 = ctl->n_cur[0], n1 = ctl->n_cur[1], n2 = ctl->n_cur[2];
  const uint32_t m0 = ctl->m[0], m1 = ctl->m[1], m2 = ctl->m[2];
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

    for (uint32_t base = blockIdx.x * kBlock; base < ntot; base += gridDim.x * kBlock) {
      const uint32_t i = base + threadIdx.x;
      const bool active = i < ntot;
      int sp = 0;
      uint32_t idx = i, msp = m0;
      if (i >= n0 + n1) {
        sp = 2;
        idx = i - n0 - n1;
        msp = m2;
      } else if (i >= n0) {
        sp = 1;
        idx = i - n0;
        msp = m1;
      }
      Trk t;
      StepOut o;
      o.nsec = 0;
      o.dep = o.escaped = o.killed = o.clen = 0.0;
      o.pair = o.annih = o.null = 0;
      bool stepped = false;
      double e_before = 0.0;
      if (active) {
        const Queue q = queue_view(a.qbase, a.cap, cur, (uint32_t)sp);
        t.x = q.x[idx];
        t.y = q.y[idx];
        t.z = q.z[idx];
        t.ux = q.ux[idx];
        t.uy = q.uy[idx];
        t.uz = q.uz[idx];
        t.E = q.E[idx];
        t.id = q.id[idx];
        t.ev = q.ev[idx];
        t.n = q.n[idx];
        t.slab = q.slab[idx];
        t.key = a.keys[t.ev];
        if (idx < msp) {
          e_before = t.E;
          take_step(env, sp, t, o);
          stepped = true;
        }
      }
      const bool alive = active && t.slab >= 0;

      // append survivors and secondaries to the next queues
#pragma unroll
      for (int qs = 0; qs < 3; ++qs) {
        uint32_t cnt = (alive && sp == qs) ? 1u : 0u;
        const bool s0 = o.nsec > 0 && o.sec[0].sp == qs, s1 = o.nsec > 1 && o.sec[1].sp == qs;
        cnt += (uint32_t)s0 + (uint32_t)s1;
        const uint32_t slot0 = wave_reserve(&ctl->n_next[qs], cnt);
        if (cnt == 0) continue;
        const Queue dq = queue_view(a.qbase, a.cap, nxt, (uint32_t)qs);
        uint32_t slot = slot0;
        if (slot + cnt > a.cap) {
          atomicOr(&ctl->error, kErrOverflow);
          continue;
        }
        if (alive && sp == qs) store_track(dq, slot++, t);
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          if (!(k < o.nsec && o.sec[k].sp == qs)) continue;
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
          store_track(dq, slot++, c);
        }
      }

      // tallies
      if (stepped) {
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
          for (int k = 0; k < 2; ++k)
            if (k < o.nsec) atomicAdd(&L.n_created[o.sec[k].sp], 1ull);
        }
        if (logging) {
          const unsigned long long slot = atomicAdd(&ctl->log_n, 1ull);
          if (slot < a.log_cap) {
            StepRec& r = a.log[slot];
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
        wave_count(&ctl->steps[s], (stepped && sp == s) ? 1u : 0u);
        uint32_t made = 0;
#pragma unroll
        for (int k = 0; k < 2; ++k) made += (k < o.nsec && o.sec[k].sp == s) ? 1u : 0u;
        wave_count(&ctl->created[s], made);
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
      if (ctl->iteration < a.profile_cap)
        for (int s = 0; s < 3; ++s) a.profile[(size_t)ctl->iteration * 3 + s] = ctl->n_cur[s];
    }
    if (ntot > 0) ctl->iteration += 1;
    for (int s = 0; s < 3; ++s) {
      const uint32_t v = atomicAdd(&ctl->n_next[s], 0u);
      ctl->n_cur[s] = v;
      ctl->n_next[s] = 0;
      ctl->peak[s] = v > ctl->peak[s] ? v : ctl->peak[s];
    }
    ctl->cur = cur ^ 1u;
    plan_iteration(ctl, a.cap);
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
      const uint32_t slot = wave_reserve(&ctl->n_cur[qs], cnt);
      if (!cnt) continue;
      if (slot >= a.cap) {
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

// One thread: plan the first iteration after injection.
__global__ void k_plan(KArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Ctl* c = a.ctl;
    for (int s = 0; s < 3; ++s) c->peak[s] = c->n_cur[s] > c->peak[s] ? c->n_cur[s] : c->peak[s];
    plan_iteration(c, a.cap);
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
hipError_t launch_plan(const KArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_plan, dim3(1), dim3(64), 0, s, a);
  return hipGetLastError();
}
hipError_t set_step_lds(uint32_t bytes) {
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_step), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)bytes);
}

}  // namespace ems
