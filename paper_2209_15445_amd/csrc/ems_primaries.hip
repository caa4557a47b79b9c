// ems_primaries.hip -- primaries handed over in device memory: the
// check, staging and id passes that ems_enqueue_device runs before the
// tracks are injected (the host path computes the same on the host).
#include <hip/hip_runtime.h>

#include "ems_runtime.hpp"

namespace ems {

namespace {

constexpr int kBlock = 256;

// Primaries handed over in device memory (section 4: the particles of a
// region given to the library; here already resident in HBM).  A primary
// is accepted under the conditions of the host path: row below max_events,
// a species, finite positive energy, a finite non-zero direction, and a
// position inside the geometry (a volume found for it in a box geometry;
// inside the stack's z range and its half width for a slab stack).
__device__ inline bool primary_valid(const KArgs& a, const PrimRec& q) {
#pragma clang fp contract(off)
  const double d2 = q.dir[0] * q.dir[0] + q.dir[1] * q.dir[1] + q.dir[2] * q.dir[2];
  if (!(q.event < a.max_events && q.species <= 2u && q.E > 0.0 && isfinite(q.E) && d2 > 0.0 && isfinite(d2)))
    return false;
  if (a.geo) {
    if (!(isfinite(q.pos[0]) && isfinite(q.pos[1]) && isfinite(q.pos[2]))) return false;
    return bvh_locate(a.env.nav, q.pos, q.dir) >= 0;
  }
  const uint32_t n = a.env.n_slabs;
  return q.pos[2] >= a.zplane[0] && q.pos[2] <= a.zplane[n] && fabs(q.pos[0]) <= a.env.half_xy &&
         fabs(q.pos[1]) <= a.env.half_xy;
}

// slab holding z (planes zp[0..n]); a point on a plane belongs to the slab
// its direction enters
__device__ inline int32_t slab_of(const double* zp, uint32_t n, double z, double uz) {
  if (z >= zp[n]) return (int32_t)n - 1;
  uint32_t lo = 0, hi = n;  // zp[lo] <= z < zp[hi]
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (zp[mid] <= z) lo = mid;
    else hi = mid;
  }
  if (lo > 0 && z == zp[lo] && uz < 0.0) lo -= 1;
  return (int32_t)lo;
}

// Check pass over n device primaries: chk[0] = n - i for the first invalid
// primary i (0: all valid), chk[1 + s] = primaries of species s.  chk is
// zero on entry.
__global__ __launch_bounds__(kBlock) void k_check_primaries(KArgs a, const PrimRec* p, uint64_t n,
                                                            unsigned long long* chk) {
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base < n; base += stride) {
    const uint64_t i = base + threadIdx.x;
    bool ok = true;
    uint32_t sp = 3;
    if (i < n) {
      const PrimRec q = p[i];
      ok = primary_valid(a, q);
      sp = ok ? q.species : 3u;
      if (!ok) atomicMax(&chk[0], (unsigned long long)(n - i));
    }
    for (uint32_t s = 0; s < 3; ++s) {
      const uint32_t c = (uint32_t)__popcll(__ballot(sp == s));
      if (__lane_id() == 0 && c) atomicAdd(&chk[1 + s], (unsigned long long)c);
    }
  }
}

// Stage pass: the injection records of k valid device primaries (direction
// normalised, volume located, the row's event key); ids are set by
// k_primary_ids.
__global__ __launch_bounds__(kBlock) void k_stage_primaries(KArgs a, const PrimRec* p, uint32_t k,
                                                            const uint32_t* keys, InjRec* out) {
  // the length as the host computes it: products and sums rounded one by
  // one (no fused multiply-add), then a correctly rounded root and quotients
#pragma clang fp contract(off)
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < k; i += gridDim.x * kBlock) {
    const PrimRec q = p[i];
    const double nrm = sqrt(q.dir[0] * q.dir[0] + q.dir[1] * q.dir[1] + q.dir[2] * q.dir[2]);
    InjRec r;
    r.x = q.pos[0];
    r.y = q.pos[1];
    r.z = q.pos[2];
    r.ux = q.dir[0] / nrm;
    r.uy = q.dir[1] / nrm;
    r.uz = q.dir[2] / nrm;
    r.E = q.E;
    r.id = 0;
    r.ev = q.event;
    r.sp = q.species;
    if (a.geo) {
      const double pp[3] = {r.x, r.y, r.z}, uu[3] = {r.ux, r.uy, r.uz};
      r.slab = bvh_locate(a.env.nav, pp, uu);
    } else {
      r.slab = slab_of(a.zplane, a.env.n_slabs, r.z, r.uz);
    }
    r.key = keys[q.event];
    out[i] = r;
  }
}

// Ids of staged primaries: the running index of a primary within its row,
// in input order, continuing from the row's count so far (row_next).  One
// block of 1024 threads takes the records in groups of 1024, in order: it
// sorts the group's (row, position) keys in LDS (bitonic), a primary's rank
// is its distance from its row's first key, and the row's first key adds
// the group's count to row_next, which returns the row's base.
constexpr uint32_t kIdGroup = 1024;
__global__ __launch_bounds__(kIdGroup) void k_primary_ids(InjRec* rec, uint32_t n, unsigned long long* row_next) {
  __shared__ unsigned long long key[kIdGroup];
  __shared__ unsigned long long base[kIdGroup];
  __shared__ uint32_t head[kIdGroup];
  const uint32_t t = threadIdx.x;
  for (uint32_t g = 0; g < n; g += kIdGroup) {
    key[t] = g + t < n ? ((unsigned long long)rec[g + t].ev << 10 | t) : ~0ull;
    __syncthreads();
    for (uint32_t size = 2; size <= kIdGroup; size <<= 1) {
      for (uint32_t j = size >> 1; j > 0; j >>= 1) {
        const uint32_t o = t ^ j;
        if (o > t) {
          const unsigned long long x = key[t], y = key[o];
          const bool up = (t & size) == 0;
          if ((x > y) == up) {
            key[t] = y;
            key[o] = x;
          }
        }
        __syncthreads();
      }
    }
    const unsigned long long kk = key[t];
    const bool valid = kk != ~0ull;
    const unsigned long long row = kk >> 10;
    const bool first = valid && (t == 0 || (key[t - 1] >> 10) != row);
    const bool last = valid && (t == kIdGroup - 1 || (key[t + 1] >> 10) != row);
    head[t] = first ? t : 0u;
    __syncthreads();
    // start of each key's row: running maximum of the row heads
    for (uint32_t off = 1; off < kIdGroup; off <<= 1) {
      const uint32_t v = t >= off && head[t - off] > head[t] ? head[t - off] : head[t];
      __syncthreads();
      head[t] = v;
      __syncthreads();
    }
    const uint32_t start = head[t];
    if (last) base[start] = atomicAdd(&row_next[row], (unsigned long long)(t - start + 1));
    __syncthreads();
    if (valid) rec[g + (uint32_t)(kk & (kIdGroup - 1))].id = base[start] + (t - start);
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_check_primaries(const KArgs& a, const void* p, uint64_t n, unsigned long long* chk, hipStream_t s) {
  const uint64_t want = (n + kBlock - 1) / kBlock;
  const uint32_t blocks = (uint32_t)(want < 4096 ? (want ? want : 1) : 4096);
  hipLaunchKernelGGL(k_check_primaries, dim3(blocks), dim3(kBlock), 0, s, a, static_cast<const PrimRec*>(p), n, chk);
  return hipGetLastError();
}
hipError_t launch_stage_primaries(const KArgs& a, const void* p, uint32_t k, const uint32_t* keys,
                                  unsigned long long* row_next, InjRec* out, hipStream_t s) {
  const uint32_t want = (k + kBlock - 1) / kBlock;
  const uint32_t blocks = want < 4096 ? (want ? want : 1) : 4096;
  hipLaunchKernelGGL(k_stage_primaries, dim3(blocks), dim3(kBlock), 0, s, a, static_cast<const PrimRec*>(p), k, keys,
                     out);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_primary_ids, dim3(1), dim3(kIdGroup), 0, s, out, k, row_next);
  return hipGetLastError();
}

}  // namespace ems
