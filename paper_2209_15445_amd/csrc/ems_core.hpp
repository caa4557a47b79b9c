// ems_core.hpp -- constants, counter-based RNG and small vector helpers shared
// by the host table builder, the host test hook and the gfx950 kernels.
//
// The RNG abstraction follows the paper's physics section (2.2): the physics
// run-time functions take their random numbers from an abstracted generator.
// Here every draw is addressed by (seed, event key, track id, step, index)
// through Philox4x32-10 (Salmon et al., SC'11), so the breadth-first GPU loop
// reproduces per-track histories regardless of scheduling.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define EMS_HD __host__ __device__ inline
#else
#define EMS_HD inline
#endif

#include <math.h>

namespace ems {

// CODATA 2018 values; kB converts p [MeV/c] = kB * B [T] * R [mm].
constexpr double kMe = 0.51099895;
constexpr double kRe = 2.8179403262e-12;  // mm
constexpr double kAlpha = 1.0 / 137.035999084;
constexpr double kNA = 6.02214076e23;
constexpr double kKB = 0.299792458;
constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647692;

constexpr int kMaxTrials = 1000;      // rejection loops accept the last candidate
constexpr double kSafetyMin = 1e-6;   // mm: helix track this close to a wall escapes
constexpr uint32_t kChildBit = 0x80000000u;

enum Species : int { kGamma = 0, kElectron = 1, kPositron = 2 };

// process mask bits (same values as the public header)
enum : uint32_t {
  kPCompton = 1u << 0, kPPhot = 1u << 1, kPConv = 1u << 2, kPEIoni = 1u << 3,
  kPEBrem = 1u << 4, kPAnnih = 1u << 5, kPCont = 1u << 6, kPMsc = 1u << 7, kPFluct = 1u << 8,
  kPAllBits = 0x1FFu
};
// step-log limiter / process codes (same values as the oracle's log)
enum : uint32_t {
  kLimZ = 0, kLimWall = 1, kLimSafety = 2, kLimCont = 3, kLimDiscrete = 4,
  kLimStopped = 5, kLimSubcut = 6, kLimEscapeSafety = 7
};
enum : uint32_t {
  kXNone = 0, kXCompton = 1, kXPhot = 2, kXConv = 3, kXMoller = 4, kXBhabha = 5,
  kXBrem = 6, kXAnnih = 7, kXAnnihRest = 8, kXNull = 9
};

// ---------------------------------------------------------------- Philox
struct U4 {
  uint32_t x, y, z, w;
};

EMS_HD U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t a = (uint64_t)0xD2511F53u * c.x;
    const uint64_t b = (uint64_t)0xCD9E8D57u * c.z;
    U4 n;
    n.x = (uint32_t)(b >> 32) ^ c.y ^ k0;
    n.y = (uint32_t)b;
    n.z = (uint32_t)(a >> 32) ^ c.w ^ k1;
    n.w = (uint32_t)a;
    c = n;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// ---------------------------------------------------------------- reals
// The step arithmetic is written once for a real type R: double for the
// FP64 form, float for the mixed form (tables, interpolation, step lengths
// and sampling in FP32; positions, boundary distances and energies stay FP64
// in the callers).  These overloads pick the single- or double-precision
// libm routine explicitly.
EMS_HD float xlog(float v) { return logf(v); }
EMS_HD double xlog(double v) { return log(v); }
EMS_HD float xexp(float v) { return expf(v); }
EMS_HD double xexp(double v) { return exp(v); }
EMS_HD float xsqrt(float v) { return sqrtf(v); }
EMS_HD double xsqrt(double v) { return sqrt(v); }
EMS_HD float xsin(float v) { return sinf(v); }
EMS_HD double xsin(double v) { return sin(v); }
EMS_HD float xcos(float v) { return cosf(v); }
EMS_HD double xcos(double v) { return cos(v); }
// sine and cosine of one angle with one argument reduction (the compiler
// does not merge separate sin and cos calls; about half the instructions)
EMS_HD void xsincos(float v, float* s, float* c) { sincosf(v, s, c); }
EMS_HD void xsincos(double v, double* s, double* c) { sincos(v, s, c); }
EMS_HD float xfloor(float v) { return floorf(v); }
EMS_HD double xfloor(double v) { return floor(v); }
EMS_HD float xceil(float v) { return ceilf(v); }
EMS_HD float xpow(float a, float b) { return powf(a, b); }
EMS_HD double xpow(double a, double b) { return pow(a, b); }
EMS_HD double xceil(double v) { return ceil(v); }

// A uniform draw in the arithmetic type: the FP64 value itself, or that
// value rounded to float and kept inside [2^-25, 1 - 2^-24] so that ln u is
// finite and u < 1 (the same draws drive both forms).
template <class R>
EMS_HD R as_real_u(double u) {
  return u;
}
template <>
EMS_HD float as_real_u<float>(double u) {
  const float f = (float)u;
  return f < 0x1p-25f ? 0x1p-25f : (f > 1.0f - 0x1p-24f ? 1.0f - 0x1p-24f : f);
}

// 64 bits (hi:lo) -> (0,1): top 52 bits plus one half ulp, exactly representable
EMS_HD double to_unit(uint32_t lo, uint32_t hi) {
  const uint64_t v = ((uint64_t)hi << 32) | lo;
  return (double)(v >> 12) * 0x1p-52 + 0x1p-53;
}

// The draws of one track step.  Block j of Philox(key, (id_lo, id_hi, step, j))
// yields U_{2j} (words x,y) and U_{2j+1} (words z,w).  next() hands out U_2,
// U_3, ... in program order; U_0 and U_1 come from block 0.
struct Draws {
  uint32_t k0, k1, id_lo, id_hi, step;
  uint32_t idx;     // next index for next()
  uint32_t cached;  // block number held in buf (or ~0u)
  U4 buf;

  EMS_HD void init(uint32_t seed, uint32_t key, uint64_t id, uint32_t n) {
    k0 = seed;
    k1 = key;
    id_lo = (uint32_t)id;
    id_hi = (uint32_t)(id >> 32);
    step = n;
    idx = 2;
    cached = ~0u;
  }
  EMS_HD double at(uint32_t i) {
    const uint32_t blk = i >> 1;
    if (blk != cached) {
      buf = philox4x32_10(U4{id_lo, id_hi, step, blk}, k0, k1);
      cached = blk;
    }
    return (i & 1u) ? to_unit(buf.z, buf.w) : to_unit(buf.x, buf.y);
  }
  EMS_HD double next() { return at(idx++); }
  template <class R>
  EMS_HD R u_at(uint32_t i) {
    return as_real_u<R>(at(i));
  }
  template <class R>
  EMS_HD R u() {
    return as_real_u<R>(at(idx++));
  }
  EMS_HD uint64_t child_id(uint32_t k) const {
    const U4 r = philox4x32_10(U4{id_lo, id_hi, step, kChildBit | k}, k0, k1);
    return (uint64_t)r.x | ((uint64_t)r.y << 32);
  }
};

// ---------------------------------------------------------------- vectors
template <class R>
struct V3T {
  R x, y, z;
};
using V3 = V3T<double>;

template <class R>
EMS_HD V3T<R> unit(V3T<R> v) {
  const R n = xsqrt(v.x * v.x + v.y * v.y + v.z * v.z);
  return V3T<R>{v.x / n, v.y / n, v.z / n};
}

// Direction with polar angle (cos t, sin t) and azimuth p about the axis u:
// the frame is (e1, e2, u) with e2 = z^ x u / |z^ x u| and e1 = e2 x u;
// u = +-z^ uses e1 = (+-1, 0, 0), e2 = (0, 1, 0).
template <class R>
EMS_HD V3T<R> about_axis(V3T<R> u, R cost, R sint, R phi) {
  R sp, cp;
  xsincos(phi, &sp, &cp);
  const R a = sint * cp, b = sint * sp;
  const R t2 = u.x * u.x + u.y * u.y;
  if (t2 > R(0)) {
    const R t = xsqrt(t2);
    return V3T<R>{(u.x * u.z * a - u.y * b) / t + u.x * cost,
                  (u.y * u.z * a + u.x * b) / t + u.y * cost,
                  -t * a + u.z * cost};
  }
  if (u.z > R(0)) return V3T<R>{a, b, cost};
  return V3T<R>{-a, b, -cost};
}

}  // namespace ems
