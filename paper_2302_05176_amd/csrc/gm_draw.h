// gm_draw.h -- device implementation of the sketch's random draws.
//
// The paper fixes the Gumbel-Max sketch only in distribution: each element i
// needs k consistent Exp(1) variables (Sec. 1: a_ij generated on the fly from
// a seeded hash instead of being stored), and FastGM needs, per element, the
// k order statistics of those variables in ascending order (Eq. (7)-(8),
// Renyi's representation) together with a uniformly random permutation that
// routes the z-th arrival to a register (Fisher-Yates, Sec. 2.2).  This
// header pins those choices down so that a sketch is a deterministic function
// of (entries, k, seed):
//
//   mix(z)       splitmix64 output function (Steele, Lea, Flood 2014).
//   prefix(i)    mix(mix(seed) ^ (u32)i): one hash state per element index.
//   draw(tag,j)  mix(prefix ^ (tag << 32 | j)); tag 1: plain register j
//                (0-based); tag 2: arrival uniform of step z; tag 3: shuffle
//                draw of step z (z 1-based).
//   uniform(x)   ((double)(x >> 11) + 0.5) * 2^-53, in [2^-54, 1].
//   neglog(u)    -ln(u), fdlibm-style reduction u = 2^e m, m in
//                [sqrt(1/2), sqrt(2)], atanh series with Taylor coefficients
//                2/(2n+1), n = 1..10, evaluated in the fixed order below.
//   randint      z + ((x >> 32) * (k - z + 1)) >> 32, in [z, k].
//
// Every floating-point step is a single IEEE double operation or an explicit
// fma, in the order written; the library is built with -ffp-contract=off so
// the compiler fuses nothing else.  The results are therefore identical on any
// IEEE-754 machine that follows the same written steps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gm {

constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr uint32_t kTagPlain = 1u;
constexpr uint32_t kTagArrival = 2u;
constexpr uint32_t kTagShuffle = 3u;

__host__ __device__ __forceinline__ uint64_t mix(uint64_t z) {
  z += kGolden;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ __forceinline__ uint64_t draw(uint64_t prefix, uint32_t tag, uint32_t j) {
  return mix(prefix ^ ((static_cast<uint64_t>(tag) << 32) | j));
}

__host__ __device__ __forceinline__ double uniform(uint64_t x) {
  return (static_cast<double>(x >> 11) + 0.5) * 0x1p-53;
}

__host__ __device__ __forceinline__ uint64_t dbits(double x) {
#ifdef __HIP_DEVICE_COMPILE__
  return static_cast<uint64_t>(__double_as_longlong(x));
#else
  uint64_t b;
  __builtin_memcpy(&b, &x, 8);
  return b;
#endif
}

__host__ __device__ __forceinline__ double bitsd(uint64_t b) {
#ifdef __HIP_DEVICE_COMPILE__
  return __longlong_as_double(static_cast<long long>(b));
#else
  double x;
  __builtin_memcpy(&x, &b, 8);
  return x;
#endif
}

// -ln(u) for u in (0, 1] (normal numbers).  +0 for u == 1.
__host__ __device__ __forceinline__ double neglog(double u) {
  const double ln2_hi = 0x1.62e42fee00000p-1;  // ln 2 truncated to 32 bits
  const double ln2_lo = 0x1.a39ef35793c76p-33; // ln 2 - ln2_hi
  uint64_t b = dbits(u);
  int e = static_cast<int>(b >> 52) - 1023;
  double m = bitsd((b & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull);
  if (m > 0x1.6a09e667f3bcdp+0) {
    m = m * 0.5;
    e = e + 1;
  }
  const double f = m - 1.0;
  const double s = f / (2.0 + f);
  const double z = s * s;
  double R = 2.0 / 21.0;
  R = fma(R, z, 2.0 / 19.0);
  R = fma(R, z, 2.0 / 17.0);
  R = fma(R, z, 2.0 / 15.0);
  R = fma(R, z, 2.0 / 13.0);
  R = fma(R, z, 2.0 / 11.0);
  R = fma(R, z, 2.0 / 9.0);
  R = fma(R, z, 2.0 / 7.0);
  R = fma(R, z, 2.0 / 5.0);
  R = fma(R, z, 2.0 / 3.0);
  R = R * z;
  const double h = 0.5 * f * f;
  const double de = static_cast<double>(e);
  const double a = h + R;
  const double t = fma(s, a, de * ln2_lo);
  const double c = h - t;
  const double d = c - f;
  return d - de * ln2_hi;
}

// Exp(1) variate of a draw.
__host__ __device__ __forceinline__ double exp1(uint64_t x) { return neglog(uniform(x)); }

// Fisher-Yates target of step z (1-based) among positions [z, k].
__host__ __device__ __forceinline__ int32_t randint(uint64_t x, int32_t z, int32_t k) {
  const uint32_t hi = static_cast<uint32_t>(x >> 32);
  const uint32_t span = static_cast<uint32_t>(k - z + 1);
  return z + static_cast<int32_t>((static_cast<uint64_t>(hi) * span) >> 32);
}

}  // namespace gm
