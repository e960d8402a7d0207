// gm_common.h -- shared device helpers and launch descriptors of libgm.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gm_draw.h"

// Pointer into LDS (address space 3): keeps the compiler on ds_* instructions
// where a generic pointer would fall back to flat ones.
#define GM_LDS __attribute__((address_space(3)))

namespace gm {

constexpr int kWave = 64;

using lds_u64 = GM_LDS unsigned long long;
using lds_u32 = GM_LDS uint32_t;
using lds_u16 = GM_LDS uint16_t;
using lds_i32 = GM_LDS int32_t;
using lds_f64 = GM_LDS double;

__device__ __forceinline__ unsigned long long lds_min(lds_u64* p, unsigned long long v) {
  return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ int32_t lds_add(lds_i32* p, int32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One DPP step of a wave-wide u64 maximum (lanes without a source keep v).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ unsigned long long dpp_max_step(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(static_cast<int>(v), static_cast<int>(v), kCtrl,
                                             kRowMask, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(static_cast<int>(v >> 32), static_cast<int>(v >> 32),
                                             kCtrl, kRowMask, 0xf, false);
  const unsigned long long o =
      (static_cast<unsigned long long>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo);
  return o > v ? o : v;
}

// Poisoned register: index -2, value NaN.  Empty register: index -1, +inf.
constexpr int32_t kIdxEmpty = -1;
constexpr int32_t kIdxPoison = -2;
constexpr uint64_t kInfBits = 0x7FF0000000000000ull;
constexpr uint64_t kNanBits = 0x7FF8000000000000ull;

// A weight is valid when it is finite and >= 0 (0 means "not in N+").
__device__ __forceinline__ bool weight_valid(float w) {
  return w >= 0.0f && w <= 3.402823466e38f;  // false for NaN, negatives, +inf
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const uint32_t lane = __lane_id();
  return lane ? (~0ull >> (64 - lane)) : 0ull;
}

__device__ __forceinline__ int32_t readlane_i32(int32_t v, int lane) {
  return __builtin_amdgcn_readlane(v, lane);
}

__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int lane) {
  const uint32_t lo = static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v), lane));
  const uint32_t hi =
      static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(v >> 32), lane));
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  return bitsd(readlane_u64(dbits(v), lane));
}

// Maximum over the wave, returned to every lane: prefix maxima inside each
// row of 16 lanes (row_shr 1, 2, 4, 8), then row 0 into 1 and 2 into 3
// (row_bcast:15), then rows 0-1 into 2-3 (row_bcast:31); lane 63 holds the
// result.  Registers only, no LDS round trip.
__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v) {
  v = dpp_max_step<0x111, 0xf>(v);
  v = dpp_max_step<0x112, 0xf>(v);
  v = dpp_max_step<0x114, 0xf>(v);
  v = dpp_max_step<0x118, 0xf>(v);
  v = dpp_max_step<0x142, 0xa>(v);
  v = dpp_max_step<0x143, 0xc>(v);
  return readlane_u64(v, 63);
}

// Value of lane l-1 in lane l (wave_shr:1); lane 0 receives `first`.
__device__ __forceinline__ double wave_shr1_f64(double v, double first) {
  const uint64_t b = dbits(v), o = dbits(first);
  const int lo = __builtin_amdgcn_update_dpp(static_cast<int>(o), static_cast<int>(b), 0x138, 0xf,
                                             0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(static_cast<int>(o >> 32), static_cast<int>(b >> 32),
                                             0x138, 0xf, 0xf, false);
  return bitsd((static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo));
}

__device__ __forceinline__ int wave_sum_i32(int v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
  return v;
}

// Arguments shared by the sketch kernels.
struct SketchArgs {
  const int32_t* idx;
  const float* w;
  const int64_t* off;
  int64_t nvec;
  int32_t k_uniform;          // used when kvec == nullptr
  const int32_t* kvec;        // per-vector k (batched) or nullptr
  const int64_t* outoff;      // per-vector output offset (batched) or nullptr
  int32_t k_max;
  uint64_t seed_mix;          // mix(seed)
  int32_t* out_idx;
  double* out_val;
  unsigned long long* err;    // data-error counter
};

// Scratch handed to a plain-form launch for splitting vectors over
// workgroups (see launch_plain): `regs` partial registers (8-byte values,
// then 4-byte indices) followed by two arrays of `counters` int32 and
// kPlainPlanBytes of split plan.
// Bytes after the counters that hold a split plan for batches of uneven
// vectors (gm_plain.hip).
constexpr size_t kPlainPlanBytes = 32768;

struct PlainScratch {
  void* base;         // nullptr: the launch does not split
  int64_t regs;
  int64_t counters;
  bool clear;         // zero the counters with a fill kernel before the launch
};

// Per-vector descriptor resolved on the device.
struct VecDesc {
  int64_t a, b;   // entry range
  int32_t k;      // register count
  int64_t o;      // first output register
  bool bad;       // structural error (decreasing offsets or k out of range)
};

__device__ __forceinline__ VecDesc vec_desc(const SketchArgs& p, int64_t v) {
  VecDesc d;
  d.a = p.off[v];
  d.b = p.off[v + 1];
  d.k = p.kvec ? p.kvec[v] : p.k_uniform;
  d.o = p.outoff ? p.outoff[v] : v * static_cast<int64_t>(p.k_uniform);
  d.bad = d.b < d.a || d.k < 1 || d.k > p.k_max;
  return d;
}

// Register count to write for a vector (a poisoned batched vector with a bad
// k writes the span its output offsets give it, capped at k_max).
__device__ __forceinline__ int32_t out_span(const SketchArgs& p, int64_t v, const VecDesc& d) {
  if (!p.outoff) return p.k_uniform;
  if (d.k >= 1 && d.k <= p.k_max) return d.k;
  const int64_t span = p.outoff[v + 1] - p.outoff[v];
  return static_cast<int32_t>(span < 0 ? 0 : (span > p.k_max ? p.k_max : span));
}

}  // namespace gm
