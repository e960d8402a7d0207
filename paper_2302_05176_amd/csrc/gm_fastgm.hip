// gm_fastgm.hip -- FastGM form of the Gumbel-Max sketch on CDNA4.
//
// What is computed (Sec. 2.2, Algorithms 1 and 2): every positive element i
// is a queue that emits its k Exp(v_i) variables in ascending order
// (t_z = O_z / v_i with O_z = O_{z-1} + E_z / (k - z + 1), Eq. (7)-(8)); the
// z-th arrival is routed to server pi_i[z] of a Fisher-Yates permutation, and
// each register keeps the first arrival it receives (lexicographic (t, i)
// minimum).  An element stops at its first arrival later than the running
// maximum register y* (FastPrune): its later arrivals are larger still and
// cannot change any register, so the result equals the unpruned one.
//
// GPU mapping.  A planner kernel sorts the vectors into classes by size (up
// to 32768 entries, or big) and k range, and inside a class by decreasing
// size; one persistent kernel per class drains its list through an atomic
// work counter.  A large vector is handled by a workgroup of W waves that
// share its registers; when the registers are small (k <= 256), vectors of
// fewer than 2048 entries are handled by one wave each:
//  * Registers live in LDS.  A register is two 64-bit words: `packed` holds
//    the top bits of the key (positive doubles order like their bit patterns)
//    above the element index (31 bits by default), updated by 64-bit LDS
//    atomic-min;
//    `fullkey` holds the exact key bits, atomic-min'ed by every arrival that
//    lowers or ties the packed prefix.  Two different entries whose keys share
//    the packed prefix raise a per-vector "contest" flag, and the vector's
//    indices are then resolved exactly by a second walk (see below).
//  * Threshold: FastSearch's role (guess how far the queues must be released)
//    is taken by a closed-form time threshold T0 = x_k / sum(v), x_k a high
//    quantile of the maximum of k Exp(1) variables (Sec. 2.5: the normalised
//    y* is that maximum): the 0.97 quantile for vectors walked over all their
//    entries, 1 - 1e-4 for big vectors walked over candidate lists.  Each
//    wave republishes T = min(T0, max_j y_j) every few iterations; registers
//    only decrease, so any snapshot bounds the final y* from above and
//    pruning stays exact.  If a register is still empty after the walk (3%
//    of vectors, or 1e-4 of big ones), the walk is repeated with a doubled
//    threshold (the repeat re-emits the same arrivals, and a minimum does
//    not care).
//  * Probe pass: 64 entries at a time (one per lane, loaded one pass ahead),
//    every lane draws its element's first arrival; it is offered to its
//    register, and an element whose first arrival is within T joins the
//    wave's candidate queue.  This part has no divergence.
//  * Light path: lanes pop candidates and continue their walks from step 2,
//    one arrival per lane per iteration.  The Fisher-Yates state of a walk is
//    the set of displaced positions, kept per lane in a small open-addressing
//    table in LDS (the lane tracks its occupied slots in a register mask, so a new
//    element starts with an empty table for free).
//  * Segment path: an element expected to walk long, or whose table fills
//    up, is listed with its walk state and continued later by a segment of
//    8, 16 or 64 lanes: consecutive arrivals are drawn in parallel, the
//    order-statistic prefix O_z = fma(E_z, c_z, O_{z-1}) is accumulated in
//    its defined serial order by a chain of DPP lane shifts, and the swaps
//    are resolved against a dense LDS permutation by a branch-free pass over
//    the batch's earlier targets.
//  * Exact indices on contest: walk again with the exact final y* and, for
//    every arrival whose key equals its register's final key, atomic-min the
//    element index into the register.
#include <atomic>
#include <cstddef>
#include <cstdio>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "gm.h"
#include "gm_common.h"

namespace gm {

constexpr int kMapSlots = 16;   // per-lane displaced-position table
// Per-wave list (device memory) of elements handed to the segment path.  The
// segment path runs when the light path has drained (list nearly full, or the
// walk is over), so that its dense permutations can reuse the LDS of the
// light path's queue and tables.
constexpr int kHeavyCapG = 512;
constexpr int kQueueCap = 128;  // per-wave candidate queue (probes run while it has room for 64)
// Vectors are grouped by size class (up to kLimM entries, and big) and k
// class (k <= 256, 1024, 2048, 4096) so that each persistent kernel sizes its
// LDS for its own k range.  Class id = size_class * kKClasses + k_class; the
// big classes (size class 1) are contiguous in the planner's list.
constexpr int kSizeClasses = 2;
constexpr int kKClasses = 4;
constexpr int kNumClasses = kSizeClasses * kKClasses;
constexpr int kBigFirst = kKClasses;

__host__ __device__ constexpr int kclass_hi(int kc) { return kc == 0 ? 256 : (kc == 1 ? 1024 : (kc == 2 ? 2048 : 4096)); }

__host__ __device__ inline int kclass_of(int32_t k) {
  return k <= 256 ? 0 : (k <= 1024 ? 1 : (k <= 2048 ? 2 : 3));
}
constexpr int kPlanBins = 32;   // size sub-bins per class (log2 of n)

// An element handed to the segment path, with the state of its walk so far:
// after z steps the order statistic is O and the displaced positions are the
// nent entries (pos-1) << 12 | (value-1); the segment path continues from
// step z + 1.  32 dwords: the fields in dwords 0-9, the entries in 16-31, so
// that the lanes of a segment load a record together, a slice each.
struct HeavyRec {
  uint64_t P;      // hash prefix
  double r;        // 1 / v
  double O;        // O_z
  int32_t unused;  // (keeps the fields' dwords)
  int32_t ind;     // element index
  int32_t z;       // steps done
  int32_t nent;
  uint32_t pad[6];
  uint32_t ent[kMapSlots];
};
static_assert(sizeof(HeavyRec) == 128 && offsetof(HeavyRec, ent) == 64, "heavy record layout");

struct PlanState {
  int count[kNumClasses];
  int offset[kNumClasses];
  int next[kNumClasses];
  int64_t big_chunks;   // chunks of kBigChunk entries over all big vectors
  int parts;            // walk tasks per big vector (1, or kMaxParts when few are big)
};

// Vectors above kLimM entries ("big") are prepared by two grid-wide passes
// before their workgroup walks them: one validates and sums the weights, the
// other draws every entry's first arrival and keeps, in a candidate list,
// the entries whose first arrival is within the closed-form threshold T0.
// Only those can reach a register once y* <= T0 (an element's arrivals only
// grow), so the walk visits the candidates instead of the whole vector.
// The passes hand out chunks of kBigChunk entries, one per workgroup at a
// time: small enough that one 10^7-entry vector spreads over every CU (1221
// chunks of 8192).
constexpr int64_t kBigChunk = 8192;

// A call with at most kSplitMaxBig big vectors walks each one's candidate
// list in up to kMaxParts parts (kPartCand candidates or more each), one
// workgroup per part.  Each part sketches its share into a scratch area;
// the last part to finish merges the partial sketches by the lexicographic
// minimum (Sec. 2.3).  A part prunes at its own y*, which bounds every
// register of the merged sketch, and walks up to T0 at most; so if no merged
// register is empty, the merge is the sketch of the vector.  Otherwise the
// last part walks the vector alone, as an unsplit vector is walked.
// (Stream vector, 10^7 entries, k = 1024, about 15,000 candidates: parts of
// 2048, 1536 and 1024 candidates gave 0.111, 0.109 and 0.115 ms per sketch.)
constexpr int kMaxParts = 16;
constexpr int kPartCand = 1536;
constexpr int kSplitMaxBig = 16;
constexpr int64_t kPartRegs = static_cast<int64_t>(kSplitMaxBig) * kMaxParts * GM_K_MAX;

constexpr int kSumSlots = 16;  // partial sums of a big vector's weights

// The probe pass lists a big vector's candidates in kCandLists sublists,
// work item u in sublist u mod kCandLists, each with a counter of its own
// 128-byte line at the head of the vector's pool region; the gather pass
// then packs them into one list.  (A returning atomic on one address takes
// tens of nanoseconds and every work item's would queue behind the
// others'.)  A sublist that fills up passes its excess to the list itself,
// through one counter (over_count).
constexpr int kCandLists = 16;
constexpr int kCntStride = 32;  // int32 words between two counters
constexpr int64_t kCandHeader = static_cast<int64_t>(kCandLists) * kCntStride;
// A big vector gets a candidate list when the list's room is at most this
// fraction of its entries.
constexpr double kListFrac = 0.8;

struct BigInfo {
  int64_t chunk_base;    // first chunk of this vector
  int64_t cand_off;      // offset of its candidate list in the pool
  int64_t sub_off;       // offset of its kCandLists sublists (the probe's output)
  double S;              // sum of weights: the slots added in order (by the probe pass)
  int bad;               // invalid weight seen (sum pass)
  int bad_index;         // negative index seen (probe pass; read after it)
  int cand_count;        // candidates found (may exceed cand_cap; set by the gather pass)
  int cand_cap;          // room in the pool (0: no list, walk everything)
  int sub_cap;           // room in each sublist
  int over_count;        // candidates past a full sublist, listed at the list's start
  int parts_done;        // parts of a split walk that have written their sketch
  int64_t part_off;      // first scratch register of its parts (kMaxParts x k_max)
  // chunk sums, added atomically into one of kSumSlots slots (one slot per
  // chunk number mod kSumSlots: one address for every chunk would
  // serialise the pass)
  double Sslot[kSumSlots];
};

struct FastArgs {
  SketchArgs s;
  int32_t pos_bits;   // element-index bits in a packed register (31..62)
  double t0_scale;    // multiplies the closed-form threshold (1.0)
  int32_t map_load;   // table entries per lane before the element goes to the wave path
  int32_t republish;  // light iterations between threshold republishes (power of two)
  double seg_rest;    // expected remaining arrivals above which a probe goes to the segment path
  const int32_t* list;  // planner output: vector ids grouped by class
  PlanState* plan;
  BigInfo* big;         // per big vector, in class-list order
  int32_t* pool;        // candidate lists of the big vectors
  int64_t pool_cap;
  int32_t cls;
  int32_t lds_k;        // register-array size this launch's LDS is laid out for
  unsigned long long* stats;  // optional counters (nullptr: off)
  HeavyRec* heavy;      // kHeavyCapG records per resident wave
  int32_t update;       // 1: merge into the sketches already in out_idx/out_val
  int64_t wave_lim;     // vectors of at most this many entries: one wave each (0: none)
  int64_t heavy_waves;  // waves the heavy buffer has room for
  int32_t* part_idx;    // partial sketches of split big vectors (kPartRegs registers)
  double* part_val;
};

// Optional per-call counters (summed over the launch), indices:
enum : int {
  kStVectors = 0,      // vectors sketched
  kStIters = 1,        // light-loop wave iterations
  kStArrivals = 2,     // arrivals drawn on the probe and light paths (lane steps)
  kStKept = 3,         // of which at or below the threshold
  kStElements = 4,     // elements continued on the light path
  kStHeavy = 5,        // elements handed to the segment path
  kStHeavyBatches = 6, // segment batches (one segment each) of that path
  kStPasses = 7,       // extra passes after an unfilled register
  kStResolves = 8,     // exact index resolutions after a contest
  // wave clock cycles (s_memtime, summed over waves) spent in:
  kStCycPrep = 9,      // register init, validation and sum
  kStCycWalk = 10,     // first walk (probe and light path, segment path included)
  kStCycSeg = 11,      // segment path (part of the walk)
  kStCycExtra = 12,    // repeated walks (fallback and exact-index resolve)
  kStCycOut = 13,      // completion checks and writeback
  kStCount = 16
};

enum : int { kWalkNormal = 0, kWalkResolve = 1 };

struct VecCtx {
  const int32_t* idx;  // entries of this vector
  const float* w;
  const int32_t* gather;  // walk these positions only (nullptr: all entries)
  int32_t n;              // entries (or candidates) to walk
  int32_t k;
  uint64_t seed_mix;
  lds_u64* packed;
  lds_u64* fullkey;
  int pos_bits;
  int mode;
  lds_i32* contest;
  int map_load;
  int republish;
  double seg_rest;
  unsigned long long* stats;
};

__device__ __forceinline__ void stat_add(unsigned long long* stats, int which,
                                         unsigned long long v) {
  if (stats && v) atomicAdd(&stats[which], v);
}

// Packed register word of arrival (t, index): the key's top 64 - B bits
// above the index.  (The index itself, not the entry's position, so that
// the writeback needs no gather, and duplicate indices never contest.)
__device__ __forceinline__ unsigned long long packed_key(const VecCtx& c, double t, int32_t ind) {
  const int B = c.pos_bits;
  return ((dbits(t) >> (B - 1)) << B) | static_cast<uint32_t>(ind);
}

// Offer arrival (t, index ind) to register srv.  Normal mode
// returns the packed word the register held before (check it later with
// contest_check); the exact-key minimum needs no answer.
__device__ __forceinline__ unsigned long long reg_offer(const VecCtx& c, int32_t srv, double t,
                                                        unsigned long long pk, int32_t ind) {
  const unsigned long long tb = dbits(t);
  if (c.mode == kWalkResolve) {
    if (tb == c.fullkey[srv])
      lds_min(&c.packed[srv], static_cast<unsigned long long>(static_cast<uint32_t>(ind)));
    return ~0ull;
  }
  lds_min(&c.fullkey[srv], tb);  // result unused: no wait
  return lds_min(&c.packed[srv], pk);
}

// Two different entries whose keys share the packed prefix: the register's
// index must be resolved exactly.
__device__ __forceinline__ void contest_check(const VecCtx& c, unsigned long long old,
                                              unsigned long long pk) {
  const int B = c.pos_bits;
  if ((old >> B) == (pk >> B) && old != pk) *c.contest = 1;
}

__device__ __forceinline__ void reg_update(const VecCtx& c, int32_t srv, double t, int32_t ind) {
  const unsigned long long pk = packed_key(c, t, ind);
  const unsigned long long old = reg_offer(c, srv, t, pk, ind);
  if (c.mode == kWalkNormal) contest_check(c, old, pk);
}

// Power of two at least max(4, k / 64): the segment path's batches between
// threshold republishes.
__device__ __forceinline__ int republish_period(int k) {
  int p = 4;
  while (p * kWave < k) p <<= 1;
  return p;
}

// max_j y_j as seen now (+inf while a register is empty).  The keys are
// non-negative doubles or +inf, whose order is that of their bit patterns:
// each lane takes a double maximum (one instruction per register), the wave
// a bitwise one.
__device__ __forceinline__ double wave_max_register(const VecCtx& c) {
  double m = 0.0;
  for (int j = __lane_id(); j < c.k; j += kWave)
    m = fmax(m, bitsd(*reinterpret_cast<volatile lds_u64*>(&c.fullkey[j])));
  return bitsd(wave_max_u64(dbits(m)));
}

// ---------------------------------------------------------------------------
// c_m = 1/m for m = 1..GM_K_MAX (the step weight 1/(k-z+1) of Eq. 7-8),
// rounded by the compiler's IEEE division, i.e. to the same value the
// device's division gives.  Read from global memory (L1/L2-resident, 32 KB)
// instead of a division sequence per arrival.
struct RecipTab {
  double v[GM_K_MAX + 1];
};
constexpr RecipTab make_recip_tab() {
  RecipTab t{};
  for (int m = 1; m <= GM_K_MAX; ++m) t.v[m] = 1.0 / static_cast<double>(m);
  return t;
}
__device__ constexpr RecipTab kRecip = make_recip_tab();

__device__ __forceinline__ double recip_step(int m) { return kRecip.v[m]; }

// Segment path.  An element whose displaced-position table fills up is walked
// on by a segment of G lanes (G = 8: half a DPP row, eight elements per
// wave; G = 16: one row, four elements; G = 64: the whole wave), G
// consecutive arrivals per batch.  Its permutation is dense in LDS: one u16
// per position, the value minus one in 12 bits (k <= 4096) under a 4-bit
// generation, so that a stale entry reads as the identity and only every
// 15th element of a segment clears the area.

// Bit 0 of every G-lane segment of the wave.
template <int G>
__host__ __device__ constexpr uint64_t seg_first_lanes() {
  uint64_t m = 0;
  for (int i = 0; i < kWave; i += G) m |= 1ull << i;
  return m;
}

// Value of lane l-1 of the segment in lane l; the segment's lane 0 keeps its
// value of `prev` (the DPP's old operand, so that no copy is needed when
// `prev` is the previous shift).  G = 8 shifts whole rows (row_shr:1) and
// keeps the row's lane 8 by a select.
template <int G>
__device__ __forceinline__ double seg_shr1(double v, double prev) {
  constexpr int kCtrl = G == 64 ? 0x138 : 0x111;  // wave_shr:1 / row_shr:1
  const uint64_t b = dbits(v), o = dbits(prev);
  const int lo = __builtin_amdgcn_update_dpp(static_cast<int>(o), static_cast<int>(b), kCtrl, 0xf,
                                             0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(static_cast<int>(o >> 32), static_cast<int>(b >> 32),
                                             kCtrl, 0xf, 0xf, false);
  const double sh =
      bitsd((static_cast<uint64_t>(static_cast<uint32_t>(hi)) << 32) | static_cast<uint32_t>(lo));
  if constexpr (G == 8) return __builtin_amdgcn_inverse_ballot_w64(seg_first_lanes<8>()) ? prev : sh;
  return sh;
}

// Value of segment lane L, in every lane of the segment (row_newbcast:L
// broadcasts lane L of each row of 16; a G = 8 segment in the upper half of
// a row takes row lane 8 + L).
template <int G, int L>
__device__ __forceinline__ uint32_t seg_bcast(uint32_t x) {
  // row_newbcast writes every lane, so no "old" value is needed (bound_ctrl)
  if constexpr (G == 16) {
    return static_cast<uint32_t>(
        __builtin_amdgcn_mov_dpp(static_cast<int>(x), 0x150 + L, 0xf, 0xf, true));
  } else if constexpr (G == 8) {
    const uint32_t a = static_cast<uint32_t>(
        __builtin_amdgcn_mov_dpp(static_cast<int>(x), 0x150 + L, 0xf, 0xf, true));
    const uint32_t b = static_cast<uint32_t>(
        __builtin_amdgcn_mov_dpp(static_cast<int>(x), 0x150 + 8 + L, 0xf, 0xf, true));
    return (__lane_id() & 8u) ? b : a;
  } else {
    return static_cast<uint32_t>(__builtin_amdgcn_readlane(static_cast<int>(x), L));
  }
}

template <int G, int L>
__device__ __forceinline__ double seg_bcast_f64(double v) {
  const uint64_t b = dbits(v);
  const uint32_t lo = seg_bcast<G, L>(static_cast<uint32_t>(b));
  const uint32_t hi = seg_bcast<G, L>(static_cast<uint32_t>(b >> 32));
  return bitsd((static_cast<uint64_t>(hi) << 32) | lo);
}

// Swap step L of a batch.  Lanes after L whose target is j_L read what step
// L moved there (the value it displaced from position z_L); a lane whose own
// position is j_L holds that value from then on; lanes before L with the
// same target lose their write.  The lane-order conditions are wave masks
// (`after`: lanes past L in their segment; `before`: lanes before it).
// Lanes past the segment's stop carry distinct negative targets, which match
// nothing.
template <int G, int L>
__device__ __forceinline__ void fy_step(int32_t j, int32_t z, uint32_t& cval, uint32_t& disp,
                                        uint64_t& after, uint64_t& before, uint64_t& killm) {
  const uint32_t dl = seg_bcast<G, L>(disp);
  const int32_t jl = static_cast<int32_t>(seg_bcast<G, L>(static_cast<uint32_t>(j)));
  const uint64_t eqj = __ballot(j == jl);
  const uint64_t eqz = __ballot(z == jl);
  cval = __builtin_amdgcn_inverse_ballot_w64(eqj & after) ? dl : cval;
  disp = __builtin_amdgcn_inverse_ballot_w64(eqz) ? dl : disp;
  killm |= eqj & before;
  before = (before << 1) | seg_first_lanes<G>();
  after = (after << 1) & after;
}

// Swap step L when no step of the batch targets a position the batch reaches
// later: every lane's displaced value is final from the start, and only
// duplicate targets interact.
template <int G, int L>
__device__ __forceinline__ void fy_step_flat(int32_t j, uint32_t& cval, uint32_t disp,
                                             uint64_t& after, uint64_t& before, uint64_t& killm) {
  const uint32_t dl = seg_bcast<G, L>(disp);
  const int32_t jl = static_cast<int32_t>(seg_bcast<G, L>(static_cast<uint32_t>(j)));
  const uint64_t eqj = __ballot(j == jl);
  cval = __builtin_amdgcn_inverse_ballot_w64(eqj & after) ? dl : cval;
  killm |= eqj & before;
  before = (before << 1) | seg_first_lanes<G>();
  after = (after << 1) & after;
}

// A batch of a 64-lane segment without the sweep.  Step L of the sweep
// swaps positions z_L and j_L, so three rules make it up:
// * a lane whose own position z is the target of earlier lanes takes, as
//   its displaced value, that of the last of them (itself resolved the same
//   way: the chain runs to ever earlier lanes);
// * a lane's server is the displaced value of the last earlier lane with
//   its target, else what it read at its target;
// * a lane's write stands only if no later lane has its target.
// One ballot per bit of j - 1 (j the 1-based target, at most GM_K_MAX) gives
// every lane the lanes whose target equals its own target and those whose
// target equals its position; the chains are followed by pointer jumping, at most
// six rounds for 64 lanes (none when no lane targets a position in its own
// batch).  Lanes past the segment's stop carry negative targets and match
// nothing.
// Bits of j - 1 compared for a segment width: its class bounds k by 256
// (8 lanes), 1024 (16) or GM_K_MAX (64).
template <int G>
constexpr int target_bits() { return G == 8 ? 8 : (G == 16 ? 10 : 12); }
static_assert(GM_K_MAX <= (1 << target_bits<64>()), "targets - 1 must fit the ballot bits");

// `inwin` false: no lane targets a position of its own batch, so no lane's
// displaced value changes during the batch (the chains are empty).
template <int G>
__device__ __forceinline__ bool fy_resolve(int32_t j, int32_t z, bool inwin, uint32_t& cval,
                                           uint32_t& disp) {
  constexpr int kBits = target_bits<G>();
  const uint32_t lane = __lane_id();
  // this lane's segment
  const uint64_t seg =
      G == 64 ? ~0ull : (((1ull << G) - 1ull) << (lane & ~static_cast<uint32_t>(G - 1)));
  const uint64_t valid = __ballot(j >= 0) & seg;
  // The sets are built as complements, per 32-bit half: a lane leaves a set
  // at the first bit of j - 1 where it differs (a lane outside the segment,
  // or invalid, is out from the start).  `m ^ -bit` is zero where a lane
  // agrees with this lane's bit, so each bit costs an xor and an or per
  // half, with the ballot as a scalar operand.
  uint32_t ns_lo = ~static_cast<uint32_t>(valid), ns_hi = ~static_cast<uint32_t>(valid >> 32);
  uint32_t nz_lo = ns_lo, nz_hi = ns_hi;
  const uint32_t jm = static_cast<uint32_t>(j) - 1u, zm = static_cast<uint32_t>(z) - 1u;
  if (inwin) {
#pragma unroll
    for (int b = 0; b < kBits; ++b) {
      const uint64_t m = __ballot(((jm >> b) & 1u) != 0);
      const uint32_t mlo = static_cast<uint32_t>(m), mhi = static_cast<uint32_t>(m >> 32);
      const uint32_t jb = 0u - ((jm >> b) & 1u);
      const uint32_t zb = 0u - ((zm >> b) & 1u);
      ns_lo |= mlo ^ jb;
      ns_hi |= mhi ^ jb;
      nz_lo |= mlo ^ zb;
      nz_hi |= mhi ^ zb;
    }
  } else {
#pragma unroll
    for (int b = 0; b < kBits; ++b) {
      const uint64_t m = __ballot(((jm >> b) & 1u) != 0);
      const uint32_t jb = 0u - ((jm >> b) & 1u);
      ns_lo |= static_cast<uint32_t>(m) ^ jb;
      ns_hi |= static_cast<uint32_t>(m >> 32) ^ jb;
    }
    nz_lo = nz_hi = ~0u;
  }
  // (a lane past the stop, j < 0, neither swaps nor reads: its sets are
  // empty; its position may exceed k, past the bits compared)
  const uint64_t same = j < 0 ? 0ull : ~((static_cast<uint64_t>(ns_hi) << 32) | ns_lo);
  const uint64_t at_z = j < 0 ? 0ull : ~((static_cast<uint64_t>(nz_hi) << 32) | nz_lo);
  const uint64_t below = (1ull << lane) - 1ull;
  // displaced values along the chains of earlier lanes targeting z
  const uint64_t zsrc = at_z & below;
  int ptr = zsrc ? 63 - __clzll(static_cast<long long>(zsrc)) : -1;
  uint32_t val = disp;
  while (__ballot(ptr >= 0) != 0) {
    const int from = ptr >= 0 ? ptr : static_cast<int>(lane);
    const uint32_t v2 = static_cast<uint32_t>(__shfl(static_cast<int>(val), from));
    const int p2 = __shfl(ptr, from);
    if (ptr >= 0) {
      val = v2;
      ptr = p2;
    }
  }
  disp = val;
  const uint64_t earlier = same & below;
  const uint64_t later = same & ~below & ~(1ull << lane);
  const int src = earlier ? 63 - __clzll(static_cast<long long>(earlier)) : static_cast<int>(lane);
  const uint32_t dl = static_cast<uint32_t>(__shfl(static_cast<int>(disp), src));
  if (earlier) cval = dl;
  return later != 0;
}

// `inwin`: some lane of the wave swaps with a position of its own batch
// beyond its step (z_L < j_L <= the batch's last step), so that a later
// step's displaced value changes during the batch.
template <int G, int... Ls>
__device__ __forceinline__ bool fy_batch(std::integer_sequence<int, Ls...>, int32_t j, int32_t z,
                                         bool inwin, uint32_t& cval, uint32_t& disp) {
  // (64-lane segments only: for 8 and 16 lanes the sweep is a few row
  // broadcasts; resolved by ballots as well, they spilled 107 VGPRs and ran
  // 3% slower at k = 256 and 1024)
  if constexpr (G == 64) {
    return fy_resolve<G>(j, z, inwin, cval, disp);
  } else {
    uint64_t after = ~seg_first_lanes<G>(), before = 0, killm = 0;
    // computed step by step with two scalar operations each: folded to
    // constants, the masks of all steps would be hoisted and held in scalar
    // registers across the whole walk
    asm volatile("" : "+s"(after), "+s"(before));
    if (inwin)
      (fy_step<G, Ls>(j, z, cval, disp, after, before, killm), ...);
    else
      (fy_step_flat<G, Ls>(j, cval, disp, after, before, killm), ...);
    return __builtin_amdgcn_inverse_ballot_w64(killm);
  }
}

// Dwords of a heavy record that one lane of a G-lane segment holds when the
// segment loads the record together (a 64-lane segment: lanes 0-31, one each).
template <int G>
constexpr int rec_dwords() { return G >= 32 ? 1 : 32 / G; }

template <int G>
__device__ __forceinline__ void rec_load(const HeavyRec* hr, int li, uint32_t (&d)[rec_dwords<G>()]) {
  constexpr int D = rec_dwords<G>();
  const uint32_t* src = reinterpret_cast<const uint32_t*>(hr) + li * D;
  if constexpr (D == 4) {
    const uint4 v = *reinterpret_cast<const uint4*>(src);
    d[0] = v.x; d[1] = v.y; d[2] = v.z; d[3] = v.w;
  } else if constexpr (D == 2) {
    const uint2 v = *reinterpret_cast<const uint2*>(src);
    d[0] = v.x; d[1] = v.y;
  } else {
    d[0] = li < 32 ? src[0] : 0u;
  }
}

// Dword I of the segment's record, in every lane of the segment.
template <int G, int I>
__device__ __forceinline__ uint32_t rec_field(const uint32_t (&d)[rec_dwords<G>()]) {
  constexpr int D = rec_dwords<G>();
  return seg_bcast<G, I / D>(d[I % D]);
}

template <int G>
__device__ void segment_walk(const VecCtx& c, const HeavyRec* heavy, const lds_i32* counts,
                             int nlists, int nheavy, lds_i32* claim, lds_u16* pm_all, int pm_stride,
                             double& T) {
  constexpr int D = rec_dwords<G>();
  const int lane = __lane_id();
  const int row = lane / G;
  const int li = lane % G;
  lds_u16* pm = pm_all + row * pm_stride;
  // The permutations share LDS with the light path: start from zeros
  // (generation 0 reads as the identity everywhere).
  {
    lds_u64* z8 = reinterpret_cast<lds_u64*>(pm_all);
    const int n8 = (kWave / G) * pm_stride / 4;
    for (int q2 = lane; q2 < n8; q2 += kWave) z8[q2] = 0ull;
  }
  uint32_t hgen = 0;
  // the lists were written by the group's lanes with vector stores
  __threadfence_block();
  const int k = c.k;
  bool active = false;
  int32_t ind = 0;
  double r = 0.0, O = 0.0;
  uint64_t P = 0;
  int z0 = 1;
  int batches = 0, elems = 0;  // per segment (statistics only)
  int round = 0;               // wave-uniform batch counter
  // Batches between threshold republishes: a republish reads all k
  // registers (k/64 per lane), so it is spread over about k/64 batches, at
  // least 4 (document batch at k = 4096: every 4 batches 15.5 ms, every 64
  // 12.6 ms; at k = 1024: every 4 2.13 ms, every 16 2.06 ms).
  const int rp_mask = republish_period(k) - 1;
  // contest check deferred by one batch (hides the atomic's latency)
  bool pend = false;
  unsigned long long pend_old = 0, pend_pk = 0;
  // Each segment holds the record of its next element, loaded when it
  // starts the previous one, so that its load latency is hidden.
  const uint64_t below = row == 0 ? 0ull : (~0ull >> (64 - row * G));
  uint32_t rec[D];
  bool have_rec = false;
  bool drained = false;        // wave-uniform: every record has been claimed
  // Records are claimed from the shared counter, a group of slots per call;
  // slot g is record g of the lists laid end to end (list u at heavy + u
  // kHeavyCapG, counts[u] records).
  auto fetch = [&]() {
    const uint64_t need = __ballot(!have_rec && li == 0);
    if (need && !drained) {
      int base = 0;
      if (lane == 0) base = lds_add(claim, __popcll(need));
      base = readlane_i32(base, 0);
      drained = base + __popcll(need) >= nheavy;
      int slot = base + __popcll(need & below);
      if (!have_rec && slot < nheavy) {
        int u = 0;
        while (u < nlists - 1 && slot >= counts[u]) slot -= counts[u++];
        rec_load<G>(heavy + static_cast<int64_t>(u) * kHeavyCapG + slot, li, rec);
        have_rec = true;
      }
    }
  };
  fetch();
  while (true) {
    // idle segments start their fetched element and fetch the one after it
    if (__ballot(!active && have_rec)) {
      if (!active && have_rec) {
        P = (static_cast<uint64_t>(rec_field<G, 1>(rec)) << 32) | rec_field<G, 0>(rec);
        r = bitsd((static_cast<uint64_t>(rec_field<G, 3>(rec)) << 32) | rec_field<G, 2>(rec));
        O = bitsd((static_cast<uint64_t>(rec_field<G, 5>(rec)) << 32) | rec_field<G, 4>(rec));
        ind = static_cast<int32_t>(rec_field<G, 7>(rec));
        z0 = static_cast<int>(rec_field<G, 8>(rec)) + 1;
        const int nent = static_cast<int>(rec_field<G, 9>(rec));
        active = true;
        have_rec = false;
        ++elems;
        hgen = hgen == 15u ? 1u : hgen + 1u;
        if (hgen == 1u) {
          // every 15th element: clear positions 0..k, four per 8-byte store
          // (the segment's area starts on an 8-byte boundary)
          lds_u64* p8 = reinterpret_cast<lds_u64*>(pm);
          for (int q = li; q < (k + 4) / 4; q += G) p8[q] = 0ull;
        }
        // the displaced positions of the walk so far (dwords 16 + e)
#pragma unroll
        for (int cc = 0; cc < D; ++cc) {
          const int e = li * D + cc - 16;
          if (e >= 0 && e < nent) {
            const uint32_t en = rec[cc];
            pm[(en >> 12) + 1] = static_cast<uint16_t>((hgen << 12) | (en & 0xFFFu));
          }
        }
      }
      fetch();
    }
    if (__ballot(active) == 0) break;
    const int z = z0 + li;
    const bool valid = active && z <= k;
    double E = 0.0, cz = 0.0;
    int32_t j = z;
    uint32_t ej = 0, ez = 0;
    if (valid) {
      j = randint(draw(P, kTagShuffle, static_cast<uint32_t>(z)), z, k);
      // the permutation entries, read before the arrival's draw hides their latency
      ej = pm[j];
      ez = pm[z];
      cz = recip_step(k - z + 1);
      E = exp1(draw(P, kTagArrival, static_cast<uint32_t>(z)));
    }
    // the previous batch's contest check, now that its atomic has returned
    if (pend) contest_check(c, pend_old, pend_pk);
    pend = false;
    // O_z = fma(E_z, c_z, O_{z-1}) in its defined order: after step i lanes
    // 0..i of the segment hold their final value.
    double Ol = fma(E, cz, O);
    double prev = O;
    // (E >= +0, so |E| is E; the modifier selects the three-operand FMA,
    // which leaves `prev` intact for the next shift instead of copying it)
    const double Ea = fabs(E);
#pragma unroll
    for (int i = 1; i < G; ++i) {
      prev = seg_shr1<G>(Ol, prev);
      Ol = fma(Ea, cz, prev);
    }
    const double t = Ol * r;
    const uint64_t stopm = __ballot(valid && t > T);
    const uint64_t validm = __ballot(valid);
    const uint64_t rmask = G == 64 ? ~0ull : ((1ull << G) - 1ull);
    const uint64_t rs = (stopm >> (row * G)) & rmask;
    const int nval = __popcll((validm >> (row * G)) & rmask);
    const int f = rs ? __ffsll(static_cast<long long>(rs)) - 1 : nval;
    uint32_t cval = 0, disp = 0;
    if (li < f) {
      cval = (ej >> 12) == hgen ? (ej & 0xFFFu) + 1u : static_cast<uint32_t>(j);
      disp = (ez >> 12) == hgen ? (ez & 0xFFFu) + 1u : static_cast<uint32_t>(z);
    }
    const int32_t jf = li < f ? j : -1 - li;
    const bool inwin = __ballot(li < f && j > z && j < z0 + f) != 0;
    const bool killed =
        fy_batch<G>(std::make_integer_sequence<int, G>{}, jf, z, inwin, cval, disp);
    if (li < f && !killed) pm[j] = static_cast<uint16_t>((hgen << 12) | (disp - 1u));
    if (li < f) {
      pend_pk = packed_key(c, t, ind);
      pend_old = reg_offer(c, static_cast<int32_t>(cval) - 1, t, pend_pk, ind);
      pend = c.mode == kWalkNormal;
    }
    const bool finished = f < nval || z0 + G > k;
    O = seg_bcast_f64<G, G - 1>(Ol);
    if (active) {
      ++batches;
      if (finished)
        active = false;
      else
        z0 += G;
    }
    // the republish is a wave-wide reduction: keep its condition wave-uniform
    if (c.mode == kWalkNormal && (++round & rp_mask) == 0) T = fmin(T, wave_max_register(c));
  }
  if (pend) contest_check(c, pend_old, pend_pk);
  if (c.stats) {
    const int e2 = wave_sum_i32(li == 0 ? elems : 0);
    const int b2 = wave_sum_i32(li == 0 ? batches : 0);
    if (lane == 0) {
      stat_add(c.stats, kStHeavy, static_cast<unsigned long long>(e2));
      stat_add(c.stats, kStHeavyBatches, static_cast<unsigned long long>(b2));
    }
  }
}

// Per-lane displaced-position table: entry = (pos-1):12 | (val-1):12 in slot
// s of this lane at mp[s * kWave], home slot (pos-1) mod kMapSlots, linear
// probing.  The lane keeps in registers which slots hold entries of its
// current element (`occ`, one bit per slot) and a 64-bit filter of the
// positions entered (`bloom`, bit pos mod 64): most lookups miss, and a
// filter miss needs no LDS read.  A new element starts with both zero.
struct LaneMap {
  uint32_t occ;
  uint64_t bloom;
};

// Home slot of position p.
__device__ __forceinline__ int map_home(uint32_t p) {
  return static_cast<int>((p - 1) & (kMapSlots - 1));
}

// Value at position p (p if not displaced); `slot` receives p's slot when
// found, `found` whether p was present.  `home` is the word of p's home slot,
// read ahead by the caller (trusted only where the slot mask marks the slot).
__device__ __forceinline__ uint32_t map_find(const lds_u32* mp, const LaneMap& m, uint32_t p,
                                             uint32_t home, int& slot, bool& found) {
  found = false;
  slot = -1;
  if (((m.bloom >> (p & 63u)) & 1ull) == 0) return p;
  const uint32_t key = p - 1;
  int s = map_home(p);
  uint32_t e = home;
  for (int q = 0; q < kMapSlots; ++q) {
    if (((m.occ >> s) & 1u) == 0) return p;
    if (q > 0) e = mp[s * kWave];
    if ((e >> 12) == key) {
      slot = s;
      found = true;
      return (e & 0xFFFu) + 1;
    }
    s = (s + 1) & (kMapSlots - 1);
  }
  return p;
}

// First free slot at or after position p's home slot (-1: table full).
__device__ __forceinline__ int map_free_slot(const LaneMap& m, uint32_t p) {
  const uint32_t h = (p - 1) & (kMapSlots - 1);
  const uint32_t fr = ~m.occ & ((1u << kMapSlots) - 1u);
  const uint32_t rot = ((fr >> h) | (fr << (kMapSlots - h))) & ((1u << kMapSlots) - 1u);
  if (rot == 0) return -1;
  return static_cast<int>((h + static_cast<uint32_t>(__builtin_ctz(rot))) & (kMapSlots - 1));
}

__device__ __forceinline__ void map_put(lds_u32* mp, LaneMap& m, int slot, uint32_t p, uint32_t v) {
  mp[slot * kWave] = ((p - 1) << 12) | (v - 1);
  m.occ |= 1u << slot;
  m.bloom |= 1ull << (p & 63u);
}

// Candidate queue of one wave: elements whose first arrival passed the
// threshold, waiting for a lane to continue their walk (structure of arrays).
struct Queue {
  lds_u64* P;
  lds_f64* r;
  lds_f64* O;
  lds_i32* ind;
  lds_u32* j1;
};

__host__ __device__ constexpr size_t queue_bytes() { return kQueueCap * (8 + 8 + 8 + 4 + 4); }

// One wave's share of a walk over the vector's entries.  Each iteration:
//  (a) while the queue has room, a uniform probe pass takes the next 64
//      entries (one per lane): hash prefix, 1/v, first arrival; the first
//      arrival is offered to its register (step 1 of the permutation swaps
//      position 1 with j_1, so it goes to server j_1) and, if it is within
//      the threshold, the element joins the queue;
//  (b) lanes without an element pop one from the queue and continue its walk
//      from step 2; every active lane draws one arrival.
// Elements expected to walk long, and those whose displaced-position table
// fills up, are listed in `hl` (device memory) for the segment path.  When
// the list is nearly full, probing pauses until nothing is in flight on the
// light path, and the wave walks its list alone (`pclaim`: its own claim
// counter); the list left at the end of the walk is returned, for the whole
// group to share.  The segment path reuses the LDS of the queue and the
// tables for its permutations (a lane trusts only the table slots its slot
// mask marks, so nothing needs clearing).  T is the threshold, tightened as
// registers improve.
template <int G>
__device__ int walk_wave(const VecCtx& c, lds_i32* cursor, double& T, HeavyRec* hl, lds_u16* pm,
                         int pm_stride, lds_u32* mp, const Queue& q, lds_i32* pclaim) {
  const int lane = __lane_id();
  const double c1 = 1.0 / static_cast<double>(c.k);
  bool have = false;
  int32_t ind = 0;
  double r = 0.0, O = 0.0;
  uint64_t P = 0;
  int32_t z = 0;
  LaneMap lm;
  lm.occ = 0;
  lm.bloom = 0;
  int qhead = 0, qtail = 0;   // wave-uniform ring counters
  int nheavy = 0;             // wave-uniform heavy-list length
  int iter = 0;
  // contest check deferred by one iteration (hides the atomic's latency)
  bool pend = false;
  unsigned long long pend_old = 0, pend_pk = 0;
  // entries of the next probe pass, loaded one pass ahead
  int pbase = 0;
  if (lane == 0) pbase = lds_add(cursor, kWave);
  pbase = readlane_i32(pbase, 0);
  bool more = pbase < c.n;    // entries left to probe
  float pf_w = 0.0f;
  int32_t pf_i = 0;
  int32_t pf_p = pbase + lane;
  if (pbase + lane < c.n) {
    if (c.gather) pf_p = c.gather[pbase + lane];
    pf_w = c.w[pf_p];
    pf_i = c.idx[pf_p];
  }
  unsigned arrivals = 0, kept = 0, started = 0;
  while (true) {
    // Until the drain: one probe pass and one overflow batch (128) per
    // iteration; after it, at most one append per element in flight or
    // queued (128).
    const bool draining = nheavy > kHeavyCapG - 4 * kWave;
    // (a) probe pass
    if (!draining && more && kQueueCap - (qtail - qhead) >= kWave) {
      const bool inb = pbase + lane < c.n;
      const float wv = pf_w;
      const int32_t pi = pf_i;
      int nb = 0;
      if (lane == 0) nb = lds_add(cursor, kWave);
      pbase = readlane_i32(nb, 0);
      pf_p = pbase + lane;
      if (pbase + lane < c.n) {
        if (c.gather) pf_p = c.gather[pbase + lane];
        pf_w = c.w[pf_p];
        pf_i = c.idx[pf_p];
      }
      bool keep = false, seg = false;
      uint64_t pP = 0;
      double pr = 0.0, pO = 0.0;
      int32_t pj = 1;
      if (inb && wv > 0.0f) {
        pP = mix(c.seed_mix ^ static_cast<uint64_t>(static_cast<uint32_t>(pi)));
        // (the first target does not depend on the arrival's time: drawn
        // ahead of its logarithm)
        pj = randint(draw(pP, kTagShuffle, 1u), 1, c.k);
        pr = 1.0 / static_cast<double>(wv);
        pO = fma(exp1(draw(pP, kTagArrival, 1u)), c1, 0.0);
        const double t = pO * pr;
        ++arrivals;
        if (t <= T) {
          ++kept;
          reg_update(c, pj - 1, t, pi);
          // Arrivals still to come before T arrive at rate about k v: a walk
          // expected to outgrow the lane's table goes to the segment path.
          const bool longwalk =
              static_cast<double>(c.k) * static_cast<double>(wv) * (T - t) > c.seg_rest;
          seg = c.k > 1 && longwalk;
          keep = c.k > 1 && !longwalk;
        }
      }
      const uint64_t sm = __ballot(seg);
      if (seg) {
        // one step done: position j1 holds value 1
        HeavyRec* hr = hl + nheavy + __popcll(sm & lanemask_lt());
        hr->P = pP;
        hr->r = pr;
        hr->O = pO;
        hr->ind = pi;
        hr->z = 1;
        hr->nent = pj != 1 ? 1 : 0;
        hr->ent[0] = static_cast<uint32_t>(pj - 1) << 12;
      }
      nheavy += __popcll(sm);
      const uint64_t km = __ballot(keep);
      if (keep) {
        const int slot = (qtail + __popcll(km & lanemask_lt())) & (kQueueCap - 1);
        q.P[slot] = pP;
        q.r[slot] = pr;
        q.O[slot] = pO;
        q.ind[slot] = pi;
        q.j1[slot] = static_cast<uint32_t>(pj);
      }
      qtail += __popcll(km);
      more = pbase < c.n;
    }
    // (b) refill idle lanes from the queue
    const uint64_t need = __ballot(!have);
    const int avail = qtail - qhead;
    if (need && avail > 0) {
      if (!have) {
        const int rank = __popcll(need & lanemask_lt());
        if (rank < avail) {
          const int slot = (qhead + rank) & (kQueueCap - 1);
          P = q.P[slot];
          r = q.r[slot];
          O = q.O[slot];
          ind = q.ind[slot];
          const uint32_t j1 = q.j1[slot];
          if (O * r <= T) {
            have = true;
            z = 1;
            ++started;
            // after step 1, position j1 holds value 1
            lm.occ = 0;
            lm.bloom = 0;
            if (j1 != 1u) map_put(mp, lm, static_cast<int>((j1 - 1) & (kMapSlots - 1)), j1, 1u);
          }
        }
      }
      const int npop = __popcll(need);
      qhead += npop < avail ? npop : avail;
    }
    const bool any_have = __ballot(have) != 0;
    // nothing in flight on the light path
    const bool idle = !any_have && qtail == qhead;
    bool overflow = false;
    if (any_have) {
      if (have) {
        ++z;
        // The step's target and the home slots of positions z and j do not
        // depend on the arrival's time: drawn and read ahead of its
        // logarithm, off the chain that decides whether the walk goes on.
        const uint32_t hz = mp[map_home(static_cast<uint32_t>(z)) * kWave];
        const int32_t j = randint(draw(P, kTagShuffle, static_cast<uint32_t>(z)), z, c.k);
        const uint32_t hj = mp[map_home(static_cast<uint32_t>(j)) * kWave];
        const double E = exp1(draw(P, kTagArrival, static_cast<uint32_t>(z)));
        const double On = fma(E, recip_step(c.k - z + 1), O);
        const double t = On * r;
        ++arrivals;
        if (pend) contest_check(c, pend_old, pend_pk);
        pend = false;
        if (t > T) {
          have = false;
        } else {
          ++kept;
          int zslot, jslot;
          bool zfound, jfound;
          const uint32_t vz = map_find(mp, lm, static_cast<uint32_t>(z), hz, zslot, zfound);
          const uint32_t vj = map_find(mp, lm, static_cast<uint32_t>(j), hj, jslot, jfound);
          if (j != z) {
            // position j now holds the value position z held
            if (!jfound) {
              jslot = __popc(lm.occ) < c.map_load ? map_free_slot(lm, static_cast<uint32_t>(j)) : -1;
              if (jslot < 0) overflow = true;
            }
            if (!overflow) map_put(mp, lm, jslot, static_cast<uint32_t>(j), vz);
          }
          if (overflow) {
            have = false;
          } else {
            O = On;
            pend_pk = packed_key(c, t, ind);
            pend_old = reg_offer(c, static_cast<int32_t>(vj) - 1, t, pend_pk, ind);
            pend = c.mode == kWalkNormal;
            if (z == c.k) have = false;
          }
        }
      }
      ++iter;
      // (the option's period at k <= 256, scaled with k above: each
      // republish reads k/64 registers per lane)
      if (c.mode == kWalkNormal && (iter & (c.republish * (republish_period(c.k) / 4) - 1)) == 0)
        T = fmin(T, wave_max_register(c));
    }
    const uint64_t om = __ballot(overflow);
    if (overflow) {
      // hand the walk over after z - 1 steps, with its displaced positions
      HeavyRec* hr = hl + nheavy + __popcll(om & lanemask_lt());
      hr->P = P;
      hr->r = r;
      hr->O = O;
      hr->ind = ind;
      hr->z = z - 1;
      int ne = 0;
      for (int s2 = 0; s2 < kMapSlots; ++s2)
        if ((lm.occ >> s2) & 1u) hr->ent[ne++] = mp[s2 * kWave];
      hr->nent = ne;
    }
    nheavy += __popcll(om);
    if (idle && (draining || !more)) {
      if (pend) {
        contest_check(c, pend_old, pend_pk);
        pend = false;
      }
      if (!more) break;
      if (nheavy > 0) {
        const uint64_t c0 = c.stats ? clock64() : 0;
        if (lane == 0) *pclaim = 0;
        segment_walk<G>(c, hl, nullptr, 1, nheavy, pclaim, pm, pm_stride, T);
        if (c.stats && lane == 0) stat_add(c.stats, kStCycSeg, clock64() - c0);
        nheavy = 0;
      }
    }
  }
  if (c.stats) {
    const int a = wave_sum_i32(static_cast<int>(arrivals));
    const int kk = wave_sum_i32(static_cast<int>(kept));
    const int st = wave_sum_i32(static_cast<int>(started));
    if (lane == 0) {
      stat_add(c.stats, kStIters, static_cast<unsigned long long>(iter));
      stat_add(c.stats, kStArrivals, static_cast<unsigned long long>(a));
      stat_add(c.stats, kStKept, static_cast<unsigned long long>(kk));
      stat_add(c.stats, kStElements, static_cast<unsigned long long>(st));
    }
  }
  return nheavy;
}

// (1 - p) quantile of the maximum of k Exp(1) variables: a vector's final
// y* exceeds x/S with probability p (Sec. 2.5).
__device__ __forceinline__ double max_exp_quantile(int k, double p = 1e-4) {
  return -log(-expm1(log1p(-p) / static_cast<double>(k)));
}

// Miss probability of the first walk's threshold for vectors walked over all
// their entries.  A miss (an empty register) costs one more walk with the
// threshold doubled, past the 1e-4 quantile; a tighter first threshold saves
// the arrivals between the two quantiles on every other vector, which
// matters most for large k, where the registers fill late in the walk and
// the running maximum cannot tighten the threshold before that.
constexpr double kFirstMiss = 0.03;

__host__ __device__ constexpr int perm_stride(int k_max) { return ((k_max + 1 + 3) / 4) * 4; }

// Lanes per segment of the segment path: 8 (eight elements per wave) or 16
// (four) while that many dense permutations stay small, else the whole wave.
__host__ __device__ constexpr int segment_lanes(int k_max) {
  return k_max <= 256 ? 8 : (k_max <= 1024 ? 16 : 64);
}

__host__ __device__ constexpr size_t light_lds_bytes() {
  return queue_bytes() + static_cast<size_t>(kMapSlots) * kWave * 4;
}

__host__ __device__ constexpr size_t perm_lds_bytes(int k_max) {
  return static_cast<size_t>(kWave / segment_lanes(k_max)) * perm_stride(k_max) * 2;
}

// Per-wave LDS: the light path's queue and tables, or (at other times) the
// segment path's permutations, whichever is larger; 16-byte multiple.
__host__ __device__ constexpr size_t wave_lds_bytes(int k_max) {
  return ((light_lds_bytes() > perm_lds_bytes(k_max) ? light_lds_bytes() : perm_lds_bytes(k_max)) +
          15) / 16 * 16;
}

// Dynamic LDS of a class kernel: reg_sets register arrays (one per wave when
// waves take vectors of their own) and each wave's working area.
size_t fastgm_lds_bytes(int k_max, int waves, int reg_sets) {
  return 16 * static_cast<size_t>(k_max) * reg_sets + waves * wave_lds_bytes(k_max);
}

struct FgShared {
  int cursor;
  int contest;
  int bad;
  int task;
  int last;         // this workgroup finished the last part of a split walk
  int hclaim;       // claim counter of the group's final heavy lists
  int hcount[16];   // records in each wave's final list
  int pclaim[16];   // each wave's own claim counter (lists walked alone)
  double wsum[16];
  unsigned long long wmax[16];
};

// Barrier of a group of GW waves (one wave: only keeps the compiler from
// moving LDS accesses across it; a wave executes its LDS operations in order).
template <int GW>
__device__ __forceinline__ void group_sync() {
  if constexpr (GW == 1)
    __builtin_amdgcn_wave_barrier();
  else
    __syncthreads();
}

template <int GW>
__device__ __forceinline__ bool group_or(bool b) {
  if constexpr (GW == 1) {
    __builtin_amdgcn_wave_barrier();
    return __ballot(b) != 0;
  } else {
    return __syncthreads_or(b) != 0;
  }
}

// One part of a split walk (see kMaxParts): part `part` of `parts` walks
// that share of the vector's candidate list into its scratch registers.
struct PartTask {
  int part, parts;
};

// Sketch vector v with a group of GW waves: the whole workgroup (GW = W) or
// a single wave (GW = 1) with its own registers and shared words.  With a
// part task, the workgroup sketches one part of a big vector and, if it is
// the last part to finish, merges the parts into the output; it returns
// true when the merged sketch has an empty register (the caller then walks
// the vector unsplit).
template <int GW, int G>
__device__ bool sketch_vector(const FastArgs& fa, int64_t v, BigInfo* bi, FgShared& sh,
                              lds_u64* packed, lds_u64* fullkey, lds_u16* pm, int pm_stride,
                              HeavyRec* hl, lds_u32* mp, const Queue& q,
                              const PartTask* pt = nullptr) {
  constexpr int kBlock = GW * kWave;
  const SketchArgs& p = fa.s;
  const int lane = threadIdx.x % kWave;
  const int tid = GW == 1 ? lane : static_cast<int>(threadIdx.x);
  const int wave = GW == 1 ? 0 : static_cast<int>(threadIdx.x) / kWave;
  const VecDesc d = vec_desc(p, v);
  const int32_t span = out_span(p, v, d);
  const int64_t n64 = d.b - d.a;
  // where this sketch goes: the output, or a part's scratch registers
  int32_t* const oidx = pt ? fa.part_idx : p.out_idx;
  double* const oval = pt ? fa.part_val : p.out_val;
  const int64_t obase = pt ? bi->part_off + static_cast<int64_t>(pt->part) * d.k : d.o;
  const bool bad0 = d.bad || n64 > 0x7FFFFFFF;
  // optional per-phase cycle accounting (statistics mode only)
  const bool timed = fa.stats != nullptr;
  uint64_t cyc = timed ? clock64() : 0;
  auto lap = [&](int slot) {
    if (timed) {
      const uint64_t now = clock64();
      if (lane == 0) stat_add(fa.stats, slot, now - cyc);
      cyc = now;
    }
  };
  if (tid == 0) {
    sh.bad = bad0 ? 1 : 0;
    sh.contest = 0;
    sh.cursor = 0;
  }
  if (!bad0) {
    for (int j = tid; j < d.k; j += kBlock) {
      packed[j] = ~0ull;
      fullkey[j] = kInfBits;
    }
  }
  group_sync<GW>();
  // Validation and the mass S = sum(v) (its rounding only moves T0); a big
  // vector had both done by the grid-wide pass.
  double part = 0.0;
  bool badl = false;
  if (bi) {
    if (tid == 0) {
      part = bi->S;
      badl = bi->bad != 0 || bi->bad_index != 0;
    }
  } else if (!bad0) {
    // four independent loads per lane in flight per step (the pass is
    // latency-bound otherwise)
    constexpr int kU = 4;
    int64_t e = d.a + tid;
    for (; e + (kU - 1) * kBlock < d.b; e += kU * kBlock) {
      int32_t iv[kU];
      float wv[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        iv[u] = p.idx[e + u * kBlock];
        wv[u] = p.w[e + u * kBlock];
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        if (iv[u] < 0 || !weight_valid(wv[u]))
          badl = true;
        else
          part += static_cast<double>(wv[u]);
      }
    }
    for (; e < d.b; e += kBlock) {
      const int32_t i = p.idx[e];
      const float wv = p.w[e];
      if (i < 0 || !weight_valid(wv))
        badl = true;
      else
        part += static_cast<double>(wv);
    }
  }
  if (badl) sh.bad = 1;
  part = wave_sum_f64(part);
  if (lane == 0) sh.wsum[wave] = part;
  group_sync<GW>();
  double S = 0.0;
  for (int qq = 0; qq < GW; ++qq) S += sh.wsum[qq];
  lap(kStCycPrep);
  if (sh.bad || !(S > 0.0)) {
    // an update with no positive entry leaves the stored sketch as it is
    const bool bad = sh.bad != 0;
    if (bad || !fa.update) {
      for (int j = tid; j < span; j += kBlock) {
        p.out_idx[d.o + j] = bad ? kIdxPoison : kIdxEmpty;
        p.out_val[d.o + j] = bitsd(bad ? kNanBits : kInfBits);
      }
    }
    if (bad && tid == 0) atomicAdd(p.err, 1ull);
    group_sync<GW>();
    return false;
  }
  // Update: the stored sketch is the sketch of the entries seen so far, so
  // an arrival above its largest register cannot change the merged result
  // (lexicographic minimum over the union, Sec. 2.3): its y* caps the walk.
  double cap = bitsd(kInfBits);
  if (fa.update) {
    unsigned long long m = 0;
    bool poisoned = false, empty = false;
    for (int j = tid; j < d.k; j += kBlock) {
      const int32_t si = p.out_idx[d.o + j];
      if (si == kIdxPoison)
        poisoned = true;
      else if (si < 0)
        empty = true;
      else
        m = dbits(p.out_val[d.o + j]) > m ? dbits(p.out_val[d.o + j]) : m;
    }
    m = wave_max_u64(m);
    if (lane == 0) sh.wmax[wave] = m;
    const bool any_poison = group_or<GW>(poisoned);  // also orders the wmax writes
    const bool any_empty = group_or<GW>(empty);
    if (any_poison) return false;  // a poisoned sketch stays poisoned
    unsigned long long ms = 0;
    for (int qq = 0; qq < GW; ++qq) ms = sh.wmax[qq] > ms ? sh.wmax[qq] : ms;
    if (!any_empty) cap = bitsd(ms);
    group_sync<GW>();
  }

  VecCtx c;
  c.idx = p.idx + d.a;
  c.w = p.w + d.a;
  c.gather = nullptr;
  c.n = static_cast<int32_t>(n64);
  if (bi && bi->cand_cap > 0 && bi->cand_count <= bi->cand_cap) {
    c.gather = fa.pool + bi->cand_off;
    c.n = bi->cand_count;
    if (pt) {
      const int lo = static_cast<int>(static_cast<int64_t>(bi->cand_count) * pt->part / pt->parts);
      const int hi = static_cast<int>(static_cast<int64_t>(bi->cand_count) * (pt->part + 1) / pt->parts);
      c.gather += lo;
      c.n = hi - lo;
    }
  }
  c.k = d.k;
  c.seed_mix = p.seed_mix;
  c.packed = packed;
  c.fullkey = fullkey;
  c.pos_bits = fa.pos_bits;
  c.mode = kWalkNormal;
  c.contest = (lds_i32*)(&sh.contest);  // address-space cast of a __shared__ object
  c.map_load = fa.map_load;
  c.republish = fa.republish;
  c.seg_rest = fa.seg_rest;
  c.stats = fa.stats;
  if (tid == 0) stat_add(fa.stats, kStVectors, 1);
  lds_i32* cursor = (lds_i32*)(&sh.cursor);

  // Walk with the closed-form threshold; repeat with a larger one while a
  // register is empty; then, if two entries tied on a packed prefix, walk
  // once more to resolve the indices exactly.  One call site keeps a single
  // copy of the walk in the kernel.
  // big vectors keep the quantile their candidate lists were cut at
  double T = fmin(max_exp_quantile(d.k, bi ? 1e-4 : kFirstMiss) * fa.t0_scale / S, cap);
  // a part leaves a register empty rather than walk further: the other
  // parts may fill it
  if (pt) cap = T;
  const double T_walk = T;  // the threshold every part walks to
  bool resolve = false;
  lds_i32* pclaim = (lds_i32*)(&sh.pclaim[wave]);
  lds_i32* hcount = (lds_i32*)(&sh.hcount[0]);
  lds_i32* hclaim = (lds_i32*)(&sh.hclaim);
  for (int pass = 0;; ++pass) {
    double Tw = T;
    const int nh = walk_wave<G>(c, cursor, Tw, hl, pm, pm_stride, mp, q, pclaim);
    // The waves' final heavy lists are walked by the whole group, each wave
    // claiming records from all of them: no wave waits on another's list.
    if (lane == 0) hcount[wave] = nh;
    if (tid == 0) *hclaim = 0;
    group_sync<GW>();
    int total = 0;
    for (int u = 0; u < GW; ++u) total += hcount[u];
    if (total > 0) {
      const uint64_t c0 = timed ? clock64() : 0;
      segment_walk<G>(c, hl - static_cast<int64_t>(wave) * kHeavyCapG, hcount, GW, total, hclaim, pm,
                      pm_stride, Tw);
      if (timed && lane == 0) stat_add(fa.stats, kStCycSeg, clock64() - c0);
    }
    group_sync<GW>();
    lap(pass == 0 ? kStCycWalk : kStCycExtra);
    if (resolve) break;
    bool miss = false;
    for (int j = tid; j < d.k; j += kBlock) miss |= fullkey[j] == kInfBits;
    // (under an update's cap, a register left empty keeps its stored value)
    if (group_or<GW>(miss) && T < cap) {
      if (tid == 0) stat_add(fa.stats, kStPasses, 1);
      T = fmin(pass >= 8 ? bitsd(kInfBits) : T * 2.0, cap);
      // above T0 the candidate list no longer covers every element
      c.gather = nullptr;
      c.n = static_cast<int32_t>(n64);
      if (tid == 0) sh.cursor = 0;
      group_sync<GW>();
      continue;
    }
    if (sh.contest == 0) break;
    // exact indices: walk again with the exact y*, keeping the index of every
    // arrival that equals its register's final key
    resolve = true;
    if (tid == 0) stat_add(fa.stats, kStResolves, 1);
    unsigned long long m = 0;
    for (int j = tid; j < d.k; j += kBlock)
      if (fullkey[j] != kInfBits) m = fullkey[j] > m ? fullkey[j] : m;
    m = wave_max_u64(m);
    if (lane == 0) sh.wmax[wave] = m;
    group_sync<GW>();
    unsigned long long ystar = 0;
    for (int qq = 0; qq < GW; ++qq) ystar = sh.wmax[qq] > ystar ? sh.wmax[qq] : ystar;
    for (int j = tid; j < d.k; j += kBlock) packed[j] = ~0ull;
    if (tid == 0) sh.cursor = 0;
    group_sync<GW>();
    c.mode = kWalkResolve;
    T = bitsd(ystar);
  }
  // Write back: the winner's index is the packed word's low bits (after a
  // resolve walk, the whole word).  An update keeps the lexicographic
  // (value, index) minimum with the stored register (a part of a split walk
  // leaves that to the merge; a register an update's cap left empty keeps
  // its stored value).
  const unsigned long long pmask = (1ull << fa.pos_bits) - 1ull;
  for (int j = tid; j < d.k; j += kBlock) {
    const unsigned long long pk = packed[j];
    const unsigned long long fk = fullkey[j];
    const int32_t oi = resolve ? static_cast<int32_t>(pk)
                               : (fk != kInfBits ? static_cast<int32_t>(pk & pmask) : kIdxEmpty);
    bool take = true;
    if (fa.update && !pt) {
      const int32_t si = p.out_idx[d.o + j];
      const unsigned long long sv = dbits(p.out_val[d.o + j]);
      take = fk != kInfBits && (si < 0 || fk < sv || (fk == sv && oi < si));
    }
    if (take) {
      oidx[obase + j] = oi;
      oval[obase + j] = bitsd(fk);
    }
  }
  group_sync<GW>();
  lap(kStCycOut);
  if (!pt) return false;
  // Publish this part's sketch; the last part to finish merges them all.
  __threadfence();
  group_sync<GW>();
  if (tid == 0) sh.last = atomicAdd(&bi->parts_done, 1) == pt->parts - 1 ? 1 : 0;
  group_sync<GW>();
  if (!sh.last) return false;
  __threadfence();
  // A register is settled when a part filled it or, in an update, when the
  // stored register lies within the parts' threshold T (no arrival above T
  // was drawn, none at or below it was missed).  Merged registers written
  // before an unsettled one sends the vector to the unsplit walk hold
  // min(stored, new): walking the new entries again changes nothing more.
  bool empty = false;
  const unsigned long long tb = dbits(T_walk);
  for (int j = tid; j < d.k; j += kBlock) {
    int32_t wi = kIdxEmpty;
    unsigned long long wv = kInfBits;
    for (int qq = 0; qq < pt->parts; ++qq) {
      const int64_t r = bi->part_off + static_cast<int64_t>(qq) * d.k + j;
      const int32_t si = fa.part_idx[r];
      const unsigned long long sv = dbits(fa.part_val[r]);
      if (si >= 0 && (wi < 0 || sv < wv || (sv == wv && si < wi))) {
        wi = si;
        wv = sv;
      }
    }
    bool settled = wi >= 0;
    if (fa.update) {
      const int32_t si = p.out_idx[d.o + j];
      const unsigned long long sv = dbits(p.out_val[d.o + j]);
      if (si >= 0 && sv <= tb) settled = true;
      if (si >= 0 && (wi < 0 || sv < wv || (sv == wv && si < wi))) {
        wi = si;
        wv = sv;
      }
    }
    if (!settled) {
      empty = true;
    } else {
      p.out_idx[d.o + j] = wi;
      p.out_val[d.o + j] = bitsd(wv);
    }
  }
  return group_or<GW>(empty);
}

// Persistent kernel of one class: workgroups of W waves pull vector ids from
// the class list (largest first) until it is exhausted.  A vector larger
// than fa.wave_lim is sketched by the whole workgroup; once the list reaches
// vectors of at most fa.wave_lim entries, every wave takes vectors of its own
// (with its own registers), so that the last large vectors overlap with the
// small ones instead of leaving the other workgroups idle.  kSplit: the
// classes of big vectors, whose walks may be split (see kMaxParts); they
// have a kernel of their own, so that the other classes carry none of it.
template <int W, int G, bool kSplit>
__device__ __forceinline__ void class_body(const FastArgs& fa) {
  extern __shared__ __align__(16) unsigned char dyn[];
  __shared__ FgShared sh[W];
  const int k_max = fa.lds_k;
  const int wave = threadIdx.x / kWave;
  const int reg_sets = fa.wave_lim > 0 ? W : 1;
  GM_LDS unsigned char* base = (GM_LDS unsigned char*)(dyn);  // address-space cast
  lds_u64* regs = reinterpret_cast<lds_u64*>(base);           // reg_sets x (packed, fullkey)
  GM_LDS unsigned char* wave_base = reinterpret_cast<GM_LDS unsigned char*>(regs + 2 * k_max * reg_sets) +
                                    wave * wave_lds_bytes(k_max);
  Queue q;
  q.P = reinterpret_cast<lds_u64*>(wave_base);
  q.r = reinterpret_cast<lds_f64*>(wave_base + kQueueCap * 8);
  q.O = reinterpret_cast<lds_f64*>(wave_base + kQueueCap * 16);
  q.ind = reinterpret_cast<lds_i32*>(wave_base + kQueueCap * 24);
  q.j1 = reinterpret_cast<lds_u32*>(wave_base + kQueueCap * 28);
  lds_u32* mp_base = reinterpret_cast<lds_u32*>(wave_base + queue_bytes());
  // the segment path's permutations reuse the same bytes
  lds_u16* pm = reinterpret_cast<lds_u16*>(wave_base);
  const int pm_stride = perm_stride(k_max);
  HeavyRec* hl = fa.heavy + (static_cast<int64_t>(blockIdx.x) * W + wave) * kHeavyCapG;
  const int lane = threadIdx.x % kWave;
  lds_u32* mp = mp_base + lane;

  const PlanState* plan = fa.plan;
  const int count = plan->count[fa.cls];
  const int32_t* list = fa.list + plan->offset[fa.cls];
  int* next = &fa.plan->next[fa.cls];
  // big vectors: `parts` tasks each (parts of a split walk, see kMaxParts)
  const bool bigc = fa.cls >= kBigFirst && fa.big;
  const int parts = kSplit && bigc ? plan->parts : 1;
  // Tasks b, b + n, .., b + (W - 1) n (n workgroups) belong to workgroup b
  // from the start: each of the first W rounds of the sorted list gives
  // every workgroup one task, largest first, as the counter would.  The
  // class counter hands out the rest, from n W on.  Without the static
  // share every wave of the grid would claim its first task from the one
  // counter at the same moment, and those device-scope atomics serialise.
  const int ngroups = static_cast<int>(gridDim.x);
  const int nstatic = ngroups * W;
  int used = 0;  // static tasks of this workgroup taken so far
  int t = 0;
  for (;;) {
    if (used < W) {
      t = static_cast<int>(blockIdx.x) + used * ngroups;
      ++used;
      __syncthreads();  // the previous vector's last reads of the shared state
    } else {
      if (threadIdx.x == 0) sh[0].task = nstatic + atomicAdd(next, 1);
      __syncthreads();
      t = sh[0].task;
      __syncthreads();
    }
    if (t >= count * parts) return;
    const int ti = t / parts;
    const int part = t - ti * parts;
    const int64_t v = list[ti];
    if (fa.wave_lim > 0 && fa.s.off[v + 1] - fa.s.off[v] <= fa.wave_lim) break;
    BigInfo* bi = bigc ? &fa.big[plan->offset[fa.cls] - plan->offset[kBigFirst] + ti] : nullptr;
    int np = 1;
    if (parts > 1 && !bi->bad && !bi->bad_index && bi->S > 0.0 && bi->cand_cap > 0 &&
        bi->cand_count <= bi->cand_cap) {
      const int want = bi->cand_count / kPartCand;
      np = want < 1 ? 1 : (want > parts ? parts : want);
    }
    if (part >= np) continue;
    const PartTask pt{part, np};
    // (one call site, so that the walk is inlined once; a split walk whose
    // merge left a register empty is walked again, unsplit)
    bool split = kSplit && np > 1;
    for (;;) {
      const bool redo = sketch_vector<W, G>(fa, v, bi, sh[0], regs, regs + k_max, pm, pm_stride, hl,
                                            mp, q, split ? &pt : nullptr);
      if (!redo) break;
      split = false;
    }
  }
  // one vector per wave from here on: wave 0 starts with the task in hand,
  // waves 1.. with the workgroup's remaining static tasks, if any
  lds_u64* wpacked = regs + 2 * k_max * wave;
  const int si = used + wave - 1;
  int mt = wave == 0 ? t : (si < W ? static_cast<int>(blockIdx.x) + si * ngroups : -1);
  for (;;) {
    if (mt < 0) {
      int got = 0;
      if (lane == 0) got = nstatic + atomicAdd(next, 1);
      mt = readlane_i32(got, 0);
    }
    if (mt >= count) break;
    sketch_vector<1, G>(fa, list[mt], nullptr, sh[wave], wpacked, wpacked + k_max, pm, pm_stride,
                        hl, mp, q);
    mt = -1;
  }
}

// Waves per SIMD the register allocation aims for: three (168 VGPRs) where
// the LDS lets three waves per SIMD in; the 64-lane-segment classes
// (k > 1024) hold one workgroup of eight waves per CU by their LDS, so two
// waves per SIMD, and may use the 256 VGPRs that leaves without spilling.
template <int G>
constexpr int class_waves_per_eu() { return G == 64 ? 2 : 3; }

template <int W, int G>
__global__ __launch_bounds__(W * kWave) __attribute__((amdgpu_waves_per_eu(class_waves_per_eu<G>())))
void fastgm_class_kernel(FastArgs fa) {
  class_body<W, G, false>(fa);
}

// The big-vector kernels walk few vectors, a split walk's parts one
// workgroup each: they run at two waves per SIMD without spills.  (With
// spills, even a launch with no big vector wrote each lane's spill slots
// before it could exit: 16 MiB per call.)
template <int W, int G>
__global__ __launch_bounds__(W * kWave) __attribute__((amdgpu_waves_per_eu(2)))
void fastgm_big_kernel(FastArgs fa) {
  class_body<W, G, true>(fa);
}

// Planner: one workgroup sorts the vector ids by (size class, decreasing
// log2 size) with a counting sort, and resets the classes' work counters.
constexpr int kPlanBlock = 1024;

__device__ __forceinline__ int plan_bin(const SketchArgs& p, int64_t v, int64_t lim_m) {
  const int64_t n = p.off[v + 1] - p.off[v];
  const int32_t k = p.kvec ? p.kvec[v] : p.k_uniform;
  const int sc = n <= lim_m ? 0 : 1;
  const int kc = (k >= 1 && k <= p.k_max) ? kclass_of(k) : 0;
  const int cls = sc * kKClasses + kc;
  const int lg = n > 0 ? 63 - __clzll(static_cast<unsigned long long>(n)) : 0;
  return cls * kPlanBins + (kPlanBins - 1 - (lg < kPlanBins ? lg : kPlanBins - 1));
}

__global__ __launch_bounds__(kPlanBlock) void plan_kernel(SketchArgs p, int32_t* list,
                                                          PlanState* plan, BigInfo* big,
                                                          int32_t* pool, int64_t pool_cap, double t0_scale,
                                                          int64_t lim_m) {
  __shared__ int hist[kNumClasses * kPlanBins];
  __shared__ int base[kNumClasses * kPlanBins];
  const int tid = threadIdx.x;
  for (int b = tid; b < kNumClasses * kPlanBins; b += kPlanBlock) hist[b] = 0;
  __syncthreads();
  for (int64_t v = tid; v < p.nvec; v += kPlanBlock) atomicAdd(&hist[plan_bin(p, v, lim_m)], 1);
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int b = 0; b < kNumClasses * kPlanBins; ++b) {
      base[b] = acc;
      acc += hist[b];
    }
    for (int c = 0; c < kNumClasses; ++c) {
      plan->offset[c] = base[c * kPlanBins];
      int cnt = 0;
      for (int b = 0; b < kPlanBins; ++b) cnt += hist[c * kPlanBins + b];
      plan->count[c] = cnt;
      plan->next[c] = 0;
    }
  }
  __syncthreads();
  for (int64_t v = tid; v < p.nvec; v += kPlanBlock) {
    const int b = plan_bin(p, v, lim_m);
    list[atomicAdd(&base[b], 1)] = static_cast<int32_t>(v);
  }
  __syncthreads();
  // Big vectors: chunk ranges and candidate-list room, by exclusive scans.
  __shared__ int64_t sc_ch[kPlanBlock];
  __shared__ int64_t sc_cap[kPlanBlock];
  __shared__ int64_t run_ch, run_cap;
  int c2 = 0;
  for (int cc = kBigFirst; cc < kNumClasses; ++cc) c2 += plan->count[cc];
  const int32_t* list2 = list + plan->offset[kBigFirst];
  if (tid == 0) {
    run_ch = 0;
    run_cap = 0;
  }
  __syncthreads();
  for (int b0 = 0; b0 < c2; b0 += kPlanBlock) {
    const int i = b0 + tid;
    int64_t nch = 0, cap = 0;
    if (i < c2) {
      const int64_t v = list2[i];
      const int64_t n = p.off[v + 1] - p.off[v];
      const int32_t k = p.kvec ? p.kvec[v] : p.k_uniform;
      nch = (n + kBigChunk - 1) / kBigChunk;
      if (k >= 1 && k <= p.k_max) {
        const double x = static_cast<double>(k) * max_exp_quantile(k) * (t0_scale > 1.0 ? t0_scale : 1.0);
        const int64_t c = static_cast<int64_t>(1.25 * x + 4.0 * sqrt(x) + 256.0);
        // a list that may hold most of the entries saves the walk little
        // and the probe's first arrivals would all be drawn twice: such a
        // vector is walked over all its entries
        cap = static_cast<double>(c) <= kListFrac * static_cast<double>(n) ? c : 0;
      }
    }
    // pool region: sublist counters, sublists, the list
    const int64_t scap = ((cap + kCandLists - 1) / kCandLists + 31) / 32 * 32;
    const int64_t region = cap > 0 ? kCandHeader + kCandLists * scap + cap : 0;
    sc_ch[tid] = nch;
    sc_cap[tid] = region;
    __syncthreads();
    for (int d = 1; d < kPlanBlock; d <<= 1) {
      const int64_t a1 = tid >= d ? sc_ch[tid - d] : 0;
      const int64_t a2 = tid >= d ? sc_cap[tid - d] : 0;
      __syncthreads();
      sc_ch[tid] += a1;
      sc_cap[tid] += a2;
      __syncthreads();
    }
    if (i < c2) {
      BigInfo bi;
      bi.chunk_base = run_ch + sc_ch[tid] - nch;
      const int64_t r0 = run_cap + sc_cap[tid] - region;
      bi.sub_off = r0 + kCandHeader;
      bi.cand_off = bi.sub_off + kCandLists * scap;
      bi.S = 0.0;
      for (int q = 0; q < kSumSlots; ++q) bi.Sslot[q] = 0.0;
      bi.bad = 0;
      bi.bad_index = 0;
      bi.cand_count = 0;
      bi.cand_cap = (cap > 0 && r0 + region <= pool_cap) ? static_cast<int>(cap) : 0;
      bi.sub_cap = static_cast<int>(scap);
      bi.over_count = 0;
      if (bi.cand_cap > 0)
        for (int q = 0; q < kCandLists; ++q) pool[r0 + q * kCntStride] = 0;
      bi.parts_done = 0;
      bi.part_off = static_cast<int64_t>(i) * kMaxParts * GM_K_MAX;
      big[i] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      run_ch += sc_ch[kPlanBlock - 1];
      run_cap += sc_cap[kPlanBlock - 1];
    }
    __syncthreads();
  }
  if (tid == 0) {
    plan->big_chunks = run_ch;
    plan->parts = c2 <= kSplitMaxBig ? kMaxParts : 1;
  }
}

// Big vector owning chunk t (largest b with chunk_base <= t).
__device__ __forceinline__ int big_of_chunk(const BigInfo* big, int c2, int64_t t) {
  int lo = 0, hi = c2 - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (big[mid].chunk_base <= t)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

constexpr int kBigBlock = 256;
// Work items of the probe pass: kProbeSplit per chunk, kProbeUnroll entries
// per lane.
constexpr int kProbeUnroll = 16;
constexpr int kProbeItem = kBigBlock * kProbeUnroll;
constexpr int kProbeSplit = static_cast<int>(kBigChunk / kProbeItem);
static_assert(kBigChunk % kProbeItem == 0, "probe items tile a chunk");
// Workgroups per CU of a probe launch: four (one round of resident
// workgroups) for a call of few vectors, whose items a contiguous share per
// workgroup splits evenly (one 10^7-entry vector: 39.7 to 34.1 us); eight
// otherwise, where the second round evens out items of unequal cost (10^5
// uneven vectors: 0.77 ms, against 0.86 ms with four).
constexpr int kProbeWgPerCu = 8;
constexpr int kProbeWgPerCuFew = 4;
constexpr int64_t kProbeFewVectors = 64;
constexpr int kProbeWaves = 4;    // waves per SIMD the probe is compiled for

// Single-precision rejection of a first arrival.  The probe keeps an entry
// when O_1 <= bound v, O_1 = RN(E_1 RN(1/k)) and E_1 = -ln u.  With
// Y = k bound v log2(e): if u < 2^-Y - 2^-21, then -ln u exceeds k bound v by
// at least 2^-21 (u <= 1), which the few ulp of the double-precision steps
// cannot undo while k bound v < 2^28, so the exact test rejects the entry
// too.  The test below implies that bound on u:
//  * y = RN32(kbl v) with kbl >= k bound log2(e) (1 + 2^-18) gives y >= Y;
//  * v_exp_f32 is accurate to 1 ulp, so exp2(-y) <= 2^-Y (1 + 2^-23), and
//    q = exp2(-y) - 2^-20 < 2^-Y - 2^-21;
//  * u <= (m + 1) 2^-24 with m the top 24 bits of the draw (u is
//    ((x >> 11) + 1/2) 2^-53, rounded to nearest).
// Where y is large (k bound v >= 2^28 included) exp2 underflows, q < 0 and
// nothing is rejected; entries within 2^-20 of the boundary take the exact
// path.
__device__ __forceinline__ float rejection_scale(int k, double bound) {
  const double want = static_cast<double>(k) * bound * 1.4426950408889634 * (1.0 + 0x1p-18);
  float f = static_cast<float>(want);
  if (static_cast<double>(f) < want) f = __uint_as_float(__float_as_uint(f) + 1u);  // round up
  return f;
}

__device__ __forceinline__ bool surely_late(uint64_t x, float kbl, float v) {
  const float y = kbl * v;
  const float q = __builtin_amdgcn_exp2f(-y) - 0x1p-20f;
  const float uhi = static_cast<float>(static_cast<uint32_t>(x >> 40) + 1u) * 0x1p-24f;
  return uhi < q;
}

// Grid-wide pass 1 over big vectors: validate weights, sum them.  (Only the
// weights are read here; the probe pass, which reads the indices anyway,
// validates those.)
__global__ __launch_bounds__(kBigBlock) void big_sum_kernel(FastArgs fa) {
  __shared__ double ws[kBigBlock / kWave];
  __shared__ int sbad;
  const SketchArgs& p = fa.s;
  int c2 = 0;
  for (int cc = kBigFirst; cc < kNumClasses; ++cc) c2 += fa.plan->count[cc];
  const int32_t* list2 = fa.list + fa.plan->offset[kBigFirst];
  const int64_t total = fa.plan->big_chunks;
  const int tid = threadIdx.x;
  // a contiguous run of chunks per workgroup: the owning vector is looked
  // up when the run enters it, not for every chunk
  const int64_t t0 = total * blockIdx.x / gridDim.x;
  const int64_t t1 = total * (blockIdx.x + 1) / gridDim.x;
  int b = -1;
  int64_t next_vec_chunk = -1;
  VecDesc d{};
  for (int64_t t = t0; t < t1; ++t) {
    if (t >= next_vec_chunk) {
      b = big_of_chunk(fa.big, c2, t);
      d = vec_desc(p, list2[b]);
      next_vec_chunk = b + 1 < c2 ? fa.big[b + 1].chunk_base : total;
    }
    if (d.bad) continue;
    const int64_t e0 = d.a + (t - fa.big[b].chunk_base) * kBigChunk;
    const int64_t e1 = e0 + kBigChunk < d.b ? e0 + kBigChunk : d.b;
    if (tid == 0) sbad = 0;
    double part = 0.0;
    bool badl = false;
    // a chunk's weights in one round: every lane's loads in flight together
    constexpr int kU = static_cast<int>(kBigChunk / kBigBlock);
    float wv[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t e = e0 + u * kBigBlock + tid;
      wv[u] = e < e1 ? p.w[e] : 0.0f;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (!weight_valid(wv[u]))
        badl = true;
      else
        part += static_cast<double>(wv[u]);
    }
    __syncthreads();
    if (badl) sbad = 1;
    part = wave_sum_f64(part);
    if (tid % kWave == 0) ws[tid / kWave] = part;
    __syncthreads();
    if (tid == 0) {
      double tot = 0.0;
      for (int q = 0; q < kBigBlock / kWave; ++q) tot += ws[q];
      atomicAdd(&fa.big[b].Sslot[t % kSumSlots], tot);
      if (sbad) atomicOr(&fa.big[b].bad, 1);
    }
    __syncthreads();
  }
}

// Grid-wide pass 2 over big vectors: first arrival of every entry; entries
// within T0 go to the vector's candidate list.
//
// The pass is bound by its arithmetic (two splitmix64 rounds per entry,
// twelve quarter-rate 32-bit multiplies), not by HBM.  Its work items are
// parts of chunks, kProbeItem entries, kProbeUnroll per lane with every
// load issued at once; a workgroup takes a contiguous run of items.  Each
// item's candidates join one of the vector's kCandLists sublists.
__global__ __launch_bounds__(kBigBlock) __attribute__((amdgpu_waves_per_eu(kProbeWaves)))
void big_probe_kernel(FastArgs fa) {
  __shared__ int32_t mlist[kProbeItem];  // entries the first round kept
  __shared__ int32_t slist[kProbeItem];  // candidates
  __shared__ int smaybe, scount, sbase, sover;
  __shared__ unsigned long long smax[kBigBlock / kWave];
  __shared__ int sempty;
  const SketchArgs& p = fa.s;
  int c2 = 0;
  for (int cc = kBigFirst; cc < kNumClasses; ++cc) c2 += fa.plan->count[cc];
  const int32_t* list2 = fa.list + fa.plan->offset[kBigFirst];
  const int64_t nchunks = fa.plan->big_chunks;
  const int64_t total = nchunks * kProbeSplit;
  const int tid = threadIdx.x;
  const int lane = tid % kWave;
  // Each workgroup takes a contiguous run of items, so that consecutive
  // items mostly share a vector and its state below is looked up once.
  const int64_t u0 = total * blockIdx.x / gridDim.x;
  const int64_t u1 = total * (blockIdx.x + 1) / gridDim.x;
  int b = -1;
  int64_t next_vec_item = -1;  // first item of the vector after b
  VecDesc d{};
  BigInfo* bi = nullptr;
  int mode = 0;  // 0 nothing to do, 1 indices only, 2 candidates
  double S = 0.0, c1 = 0.0, bound = 0.0;
  float kbl = 0.0f;
  for (int64_t u = u0; u < u1; ++u) {
    const int64_t t = u / kProbeSplit;
    if (u >= next_vec_item) {
      b = big_of_chunk(fa.big, c2, t);
      bi = &fa.big[b];
      d = vec_desc(p, list2[b]);
      next_vec_item = (b + 1 < c2 ? fa.big[b + 1].chunk_base : nchunks) * kProbeSplit;
      S = 0.0;
      for (int q = 0; q < kSumSlots; ++q) S += bi->Sslot[q];
      if (d.bad || bi->bad) {
        mode = 0;  // poisoned already
      } else if (!(S > 0.0) || bi->cand_cap <= 0) {
        // no candidate list (no positive weight, a list not worth keeping,
        // or no room in the pool): only the indices are checked here
        mode = 1;
      } else {
        mode = 2;
        double T0 = max_exp_quantile(d.k) * fa.t0_scale / S;
        if (fa.update) {
          // an update's walk stops at the stored sketch's largest register
          if (tid == 0) sempty = 0;
          __syncthreads();
          unsigned long long m = 0;
          bool empty = false;
          for (int j = tid; j < d.k; j += kBigBlock) {
            if (p.out_idx[d.o + j] < 0)
              empty = true;
            else
              m = dbits(p.out_val[d.o + j]) > m ? dbits(p.out_val[d.o + j]) : m;
          }
          m = wave_max_u64(m);
          if (lane == 0) smax[tid / kWave] = m;
          if (empty) sempty = 1;
          __syncthreads();
          unsigned long long ms = 0;
          for (int qq = 0; qq < kBigBlock / kWave; ++qq) ms = smax[qq] > ms ? smax[qq] : ms;
          if (!sempty) T0 = fmin(T0, bitsd(ms));
          __syncthreads();
        }
        c1 = 1.0 / static_cast<double>(d.k);
        // The walk keeps an element when RN(O_1 RN(1/v)) <= T (T <= T0),
        // which implies O_1 <= T0 v (1 + 2^-51.9); the test below, with two
        // roundings of its own, admits at least that and needs no division.
        bound = T0 * (1.0 + 0x1p-50);
        kbl = rejection_scale(d.k, bound);
      }
    }
    // (every workgroup of the vector computes the same S; later launches read it)
    if (tid == 0 && u == bi->chunk_base * kProbeSplit) bi->S = S;
    const int qpart = static_cast<int>(u - t * kProbeSplit);
    const int64_t e0 = d.a + (t - bi->chunk_base) * kBigChunk + static_cast<int64_t>(qpart) * kProbeItem;
    if (mode == 0 || e0 >= d.b) continue;  // (past the end of the vector's last chunk)
    const int64_t e1 = e0 + kProbeItem < d.b ? e0 + kProbeItem : d.b;
    if (mode == 1) {
      bool badi = false;
      for (int64_t e = e0 + tid; e < e1; e += kBigBlock) badi |= p.idx[e] < 0;
      if (__ballot(badi) != 0 && lane == 0) atomicOr(&bi->bad_index, 1);
      continue;
    }
    // Two rounds per item.  First every entry's first arrival is drawn and
    // the single-precision test rejects all but a few (about 0.2 % at
    // k = 1024); the rest are listed in LDS.  Then the workgroup's lanes take
    // the listed entries densely and apply the exact test in double
    // precision; the candidates go to a second LDS list, which one of the
    // vector's sublists takes with one atomic.  Keeping the logarithm out of
    // the unrolled round keeps the kernel small enough for many resident
    // waves.
    if (tid == 0) {
      smaybe = 0;
      scount = 0;
    }
    __syncthreads();
    bool badl = false;
    constexpr int kPU = kProbeUnroll;
    float wv[kPU];
    int32_t iv[kPU];
#pragma unroll
    for (int q = 0; q < kPU; ++q) {
      const int64_t e = e0 + q * kBigBlock + tid;
      wv[q] = e < e1 ? p.w[e] : 0.0f;
      iv[q] = e < e1 ? p.idx[e] : 0;
    }
#pragma unroll
    for (int q = 0; q < kPU; ++q) {
      const int64_t e = e0 + q * kBigBlock + tid;
      bool maybe = false;
      if (iv[q] < 0) badl = true;
      if (wv[q] > 0.0f) {
        const uint64_t P = mix(p.seed_mix ^ static_cast<uint64_t>(static_cast<uint32_t>(iv[q])));
        maybe = !surely_late(draw(P, kTagArrival, 1u), kbl, wv[q]);
      }
      const uint64_t m = __ballot(maybe);
      if (m) {
        const int leader = __ffsll(static_cast<long long>(m)) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(&smaybe, __popcll(m));
        base = readlane_i32(base, leader);
        // (at most kProbeItem entries per item: the lists always have room)
        if (maybe) mlist[base + __popcll(m & lanemask_lt())] = static_cast<int32_t>(e - d.a);
      }
    }
    __syncthreads();
    const int nm = smaybe;
    for (int r = 0; r < nm; r += kBigBlock) {
      bool cand = false;
      int32_t rel = 0;
      if (r + tid < nm) {
        rel = mlist[r + tid];
        const float w = p.w[d.a + rel];
        const uint64_t P = mix(p.seed_mix ^ static_cast<uint64_t>(static_cast<uint32_t>(p.idx[d.a + rel])));
        const double O1 = fma(exp1(draw(P, kTagArrival, 1u)), c1, 0.0);
        cand = O1 <= bound * static_cast<double>(w);
      }
      const uint64_t m = __ballot(cand);
      if (m) {
        const int leader = __ffsll(static_cast<long long>(m)) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(&scount, __popcll(m));
        base = readlane_i32(base, leader);
        if (cand) slist[base + __popcll(m & lanemask_lt())] = rel;
      }
    }
    // a negative index poisons the vector (the walk reads the flag; this
    // pass never does, so its workgroups take the same branches)
    if (__ballot(badl) != 0 && lane == 0) atomicOr(&bi->bad_index, 1);
    __syncthreads();
    const int nc = scount;
    if (nc > 0) {
      // the item's sublist takes what it has room for, the list the rest
      const int scap = bi->sub_cap;
      const int ql = static_cast<int>((u - bi->chunk_base * kProbeSplit) % kCandLists);
      int32_t* subl = fa.pool + bi->sub_off + static_cast<int64_t>(ql) * scap;
      if (tid == 0) {
        const int b0 = atomicAdd(fa.pool + bi->sub_off - kCandHeader + ql * kCntStride, nc);
        const int fit = b0 >= scap ? 0 : (scap - b0 < nc ? scap - b0 : nc);
        sbase = b0;
        sover = fit < nc ? atomicAdd(&bi->over_count, nc - fit) - fit : 0;
      }
      __syncthreads();
      const int b0 = sbase;
      for (int q = tid; q < nc; q += kBigBlock) {
        if (b0 + q < scap) {
          subl[b0 + q] = slist[q];
        } else {
          const int slot = sover + q;  // (over_count + q - fit)
          if (slot < bi->cand_cap) fa.pool[bi->cand_off + slot] = slist[q];
        }
      }
    }
    __syncthreads();
  }
}

// Gather pass: each big vector's sublists packed after the entries that
// overflowed into its list; cand_count set to the total, or past cand_cap
// if the list cannot hold them all (the walk then takes every entry).
// Work items are (vector, sublist) pairs.
__global__ __launch_bounds__(kBigBlock) void big_gather_kernel(FastArgs fa) {
  int c2 = 0;
  for (int cc = kBigFirst; cc < kNumClasses; ++cc) c2 += fa.plan->count[cc];
  const int64_t total = static_cast<int64_t>(c2) * kCandLists;
  const int tid = threadIdx.x;
  for (int64_t u = blockIdx.x; u < total; u += gridDim.x) {
    const int b = static_cast<int>(u / kCandLists);
    const int q = static_cast<int>(u - static_cast<int64_t>(b) * kCandLists);
    BigInfo* bi = &fa.big[b];
    if (bi->cand_cap <= 0) continue;
    const int scap = bi->sub_cap;
    const int32_t* cnt = fa.pool + bi->sub_off - kCandHeader;
    int64_t at = bi->over_count, all = at;
    for (int r = 0; r < kCandLists; ++r) {
      const int m = cnt[r * kCntStride] < scap ? cnt[r * kCntStride] : scap;
      if (r < q) at += m;
      all += m;
    }
    const bool fits = all <= bi->cand_cap;
    if (q == 0 && tid == 0) bi->cand_count = fits ? static_cast<int>(all) : bi->cand_cap + 1;
    if (!fits) continue;
    const int mq = cnt[q * kCntStride] < scap ? cnt[q * kCntStride] : scap;
    const int32_t* src = fa.pool + bi->sub_off + static_cast<int64_t>(q) * scap;
    int32_t* dst = fa.pool + bi->cand_off + at;
    for (int i = tid; i < mq; i += kBigBlock) dst[i] = src[i];
  }
}

// Waves per workgroup of a class (four, eight for k > 2048 and for big
// vectors; halved while the LDS does not fit in 160 KB), and its one-wave
// size limit: vectors of at most `one_wave` entries are sketched one per
// wave where the register arrays are small enough for a set per wave
// (k <= 256).  The limit is a power of two minus one, so that it falls
// between the planner's log2 size bins; 8191 by default (document batch at
// k = 256: 0 -> 0.648 ms, 511 -> 0.599, 2047 -> 0.535, 8191 -> 0.527,
// 32767 -> 0.528).
void class_shape(int sc, int k_max, int small_waves, int one_wave, int* waves, int64_t* wave_lim) {
  int want = sc == 0 ? (k_max > 2048 ? 8 : 4) : 8;
  if (sc == 0 && small_waves > 0) want = small_waves;
  const int64_t lim = (sc == 0 && k_max <= 256) ? one_wave : 0;
  int w = want;
  while (w > 1 && fastgm_lds_bytes(k_max, w, lim > 0 ? w : 1) + w * sizeof(FgShared) > 160 * 1024)
    w /= 2;
  *waves = w;
  *wave_lim = lim;
}

// ---------------------------------------------------------------------------
// Optional per-kernel timing: HIP events recorded around each FastGM launch on
// its own stream, summed per kernel instance by gm_get_timing.
struct TimedLaunch {
  int id;
  hipEvent_t a, b;
};

// Shared by every host thread that launches: one mutex guards the lists.
struct TimingState {
  std::atomic<int> level{0};  // 0 off, 1 every launch, 2 the sketch kernels only
  std::mutex mu;
  std::vector<TimedLaunch> pending;
  std::vector<hipEvent_t> free_events;
  std::vector<std::string> names;
  std::vector<double> total_ms;
  std::vector<long long> launches;
};

TimingState& timing() {
  static TimingState t;
  return t;
}

void timing_enable(int level) { timing().level = level; }

static int timing_id(const std::string& name) {
  TimingState& t = timing();
  for (size_t i = 0; i < t.names.size(); ++i)
    if (t.names[i] == name) return static_cast<int>(i);
  t.names.push_back(name);
  t.total_ms.push_back(0.0);
  t.launches.push_back(0);
  return static_cast<int>(t.names.size()) - 1;
}

static hipEvent_t timing_event() {
  TimingState& t = timing();
  if (!t.free_events.empty()) {
    hipEvent_t e = t.free_events.back();
    t.free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Bracket one launch (returns -1 when timing is off).  `main`: a sketch
// kernel (FastGM class or plain), timed at both levels; the planning and
// big-vector passes only at level 1.
static int timing_begin(const char* name, bool main, hipStream_t stream, hipEvent_t* a) {
  const int level = timing().level;
  if (level == 0 || (level == 2 && !main)) return -1;
  std::lock_guard<std::mutex> lock(timing().mu);
  *a = timing_event();
  (void)hipEventRecord(*a, stream);
  return timing_id(name);
}

static void timing_end(int id, hipEvent_t a, hipStream_t stream) {
  if (id < 0) return;
  std::lock_guard<std::mutex> lock(timing().mu);
  hipEvent_t b = timing_event();
  (void)hipEventRecord(b, stream);
  timing().pending.push_back(TimedLaunch{id, a, b});
}

// Sum the finished launches; copy up to n (name, total ms, launches).
int timing_collect(int n, char (*names)[64], double* ms, long long* launches) {
  TimingState& t = timing();
  std::lock_guard<std::mutex> lock(t.mu);
  for (TimedLaunch& l : t.pending) {
    (void)hipEventSynchronize(l.b);
    float m = 0.0f;
    if (hipEventElapsedTime(&m, l.a, l.b) == hipSuccess) {
      t.total_ms[l.id] += m;
      t.launches[l.id] += 1;
    }
    t.free_events.push_back(l.a);
    t.free_events.push_back(l.b);
  }
  t.pending.clear();
  const int m = static_cast<int>(t.names.size()) < n ? static_cast<int>(t.names.size()) : n;
  for (int i = 0; i < m; ++i) {
    std::snprintf(names[i], 64, "%s", t.names[i].c_str());
    ms[i] = t.total_ms[i];
    launches[i] = t.launches[i];
  }
  return m;
}

void timing_reset() {
  TimingState& t = timing();
  (void)timing_collect(0, nullptr, nullptr, nullptr);
  std::lock_guard<std::mutex> lock(t.mu);
  t.names.clear();
  t.total_ms.clear();
  t.launches.clear();
}

int timing_begin_plain(hipStream_t stream, hipEvent_t* a) {
  return timing_begin("plain_kernel", true, stream, a);
}
void timing_end_plain(int id, hipEvent_t a, hipStream_t stream) { timing_end(id, a, stream); }

struct OccKey {
  const void* fn;
  size_t lds;
  int per_cu;
};

template <int W, int G>
static hipError_t launch_class(const FastArgs& fa, int cus, hipStream_t stream) {
  const size_t lds = fastgm_lds_bytes(fa.lds_k, W, fa.wave_lim > 0 ? W : 1);
  const bool big = fa.cls >= kBigFirst;
  const void* fn = big ? reinterpret_cast<const void*>(fastgm_big_kernel<W, G>)
                       : reinterpret_cast<const void*>(fastgm_class_kernel<W, G>);
  // occupancy per (kernel, LDS size), computed once (guarded: several host
  // threads may launch)
  static OccKey cache[64];
  static int ncache = 0;
  static std::mutex cache_mu;
  int per_cu = 0;
  {
    std::lock_guard<std::mutex> lock(cache_mu);
    for (int i = 0; i < ncache; ++i)
      if (cache[i].fn == fn && cache[i].lds == lds) per_cu = cache[i].per_cu;
    if (per_cu == 0) {
      hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         static_cast<int>(lds));
      if (e != hipSuccess) return e;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, W * kWave, lds);
      if (e != hipSuccess) return e;
      if (per_cu < 1) per_cu = 1;
      if (ncache < 64) cache[ncache++] = OccKey{fn, lds, per_cu};
    }
  }
  int64_t grid = static_cast<int64_t>(cus) * per_cu;
  // tasks: one per vector, or up to kMaxParts per big vector
  const int64_t tasks = fa.cls >= kBigFirst ? fa.s.nvec * kMaxParts : fa.s.nvec;
  if (grid > tasks) grid = tasks;
  if (grid * W > fa.heavy_waves) grid = fa.heavy_waves / W;  // room in the heavy buffer
  if (grid < 1) return hipErrorInvalidValue;
  hipEvent_t ta = nullptr;
  // named as rocprofv3 names the kernel, plus the class it drains
  char name[64];
  std::snprintf(name, sizeof(name), "%s<%d, %d> [class %d]",
                big ? "fastgm_big_kernel" : "fastgm_class_kernel", W, G, fa.cls);
  const int tid = timing_begin(name, true, stream, &ta);
  if (big)
    hipLaunchKernelGGL((fastgm_big_kernel<W, G>), dim3(static_cast<unsigned>(grid)), dim3(W * kWave),
                       lds, stream, fa);
  else
    hipLaunchKernelGGL((fastgm_class_kernel<W, G>), dim3(static_cast<unsigned>(grid)),
                       dim3(W * kWave), lds, stream, fa);
  timing_end(tid, ta, stream);
  return hipGetLastError();
}

template <int G>
static hipError_t launch_class_w(const FastArgs& fa, int waves, int cus, hipStream_t stream) {
  switch (waves) {
    case 1: return launch_class<1, G>(fa, cus, stream);
    case 2: return launch_class<2, G>(fa, cus, stream);
    case 4: return launch_class<4, G>(fa, cus, stream);
    default: return launch_class<8, G>(fa, cus, stream);
  }
}

// Vectors above kLimM entries are "big": validated, summed and probed by
// grid-wide passes first, then walked over their candidate lists.
constexpr int64_t kLimM = 32768;

hipError_t launch_fastgm(const SketchArgs& s, int pos_bits, double t0_scale, int map_load,
                         int republish, double seg_rest, int small_waves, int one_wave, int32_t* list,
                         void* plan, void* big, int32_t* pool, int64_t pool_cap,
                         void* heavy, int64_t heavy_waves, void* part, int update, int cus,
                         unsigned long long* stats, hipStream_t stream) {
  FastArgs fa;
  fa.update = update;
  fa.part_idx = static_cast<int32_t*>(part);
  fa.part_val = reinterpret_cast<double*>(static_cast<char*>(part) + kPartRegs * sizeof(int32_t));
  fa.heavy = static_cast<HeavyRec*>(heavy);
  fa.heavy_waves = heavy_waves;
  fa.big = static_cast<BigInfo*>(big);
  fa.pool = pool;
  fa.pool_cap = pool_cap;
  fa.stats = stats;
  fa.seg_rest = seg_rest;
  fa.s = s;
  fa.pos_bits = pos_bits;
  fa.t0_scale = t0_scale;
  fa.map_load = map_load;
  fa.republish = republish;
  fa.list = list;
  fa.plan = static_cast<PlanState*>(plan);
  hipEvent_t ta = nullptr;
  int tid = timing_begin("plan_kernel", false, stream, &ta);
  hipLaunchKernelGGL(plan_kernel, dim3(1), dim3(kPlanBlock), 0, stream, s, list, fa.plan, fa.big,
                     pool, pool_cap, t0_scale, kLimM);
  timing_end(tid, ta, stream);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  tid = timing_begin("big_sum_kernel", false, stream, &ta);
  hipLaunchKernelGGL(big_sum_kernel, dim3(cus * 8), dim3(kBigBlock), 0, stream, fa);
  timing_end(tid, ta, stream);
  tid = timing_begin("big_probe_kernel", false, stream, &ta);
  const int probe_wg = s.nvec <= kProbeFewVectors ? kProbeWgPerCuFew : kProbeWgPerCu;
  hipLaunchKernelGGL(big_probe_kernel, dim3(cus * probe_wg), dim3(kBigBlock), 0, stream, fa);
  timing_end(tid, ta, stream);
  tid = timing_begin("big_gather_kernel", false, stream, &ta);
  hipLaunchKernelGGL(big_gather_kernel, dim3(cus * 8), dim3(kBigBlock), 0, stream, fa);
  timing_end(tid, ta, stream);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // One persistent kernel per (size class, k class) that the call's k can
  // reach; an empty class exits at once.
  for (int sc = 0; sc < kSizeClasses; ++sc) {
    for (int kc = 0; kc < kKClasses; ++kc) {
      const int lo = kc == 0 ? 1 : kclass_hi(kc - 1) + 1;
      if (lo > s.k_max) break;
      // one k for every vector: the other k ranges are empty
      if (!s.kvec && kclass_hi(kc) < s.k_uniform) continue;
      fa.cls = sc * kKClasses + kc;
      fa.lds_k = s.k_max < kclass_hi(kc) ? s.k_max : kclass_hi(kc);
      int waves = 1;
      class_shape(sc, fa.lds_k, small_waves, one_wave, &waves, &fa.wave_lim);
      const int g = segment_lanes(fa.lds_k);
      e = g == 8 ? launch_class_w<8>(fa, waves, cus, stream)
                 : (g == 16 ? launch_class_w<16>(fa, waves, cus, stream)
                            : launch_class_w<64>(fa, waves, cus, stream));
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

size_t plan_state_bytes() { return sizeof(PlanState); }
int64_t heavy_list_bytes() { return kHeavyCapG * static_cast<int64_t>(sizeof(HeavyRec)); }
size_t big_info_bytes() { return sizeof(BigInfo); }
size_t part_scratch_bytes() {
  return static_cast<size_t>(kPartRegs) * (sizeof(int32_t) + sizeof(double));
}

}  // namespace gm
