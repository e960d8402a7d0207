// gm_plain.hip -- plain O(k n+) form of the Gumbel-Max sketch.
//
// Eq. (1)/(2): s_j = argmin_i E_ij / v_i and y_j = min_i E_ij / v_i over the
// positive entries of the vector, with E_ij drawn independently for every
// (element, register) pair (Sec. 1, the straightforward method with the
// variables generated on the fly).  This is the O(k n+) baseline the FastGM
// form is measured against.
//
// Mapping: one workgroup handles one (vector, part of its entries, tile of
// kPlainBlock registers); every lane owns one register, so registers need
// no atomics.  The part's entries are staged through LDS kPlainBlock at a
// time; each lane computes the per-element hash prefix and 1/v_i of one
// staged entry, then every lane walks the staged entries and draws its own
// register's key.  The hot loop is pure VALU (two 64-bit multiplies of the
// hash, the fixed-order -ln, one multiply and a compare per key).
//
// A batch with few (vector, tile) pairs would leave most CUs idle (one
// vector of 10^7 entries at k = 1024 is four workgroups), so such a batch
// splits each vector's entries into up to `parts` ranges of at least
// kPlainMinPart entries.  A batch of many vectors of uneven sizes would wait
// on its largest (in the document batch at k = 256, one 5x10^4-entry vector
// took 6.7 of 8.0 ms), so a planning pass splits the vectors far above the
// batch's mean share of work per workgroup (see plain_plan_kernel).  Each range writes its registers' partial minimum
// to a scratch row, and the last range of a (vector, tile) to finish takes
// the lexicographic minimum over the rows -- the merge of Sec. 2.3, which is
// exact because a minimum over a union is the minimum of the minima.
#include "gm_common.h"

namespace gm {

constexpr int kPlainBlock = 256;
constexpr int64_t kPlainMinPart = 1024;

// Scratch of a split launch (all device memory owned by the library's
// per-stream workspace; counters and flags start at zero and are left at
// zero by the workgroup that merges).
// Split plan of a batch of uneven vectors, written by plain_plan_kernel:
// the vectors split (ascending), their part counts and their first scratch
// row and counter.  The parts of the split vectors, the longest tasks, are
// tasks e in [0, extra) and start first; task kPlainMaxExtra + v is vector v
// whole, or nothing if it is split.
constexpr int kPlainMaxSplit = 1024;
constexpr int kPlainMaxParts = 32;
constexpr int kPlainMaxExtra = 8192;
constexpr int kPlainSplitAbove = 1;  // split vectors above this many times L
struct PlainPlan {
  int64_t min_split_n;  // vectors of at most this many entries are not split
  int32_t nsplit;
  int32_t extra;
  int32_t v[kPlainMaxSplit];
  int32_t np[kPlainMaxSplit];
  int32_t extra_base[kPlainMaxSplit];  // its first part's task
  int32_t cnt[kPlainMaxSplit];         // first counter (one per tile)
  int64_t row[kPlainMaxSplit];         // first row of k_max partial registers
};
static_assert(sizeof(PlainPlan) <= kPlainPlanBytes, "split plan must fit its scratch");

struct PlainSplit {
  int32_t parts;       // ranges per vector (1: no split)
  int32_t tiles;       // register tiles per vector
  double* part_val;    // [nvec * parts][k_max] partial minima
  int32_t* part_idx;
  int32_t* count;      // [nvec * tiles] ranges finished
  int32_t* bad;        // [nvec * tiles] an invalid entry was seen
  const PlainPlan* plan;  // uneven split (parts == 1): the planner's output
};

// Index of the last entry of a[0..n) that is <= x (a ascending, a[0] <= x).
__device__ __forceinline__ int last_le(const int32_t* a, int n, int32_t x) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (a[mid] <= x)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kPlainBlock) void plain_kernel(SketchArgs p, PlainSplit sp) {
  __shared__ uint64_t s_prefix[kPlainBlock];
  __shared__ double s_r[kPlainBlock];
  __shared__ int32_t s_idx[kPlainBlock];
  __shared__ int s_bad;
  __shared__ int s_last;

  const int tid = threadIdx.x;
  const int tile = blockIdx.y;
  const int32_t j = tile * kPlainBlock + tid;
  const PlainPlan* pl = sp.plan;
  const int64_t ntask = pl ? p.nvec + kPlainMaxExtra : p.nvec * sp.parts;

  for (int64_t t = blockIdx.x; t < ntask; t += gridDim.x) {
    int64_t v;
    int part, np = 1;
    int64_t prow = 0;  // first partial-register row of the vector
    int64_t pcnt = 0;  // first counter of the vector
    if (pl) {
      // uneven split: a part of a split vector, or an unsplit vector whole
      const int ns = pl->nsplit;
      if (t >= kPlainMaxExtra) {
        v = t - kPlainMaxExtra;
        part = 0;
        if (ns > 0 && p.off[v + 1] - p.off[v] > pl->min_split_n && pl->v[0] <= v &&
            pl->v[last_le(pl->v, ns, static_cast<int32_t>(v))] == v)
          continue;  // split: its parts are the first tasks
      } else {
        if (t >= pl->extra) continue;
        const int i = last_le(pl->extra_base, ns, static_cast<int32_t>(t));
        v = pl->v[i];
        part = static_cast<int>(t - pl->extra_base[i]);
        np = pl->np[i];
        prow = pl->row[i];
        pcnt = pl->cnt[i];
      }
    } else {
      v = t / sp.parts;
      part = static_cast<int>(t - v * sp.parts);
      prow = v * sp.parts;
      pcnt = v * sp.tiles;
    }
    const VecDesc d = vec_desc(p, v);
    const int32_t span = out_span(p, v, d);
    // Tiles past this vector's registers have nothing to do (block-uniform);
    // tile 0 always runs so a bad vector is counted once.
    if (tile > 0 && static_cast<int64_t>(tile) * kPlainBlock >= span) continue;
    const int64_t n = d.b > d.a ? d.b - d.a : 0;
    if (!pl && sp.parts > 1) {
      // this vector's ranges: as many as its size allows, at most sp.parts
      const int64_t want = (n + kPlainMinPart - 1) / kPlainMinPart;
      np = want < 1 ? 1 : (want > sp.parts ? sp.parts : static_cast<int>(want));
    }
    if (part >= np) continue;
    const int64_t ea = d.a + n * part / np;
    const int64_t eb = d.a + n * (part + 1) / np;

    if (tid == 0) s_bad = d.bad ? 1 : 0;
    double best = bitsd(kInfBits);
    int32_t best_i = 0x7FFFFFFF;
    __syncthreads();
    if (!s_bad) {
      for (int64_t base = ea; base < eb; base += kPlainBlock) {
        const int m = static_cast<int>(eb - base < kPlainBlock ? eb - base : kPlainBlock);
        if (tid < m) {
          const int32_t i = p.idx[base + tid];
          const float w = p.w[base + tid];
          int32_t keep = -1;
          if (i < 0 || !weight_valid(w)) {
            s_bad = 1;
          } else if (w > 0.0f) {
            s_prefix[tid] = mix(p.seed_mix ^ static_cast<uint64_t>(static_cast<uint32_t>(i)));
            s_r[tid] = 1.0 / static_cast<double>(w);
            keep = i;
          }
          s_idx[tid] = keep;
        }
        __syncthreads();
        if (s_bad) break;
        if (j < d.k) {
          for (int e = 0; e < m; ++e) {
            const int32_t i = s_idx[e];
            if (i < 0) continue;
            const double key =
                exp1(draw(s_prefix[e], kTagPlain, static_cast<uint32_t>(j))) * s_r[e];
            if (key < best || (key == best && i < best_i)) {
              best = key;
              best_i = i;
            }
          }
        }
        __syncthreads();
      }
    }
    __syncthreads();
    bool bad = s_bad != 0;
    if (np > 1) {
      // publish this range's minima; the last range of the tile merges
      const int64_t row = (prow + part) * static_cast<int64_t>(p.k_max);
      const int64_t ct = pcnt + tile;
      if (j < span) {
        sp.part_val[row + j] = best;
        sp.part_idx[row + j] = best_i;
      }
      __threadfence();
      __syncthreads();
      if (tid == 0) {
        if (bad) atomicOr(&sp.bad[ct], 1);
        __threadfence();
        s_last = atomicAdd(&sp.count[ct], 1) == np - 1 ? 1 : 0;
      }
      __syncthreads();
      if (!s_last) continue;
      __threadfence();
      bad = __hip_atomic_load(&sp.bad[ct], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
      if (!bad && j < span) {
        best = bitsd(kInfBits);
        best_i = 0x7FFFFFFF;
        for (int q = 0; q < np; ++q) {
          const int64_t r2 = (prow + q) * static_cast<int64_t>(p.k_max) + j;
          const double key = sp.part_val[r2];
          const int32_t i = sp.part_idx[r2];
          if (key < best || (key == best && i < best_i)) {
            best = key;
            best_i = i;
          }
        }
      }
      __syncthreads();
      // leave the tile's counter and flag at zero for the next call
      if (tid == 0) {
        sp.count[ct] = 0;
        sp.bad[ct] = 0;
      }
    }
    if (j < span) {
      int32_t oi;
      double ov;
      if (bad) {
        oi = kIdxPoison;
        ov = bitsd(kNanBits);
      } else if (best_i == 0x7FFFFFFF) {
        oi = kIdxEmpty;
        ov = bitsd(kInfBits);
      } else {
        oi = best_i;
        ov = best;
      }
      p.out_idx[d.o + j] = oi;
      p.out_val[d.o + j] = ov;
    }
    if (bad && tile == 0 && tid == 0) atomicAdd(p.err, 1ull);
    __syncthreads();
  }
}

// Planning pass of a batch of many vectors (one workgroup): L is half the
// batch's mean entries per workgroup (total entries x tiles / target
// workgroups / 2, at least kPlainMinPart); a vector of more than L entries
// is split into ceil(n / L) parts, at most kPlainMaxParts, in vector order
// while the scratch rows and counters and the plan's lists hold them.  The
// unsplit vectors then run after the parts, each at most L entries, so the
// launch ends within about one such task of its mean (document batch at
// k = 256: 8.0 ms unsplit, 7.6 with L the mean and twice L the cut, 6.1 ms).
__global__ __launch_bounds__(kPlainBlock) void plain_plan_kernel(SketchArgs p, PlainPlan* pl,
                                                                 int64_t rows_cap, int64_t cnt_cap,
                                                                 int tiles, int64_t target) {
  __shared__ int64_t red[kPlainBlock / kWave];
  __shared__ int64_t sc[4][kPlainBlock];
  __shared__ int64_t run[4];
  __shared__ int s_ns, s_extra;
  const int tid = threadIdx.x;
  int64_t tot = 0;
  for (int64_t v = tid; v < p.nvec; v += kPlainBlock) {
    const int64_t n = p.off[v + 1] - p.off[v];
    if (n > 0) tot += n;
  }
  tot = wave_sum_i64(tot);
  if (tid % kWave == 0) red[tid / kWave] = tot;
  if (tid < 4) run[tid] = 0;
  if (tid == 0) {
    s_ns = 0;
    s_extra = 0;
  }
  __syncthreads();
  tot = 0;
  for (int q = 0; q < kPlainBlock / kWave; ++q) tot += red[q];
  const int64_t want = (tot * tiles + 2 * target - 1) / (2 * target);
  const int64_t L = want > kPlainMinPart ? want : kPlainMinPart;
  for (int64_t b0 = 0; b0 < p.nvec; b0 += kPlainBlock) {
    const int64_t v = b0 + tid;
    int np = 1;
    if (v < p.nvec) {
      const VecDesc d = vec_desc(p, v);
      const int64_t n = d.b - d.a;
      if (!d.bad && n > kPlainSplitAbove * L) {
        const int64_t q = (n + L - 1) / L;
        np = q > kPlainMaxParts ? kPlainMaxParts : static_cast<int>(q);
      }
    }
    // demands of the split vectors: rows, counters, extra tasks, list entries
    const int64_t dem[4] = {np > 1 ? np : 0, np > 1 ? tiles : 0, np > 1 ? np : 0, np > 1 ? 1 : 0};
    for (int c = 0; c < 4; ++c) sc[c][tid] = dem[c];
    __syncthreads();
    for (int dd = 1; dd < kPlainBlock; dd <<= 1) {
      int64_t a[4];
      for (int c = 0; c < 4; ++c) a[c] = tid >= dd ? sc[c][tid - dd] : 0;
      __syncthreads();
      for (int c = 0; c < 4; ++c) sc[c][tid] += a[c];
      __syncthreads();
    }
    // inclusive prefixes over every candidate so far: past the first that
    // does not fit, none fits (the prefixes only grow)
    const int64_t e_rows = run[0] + sc[0][tid], e_cnt = run[1] + sc[1][tid];
    const int64_t e_extra = run[2] + sc[2][tid], e_ns = run[3] + sc[3][tid];
    if (np > 1 && e_rows <= rows_cap && e_cnt <= cnt_cap && e_extra <= kPlainMaxExtra &&
        e_ns <= kPlainMaxSplit) {
      const int i = static_cast<int>(e_ns) - 1;
      pl->v[i] = static_cast<int32_t>(v);
      pl->np[i] = np;
      pl->extra_base[i] = static_cast<int32_t>(e_extra) - np;
      pl->cnt[i] = static_cast<int32_t>(e_cnt) - tiles;
      pl->row[i] = e_rows - np;
      atomicMax(&s_ns, i + 1);
      atomicMax(&s_extra, static_cast<int>(e_extra));
    }
    __syncthreads();
    if (tid < 4) run[tid] += sc[tid][kPlainBlock - 1];
    __syncthreads();
  }
  if (tid == 0) {
    pl->min_split_n = kPlainSplitAbove * L;
    pl->nsplit = s_ns;
    pl->extra = s_extra;
  }
}

int timing_begin_plain(hipStream_t stream, hipEvent_t* a);
void timing_end_plain(int id, hipEvent_t a, hipStream_t stream);

// Workgroups a launch aims for before it splits vectors (eight per CU), and
// the scratch that bounds: a split launch has fewer than half that many
// (vector, tile) pairs, so parts * nvec * tiles < 1.5 x the target.
constexpr int kPlainWgPerCu = 8;

int64_t plain_scratch_regs(int cus) {
  return static_cast<int64_t>(cus) * kPlainWgPerCu * 3 / 2 * kPlainBlock + kPlainBlock;
}
int64_t plain_scratch_counters(int cus) { return static_cast<int64_t>(cus) * kPlainWgPerCu / 2 + 1; }

__global__ void zero_i32_kernel(int32_t* p, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0;
}

// Scratch of a split launch: `regs` partial registers (8-byte values, then
// 4-byte indices), then two arrays of `counters` int32.  With `clear`, the
// counters the launch uses are zeroed by a fill kernel first; otherwise they
// must be zero on entry (the kernel leaves them at zero).  A launch splits
// only as far as the scratch holds; without scratch it does not split.
// Batches of more vectors than this are not planned (the planning pass is
// one workgroup).
constexpr int64_t kPlainPlanMaxVectors = 65536;

hipError_t launch_plain(const SketchArgs& p, const PlainScratch& ps, int cus, hipStream_t stream) {
  const int tiles = (p.k_max + kPlainBlock - 1) / kPlainBlock;
  const int64_t target = static_cast<int64_t>(cus) * kPlainWgPerCu;
  PlainSplit sp{1, tiles, nullptr, nullptr, nullptr, nullptr, nullptr};
  const int64_t pairs = p.nvec * tiles;
  auto use_scratch = [&]() {
    sp.part_val = static_cast<double*>(ps.base);
    sp.part_idx = reinterpret_cast<int32_t*>(sp.part_val + ps.regs);
    sp.count = sp.part_idx + ps.regs;
    sp.bad = sp.count + ps.counters;
    if (ps.clear) {
      // (a fill kernel rather than a memset node: the call may be captured)
      const int64_t n = ps.counters * 2;
      hipLaunchKernelGGL(zero_i32_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0,
                         stream, sp.count, n);
    }
  };
  if (ps.base && 2 * pairs < target && pairs <= ps.counters) {
    int64_t parts = (target + pairs - 1) / pairs;
    while (parts > 1 && p.nvec * parts * p.k_max > ps.regs) --parts;
    if (parts > 1) {
      sp.parts = static_cast<int32_t>(parts);
      use_scratch();
    }
  } else if (ps.base && p.nvec >= 2 && p.nvec <= kPlainPlanMaxVectors) {
    use_scratch();
    PlainPlan* pl = reinterpret_cast<PlainPlan*>(sp.bad + ps.counters);
    hipLaunchKernelGGL(plain_plan_kernel, dim3(1), dim3(kPlainBlock), 0, stream, p, pl,
                       ps.regs / p.k_max, ps.counters, tiles, target);
    sp.plan = pl;
  }
  const int64_t ntask = sp.plan ? p.nvec + kPlainMaxExtra : p.nvec * sp.parts;
  const int64_t gx = ntask < (1 << 22) ? ntask : (1 << 22);
  dim3 grid(static_cast<unsigned>(gx), static_cast<unsigned>(tiles));
  hipEvent_t ta = nullptr;
  const int tid = timing_begin_plain(stream, &ta);
  hipLaunchKernelGGL(plain_kernel, grid, dim3(kPlainBlock), 0, stream, p, sp);
  timing_end_plain(tid, ta, stream);
  return hipGetLastError();
}

}  // namespace gm
