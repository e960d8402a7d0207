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
// kPlainMinPart entries.  Each range writes its registers' partial minimum
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
struct PlainSplit {
  int32_t parts;       // ranges per vector (1: no split)
  int32_t tiles;       // register tiles per vector
  double* part_val;    // [nvec * parts][k_max] partial minima
  int32_t* part_idx;
  int32_t* count;      // [nvec * tiles] ranges finished
  int32_t* bad;        // [nvec * tiles] an invalid entry was seen
};

__global__ __launch_bounds__(kPlainBlock) void plain_kernel(SketchArgs p, PlainSplit sp) {
  __shared__ uint64_t s_prefix[kPlainBlock];
  __shared__ double s_r[kPlainBlock];
  __shared__ int32_t s_idx[kPlainBlock];
  __shared__ int s_bad;
  __shared__ int s_last;

  const int tid = threadIdx.x;
  const int tile = blockIdx.y;
  const int32_t j = tile * kPlainBlock + tid;
  const int64_t ntask = p.nvec * sp.parts;

  for (int64_t t = blockIdx.x; t < ntask; t += gridDim.x) {
    const int64_t v = t / sp.parts;
    const int part = static_cast<int>(t - v * sp.parts);
    const VecDesc d = vec_desc(p, v);
    const int32_t span = out_span(p, v, d);
    // Tiles past this vector's registers have nothing to do (block-uniform);
    // tile 0 always runs so a bad vector is counted once.
    if (tile > 0 && static_cast<int64_t>(tile) * kPlainBlock >= span) continue;
    // this vector's ranges: as many as its size allows, at most sp.parts
    const int64_t n = d.b > d.a ? d.b - d.a : 0;
    int np = 1;
    if (sp.parts > 1) {
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
      const int64_t row = (v * sp.parts + part) * static_cast<int64_t>(p.k_max);
      const int64_t ct = v * sp.tiles + tile;
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
          const int64_t r2 = (v * sp.parts + q) * static_cast<int64_t>(p.k_max) + j;
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
hipError_t launch_plain(const SketchArgs& p, const PlainScratch& ps, int cus, hipStream_t stream) {
  const int tiles = (p.k_max + kPlainBlock - 1) / kPlainBlock;
  const int64_t target = static_cast<int64_t>(cus) * kPlainWgPerCu;
  PlainSplit sp{1, tiles, nullptr, nullptr, nullptr, nullptr};
  const int64_t pairs = p.nvec * tiles;
  if (ps.base && 2 * pairs < target && pairs <= ps.counters) {
    int64_t parts = (target + pairs - 1) / pairs;
    while (parts > 1 && p.nvec * parts * p.k_max > ps.regs) --parts;
    if (parts > 1) {
      sp.parts = static_cast<int32_t>(parts);
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
    }
  }
  const int64_t ntask = p.nvec * sp.parts;
  const int64_t gx = ntask < (1 << 22) ? ntask : (1 << 22);
  dim3 grid(static_cast<unsigned>(gx), static_cast<unsigned>(tiles));
  hipEvent_t ta = nullptr;
  const int tid = timing_begin_plain(stream, &ta);
  hipLaunchKernelGGL(plain_kernel, grid, dim3(kPlainBlock), 0, stream, p, sp);
  timing_end_plain(tid, ta, stream);
  return hipGetLastError();
}

}  // namespace gm
