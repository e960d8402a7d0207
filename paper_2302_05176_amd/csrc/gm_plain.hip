// gm_plain.hip -- plain O(k n+) form of the Gumbel-Max sketch.
//
// Eq. (1)/(2): s_j = argmin_i E_ij / v_i and y_j = min_i E_ij / v_i over the
// positive entries of the vector, with E_ij drawn independently for every
// (element, register) pair (Sec. 1, the straightforward method with the
// variables generated on the fly).  This is the O(k n+) baseline the FastGM
// form is measured against.
//
// Mapping: one workgroup handles one (vector, tile of kPlainBlock registers);
// every lane owns one register, so registers need no atomics.  The vector's
// entries are staged through LDS kPlainBlock at a time; each lane computes the
// per-element hash prefix and 1/v_i of one staged entry, then every lane walks
// the staged entries and draws its own register's key.  The hot loop is pure
// VALU (two 64-bit multiplies of the hash, the fixed-order -ln, one multiply
// and a compare per key).
#include "gm_common.h"

namespace gm {

constexpr int kPlainBlock = 256;

__global__ __launch_bounds__(kPlainBlock) void plain_kernel(SketchArgs p) {
  __shared__ uint64_t s_prefix[kPlainBlock];
  __shared__ double s_r[kPlainBlock];
  __shared__ int32_t s_idx[kPlainBlock];
  __shared__ int s_bad;

  const int tid = threadIdx.x;
  const int32_t j = blockIdx.y * kPlainBlock + tid;

  for (int64_t v = blockIdx.x; v < p.nvec; v += gridDim.x) {
    const VecDesc d = vec_desc(p, v);
    const int32_t span = out_span(p, v, d);
    // Tiles past this vector's registers have nothing to do (block-uniform);
    // tile 0 always runs so a bad vector is counted once.
    if (blockIdx.y > 0 && static_cast<int64_t>(blockIdx.y) * kPlainBlock >= span) continue;

    if (tid == 0) s_bad = d.bad ? 1 : 0;
    double best = __longlong_as_double(static_cast<long long>(kInfBits));
    int32_t best_i = 0x7FFFFFFF;
    __syncthreads();
    if (!s_bad) {
      for (int64_t base = d.a; base < d.b; base += kPlainBlock) {
        const int n = static_cast<int>(d.b - base < kPlainBlock ? d.b - base : kPlainBlock);
        if (tid < n) {
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
          for (int e = 0; e < n; ++e) {
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
    const bool bad = s_bad != 0;
    if (j < span) {
      int32_t oi;
      double ov;
      if (bad) {
        oi = kIdxPoison;
        ov = __longlong_as_double(static_cast<long long>(kNanBits));
      } else if (best_i == 0x7FFFFFFF) {
        oi = kIdxEmpty;
        ov = __longlong_as_double(static_cast<long long>(kInfBits));
      } else {
        oi = best_i;
        ov = best;
      }
      p.out_idx[d.o + j] = oi;
      p.out_val[d.o + j] = ov;
    }
    if (bad && blockIdx.y == 0 && tid == 0) atomicAdd(p.err, 1ull);
    __syncthreads();
  }
}

int timing_begin_plain(hipStream_t stream, hipEvent_t* a);
void timing_end_plain(int id, hipEvent_t a, hipStream_t stream);

hipError_t launch_plain(const SketchArgs& p, hipStream_t stream) {
  const int tiles = (p.k_max + kPlainBlock - 1) / kPlainBlock;
  const int64_t gx = p.nvec < (1 << 22) ? p.nvec : (1 << 22);
  dim3 grid(static_cast<unsigned>(gx), static_cast<unsigned>(tiles));
  hipEvent_t ta = nullptr;
  const int tid = timing_begin_plain(stream, &ta);
  hipLaunchKernelGGL(plain_kernel, grid, dim3(kPlainBlock), 0, stream, p);
  timing_end_plain(tid, ta, stream);
  return hipGetLastError();
}

}  // namespace gm
