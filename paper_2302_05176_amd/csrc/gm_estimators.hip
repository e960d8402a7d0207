// gm_estimators.hip -- estimators and merge on stored sketches.
//
//  * Probability-Jaccard estimate (Sec. 1; Theorem 1): fraction of registers
//    whose Gumbel-ArgMax values agree.  One wave per pair, lanes stride over
//    the registers (coalesced int32 loads), integer reduction.
//  * Weighted-cardinality estimate (Sec. 1; Theorem 2): (k-1) / sum_j y_j,
//    sum taken left to right.  One wave per sketch.
//  * Merge (Sec. 2.3): registerwise lexicographic (y, s) minimum over r
//    sketches.  One thread per register.
//  * Two-set algebra: union, intersection, relative complements and J_W of
//    two sets from their sketches (see setops_kernel).
#include "gm_common.h"

namespace gm {

__global__ __launch_bounds__(256) void jaccard_kernel(const int32_t* a, const int32_t* b,
                                                      int64_t npairs, int32_t k, double* out) {
  const int lane = threadIdx.x % kWave;
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x / kWave);
  for (int64_t pr = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + threadIdx.x / kWave;
       pr < npairs; pr += waves) {
    const int32_t* ra = a + pr * k;
    const int32_t* rb = b + pr * k;
    int m = 0;
    for (int j = lane; j < k; j += kWave) {
      const int32_t x = ra[j];
      m += (x == rb[j] && x >= 0) ? 1 : 0;
    }
    m = wave_sum_i32(m);
    if (lane == 0) out[pr] = static_cast<double>(m) / static_cast<double>(k);
  }
}

__global__ __launch_bounds__(256) void jaccard_pairs_kernel(const int32_t* store, int64_t nstore,
                                                            int32_t k, const int64_t* ia,
                                                            const int64_t* ib, int64_t npairs,
                                                            double* out,
                                                            unsigned long long* err) {
  const int lane = threadIdx.x % kWave;
  const int64_t waves = static_cast<int64_t>(gridDim.x) * (blockDim.x / kWave);
  for (int64_t pr = static_cast<int64_t>(blockIdx.x) * (blockDim.x / kWave) + threadIdx.x / kWave;
       pr < npairs; pr += waves) {
    const int64_t x = ia[pr], y = ib[pr];
    if (x < 0 || x >= nstore || y < 0 || y >= nstore) {
      if (lane == 0) {
        out[pr] = bitsd(kNanBits);
        atomicAdd(err, 1ull);
      }
      continue;
    }
    const int32_t* ra = store + x * k;
    const int32_t* rb = store + y * k;
    int m = 0;
    for (int j = lane; j < k; j += kWave) {
      const int32_t u = ra[j];
      m += (u == rb[j] && u >= 0) ? 1 : 0;
    }
    m = wave_sum_i32(m);
    if (lane == 0) out[pr] = static_cast<double>(m) / static_cast<double>(k);
  }
}

// One wave per sketch: the row is staged in LDS by coalesced loads, 1024
// registers at a time, and one lane adds them up left to right, reading two
// values per LDS access eight accesses ahead (a thread walking its row in
// device memory waited on one load per register: 0.19 ms for one row of
// 4096).
constexpr int kWcardChunk = 1024;

__global__ __launch_bounds__(kWave) void wcard_kernel(const double* val, int64_t nvec, int32_t k,
                                                      double* out) {
  __shared__ double sy[kWcardChunk];
  const int lane = threadIdx.x;
  for (int64_t v = blockIdx.x; v < nvec; v += gridDim.x) {
    const double* y = val + v * k;
    double s = 0.0;
    for (int32_t c0 = 0; c0 < k; c0 += kWcardChunk) {
      const int32_t m = k - c0 < kWcardChunk ? k - c0 : kWcardChunk;
      for (int32_t j = lane; j < m; j += kWave) sy[j] = y[c0 + j];
      __syncthreads();
      if (lane == 0) {
        int32_t j = 0;
        for (; j + 16 <= m; j += 16) {
          double2 a[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) a[q] = reinterpret_cast<const double2*>(sy + j)[q];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            s = s + a[q].x;
            s = s + a[q].y;
          }
        }
        for (; j < m; ++j) s = s + sy[j];
      }
      __syncthreads();
    }
    if (lane == 0) out[v] = static_cast<double>(k - 1) / s;
  }
}

__global__ __launch_bounds__(256) void merge_kernel(const int32_t* in_idx, const double* in_val,
                                                    int64_t r, int32_t k, int32_t* out_idx,
                                                    double* out_val) {
  const int32_t j = static_cast<int32_t>(static_cast<int64_t>(blockIdx.x) * blockDim.x +
                                         threadIdx.x);
  if (j >= k) return;
  double by = bitsd(kInfBits);
  int32_t bs = kIdxEmpty;
  bool poison = false;
  for (int64_t q = 0; q < r; ++q) {
    const double y = in_val[q * k + j];
    const int32_t s = in_idx[q * k + j];
    if (y != y || s == kIdxPoison) {
      poison = true;
      continue;
    }
    if (y < by || (y == by && s < bs && s >= 0)) {
      by = y;
      bs = s;
    }
  }
  out_idx[j] = poison ? kIdxPoison : bs;
  out_val[j] = poison ? bitsd(kNanBits) : by;
}

// Weighted cardinalities of two sets A and B from their sketches (union,
// intersection, A minus B, B minus A, J_W).  Register j of the union is the
// lexicographic minimum of the two registers (Sec. 2.3); its winner lies in
// both sets when the two registers are equal, in A only when A's is the
// smaller, in B only when B's is.  The union's weighted cardinality is the
// Sec. 1 estimator (k-1)/sum_j y_j of the merged values, summed left to
// right; each part is the union times its fraction of the k registers.
//
// One thread per pair, so that its sum keeps the left-to-right order.  The
// rows are read through LDS in tiles of kSetTile registers: the wave loads
// 64 pairs x kSetTile registers with consecutive lanes on consecutive
// addresses, then each lane runs through its own pair's tile.
constexpr int kSetPairs = 64;   // pairs per workgroup (one wave)
constexpr int kSetTile = 16;    // registers per tile

__global__ __launch_bounds__(kSetPairs) void setops_kernel(const int32_t* sa, const double* ya,
                                                           const int32_t* sb, const double* yb,
                                                           int64_t npairs, int32_t k, double* out) {
  __shared__ double t_ya[kSetPairs][kSetTile + 1];
  __shared__ double t_yb[kSetPairs][kSetTile + 1];
  __shared__ int32_t t_sa[kSetPairs][kSetTile + 1];
  __shared__ int32_t t_sb[kSetPairs][kSetTile + 1];
  const int lane = threadIdx.x;
  for (int64_t p0 = static_cast<int64_t>(blockIdx.x) * kSetPairs; p0 < npairs;
       p0 += static_cast<int64_t>(gridDim.x) * kSetPairs) {
    const int np = npairs - p0 < kSetPairs ? static_cast<int>(npairs - p0) : kSetPairs;
    double sum = 0.0;
    int64_t neq = 0, nlt = 0, ngt = 0;
    bool poison = false;
    for (int j0 = 0; j0 < k; j0 += kSetTile) {
      const int nj = k - j0 < kSetTile ? k - j0 : kSetTile;
      // stage: element e of the (np x nj) tile goes to lane e % 64
      for (int e = lane; e < np * nj; e += kSetPairs) {
        const int q = e / nj, jj = e - q * nj;
        const int64_t g = (p0 + q) * static_cast<int64_t>(k) + j0 + jj;
        t_ya[q][jj] = ya[g];
        t_yb[q][jj] = yb[g];
        t_sa[q][jj] = sa[g];
        t_sb[q][jj] = sb[g];
      }
      __syncthreads();
      if (lane < np) {
        for (int jj = 0; jj < nj; ++jj) {
          const double a = t_ya[lane][jj], b = t_yb[lane][jj];
          const int32_t ia = t_sa[lane][jj], ib = t_sb[lane][jj];
          if (ia == kIdxPoison || ib == kIdxPoison || a != a || b != b) {
            poison = true;
            continue;
          }
          double m;
          if (a < b || (a == b && ia < ib)) {
            m = a;
            nlt += ia >= 0 ? 1 : 0;
          } else if (b < a || (a == b && ib < ia)) {
            m = b;
            ngt += ib >= 0 ? 1 : 0;
          } else {
            m = a;
            neq += ia >= 0 ? 1 : 0;
          }
          sum = sum + m;
        }
      }
      __syncthreads();
    }
    if (lane < np) {
      double* o = out + (p0 + lane) * 5;
      if (poison) {
        for (int c = 0; c < 5; ++c) o[c] = bitsd(kNanBits);
      } else {
        const double uni = static_cast<double>(k - 1) / sum;
        const double dk = static_cast<double>(k);
        o[0] = uni;
        o[1] = uni * (static_cast<double>(neq) / dk);
        o[2] = uni * (static_cast<double>(nlt) / dk);
        o[3] = uni * (static_cast<double>(ngt) / dk);
        o[4] = static_cast<double>(neq) / dk;
      }
    }
  }
}

__global__ void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }

static unsigned grid_for(int64_t items, int per_block) {
  int64_t g = (items + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > (1 << 20)) g = 1 << 20;
  return static_cast<unsigned>(g);
}

hipError_t launch_jaccard(const int32_t* a, const int32_t* b, int64_t npairs, int32_t k,
                          double* out, hipStream_t stream) {
  hipLaunchKernelGGL(jaccard_kernel, dim3(grid_for(npairs, 4)), dim3(256), 0, stream, a, b, npairs,
                     k, out);
  return hipGetLastError();
}

hipError_t launch_jaccard_pairs(const int32_t* store, int64_t nstore, int32_t k, const int64_t* ia,
                                const int64_t* ib, int64_t npairs, double* out,
                                unsigned long long* err, hipStream_t stream) {
  hipLaunchKernelGGL(jaccard_pairs_kernel, dim3(grid_for(npairs, 4)), dim3(256), 0, stream, store,
                     nstore, k, ia, ib, npairs, out, err);
  return hipGetLastError();
}

hipError_t launch_wcard(const double* val, int64_t nvec, int32_t k, double* out,
                        hipStream_t stream) {
  hipLaunchKernelGGL(wcard_kernel, dim3(grid_for(nvec, 1)), dim3(kWave), 0, stream, val, nvec, k,
                     out);
  return hipGetLastError();
}

hipError_t launch_merge(const int32_t* in_idx, const double* in_val, int64_t r, int32_t k,
                        int32_t* out_idx, double* out_val, hipStream_t stream) {
  hipLaunchKernelGGL(merge_kernel, dim3(grid_for(k, 256)), dim3(256), 0, stream, in_idx, in_val, r,
                     k, out_idx, out_val);
  return hipGetLastError();
}

hipError_t launch_setops(const int32_t* sa, const double* ya, const int32_t* sb, const double* yb,
                         int64_t npairs, int32_t k, double* out, hipStream_t stream) {
  hipLaunchKernelGGL(setops_kernel, dim3(grid_for(npairs, kSetPairs)), dim3(kSetPairs), 0, stream,
                     sa, ya, sb, yb, npairs, k, out);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, hipStream_t stream) {
  hipLaunchKernelGGL(zero_u64_kernel, dim3(1), dim3(1), 0, stream, p);
  return hipGetLastError();
}

}  // namespace gm
