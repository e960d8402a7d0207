// Banding LSH index over stored Gumbel-Max sketches (Sec. 1: each register
// s_j maps similar vectors to the same element with probability J_P, so the
// registers can key a locality-sensitive index for sub-linear similarity
// search).
//
// Band b of a sketch is its registers b*rows .. b*rows + rows - 1.  A stored
// item is a candidate for a query when, in some band, all `rows` register
// indices are equal and non-negative (an empty or poisoned register never
// matches, as in the Jaccard estimator).  With independent registers a pair
// at probability-Jaccard J is a candidate with probability
// 1 - (1 - J^rows)^bands.
//
// Build: one 64-bit key per (item, band): the band in the top 6 bits over 58
// bits of a splitmix64 chain of the band's indices (a band with a negative
// index gets a key that no query searches for); keys and item ids are sorted
// together (radix sort).  Query: one wave per query; each lane takes bands,
// binary-searches its band key, and verifies every item under that key
// against the query's indices exactly (so a hash collision never makes a
// candidate); the matches are deduplicated by a sort in LDS.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>
#include <stdint.h>

#include "gm.h"
#include "gm_common.h"

struct gm_lsh_index {
  const int32_t* store;  // caller's [nstore][k] indices (not owned)
  int64_t nstore;
  int32_t k, bands, rows;
  uint64_t* keys;        // [nstore * bands], sorted
  int32_t* ids;          // item of each key
  int64_t n;             // nstore * bands
};

namespace gm {
namespace {

constexpr int kLshMaxBands = 64;
constexpr uint64_t kNoBand = ~0ull;     // key of a band with a negative index
constexpr int kLshCap = 2048;           // band matches per query held in LDS
constexpr int kLshBlock = 64;           // one wave per query

__device__ __forceinline__ uint64_t band_hash(uint64_t band, const int32_t* s, int rows, bool& ok) {
  uint64_t h = mix(0x4C5348ull ^ band);
  ok = true;
  for (int t = 0; t < rows; ++t) {
    const int32_t v = s[t];
    ok = ok && v >= 0;
    h = mix(h ^ static_cast<uint64_t>(static_cast<uint32_t>(v)));
  }
  return (band << 58) | (h >> 6);
}

__global__ void lsh_keys_kernel(const int32_t* store, int64_t nstore, int k, int bands, int rows,
                                uint64_t* keys, int32_t* ids) {
  const int64_t n = nstore * bands;
  for (int64_t t = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; t < n;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t item = t / bands;
    const int b = static_cast<int>(t - item * bands);
    bool ok;
    const uint64_t key = band_hash(static_cast<uint64_t>(b), store + item * k + b * rows, rows, ok);
    keys[t] = ok ? key : kNoBand;
    ids[t] = static_cast<int32_t>(item);
  }
}

// First position in [0, n) whose key is >= x.
__device__ __forceinline__ int64_t lower_bound(const uint64_t* keys, int64_t n, uint64_t x) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (keys[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(kLshBlock) void lsh_query_kernel(gm_lsh_index ix, const int32_t* query,
                                                              int64_t nq, int max_cand,
                                                              int32_t* cand, int32_t* count) {
  __shared__ int32_t found[kLshCap];
  __shared__ int nfound;
  const int lane = threadIdx.x;
  for (int64_t q = blockIdx.x; q < nq; q += gridDim.x) {
    const int32_t* qs = query + q * ix.k;
    if (lane == 0) nfound = 0;
    __syncthreads();
    for (int b = lane; b < ix.bands; b += kLshBlock) {
      bool ok;
      const uint64_t key = band_hash(static_cast<uint64_t>(b), qs + b * ix.rows, ix.rows, ok);
      if (!ok) continue;
      for (int64_t p = lower_bound(ix.keys, ix.n, key); p < ix.n && ix.keys[p] == key; ++p) {
        const int32_t item = ix.ids[p];
        const int32_t* ss = ix.store + static_cast<int64_t>(item) * ix.k + b * ix.rows;
        bool same = true;
        for (int t = 0; t < ix.rows && same; ++t) same = ss[t] == qs[b * ix.rows + t];
        if (same) {
          const int slot = atomicAdd(&nfound, 1);
          if (slot < kLshCap) found[slot] = item;
        }
      }
    }
    __syncthreads();
    const int nf = nfound;
    if (nf > kLshCap) {
      // more band matches than the LDS list holds: reported, not truncated
      if (lane == 0) count[q] = -1;
      __syncthreads();
      continue;
    }
    // sort the matches (bitonic, padded to a power of two with INT32_MAX)
    int np2 = 1;
    while (np2 < nf) np2 <<= 1;
    for (int i = nf + lane; i < np2; i += kLshBlock) found[i] = 0x7FFFFFFF;
    __syncthreads();
    for (int size = 2; size <= np2; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = lane; i < np2; i += kLshBlock) {
          const int j = i ^ stride;
          if (j > i) {
            const bool up = (i & size) == 0;
            const int32_t a = found[i], c = found[j];
            if ((a > c) == up) {
              found[i] = c;
              found[j] = a;
            }
          }
        }
        __syncthreads();
      }
    }
    // unique ids in ascending order: a stable compaction, 64 at a time
    int written = 0;
    for (int base = 0; base < nf; base += kLshBlock) {
      const int i = base + lane;
      const bool first = i < nf && (i == 0 || found[i] != found[i - 1]);
      const uint64_t m = __ballot(first);
      const int pos = written + __popcll(m & ((1ull << lane) - 1ull));
      if (first && pos < max_cand) cand[q * max_cand + pos] = found[i];
      written += __popcll(m);
    }
    if (lane == 0) count[q] = written;
    __syncthreads();
  }
}

}  // namespace
}  // namespace gm

extern "C" {

gm_status gm_lsh_build(const int32_t* store_idx, int64_t nstore, int32_t k, int32_t bands,
                       int32_t rows, gm_lsh_index** out, hipStream_t stream) {
  if (!out) return GM_ERR_INVALID_ARG;
  *out = nullptr;
  if (!store_idx || nstore < 1 || k < 1 || k > GM_K_MAX || bands < 1 ||
      bands > gm::kLshMaxBands || rows < 1 || static_cast<int64_t>(bands) * rows > k)
    return GM_ERR_INVALID_ARG;
  // item ids and the sort's item count are 32-bit
  if (nstore * bands > 0x7FFFFFFF) return GM_ERR_UNSUPPORTED;
  gm_lsh_index* ix = new gm_lsh_index();
  ix->store = store_idx;
  ix->nstore = nstore;
  ix->k = k;
  ix->bands = bands;
  ix->rows = rows;
  ix->n = nstore * bands;
  uint64_t* keys_in = nullptr;
  int32_t* ids_in = nullptr;
  void* temp = nullptr;
  size_t temp_bytes = 0;
  hipError_t e = hipMalloc(&ix->keys, sizeof(uint64_t) * ix->n);
  if (e == hipSuccess) e = hipMalloc(&ix->ids, sizeof(int32_t) * ix->n);
  if (e == hipSuccess) e = hipMalloc(&keys_in, sizeof(uint64_t) * ix->n);
  if (e == hipSuccess) e = hipMalloc(&ids_in, sizeof(int32_t) * ix->n);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(gm::lsh_keys_kernel, dim3(4096), dim3(256), 0, stream, store_idx, nstore, k,
                       bands, rows, keys_in, ids_in);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipcub::DeviceRadixSort::SortPairs(nullptr, temp_bytes, keys_in, ix->keys, ids_in, ix->ids,
                                           static_cast<int>(ix->n), 0, 64, stream);
  if (e == hipSuccess) e = hipMalloc(&temp, temp_bytes > 0 ? temp_bytes : 1);
  if (e == hipSuccess)
    e = hipcub::DeviceRadixSort::SortPairs(temp, temp_bytes, keys_in, ix->keys, ids_in, ix->ids,
                                           static_cast<int>(ix->n), 0, 64, stream);
  // the inputs of the sort are freed once it has run
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  (void)hipFree(temp);
  (void)hipFree(keys_in);
  (void)hipFree(ids_in);
  if (e != hipSuccess) {
    (void)hipFree(ix->keys);
    (void)hipFree(ix->ids);
    delete ix;
    return e == hipErrorOutOfMemory ? GM_ERR_OUT_OF_MEMORY : GM_ERR_DEVICE;
  }
  *out = ix;
  return GM_OK;
}

gm_status gm_lsh_query(const gm_lsh_index* index, const int32_t* query_idx, int64_t nq,
                       int32_t max_cand, int32_t* cand, int32_t* count, hipStream_t stream) {
  if (!index || nq < 0 || max_cand < 0) return GM_ERR_INVALID_ARG;
  if (nq == 0) return GM_OK;
  if (!query_idx || !count || (max_cand > 0 && !cand)) return GM_ERR_INVALID_ARG;
  const int64_t blocks = nq < 65536 ? nq : 65536;
  hipLaunchKernelGGL(gm::lsh_query_kernel, dim3(static_cast<unsigned>(blocks)), dim3(gm::kLshBlock),
                     0, stream, *index, query_idx, nq, max_cand, cand, count);
  return hipGetLastError() == hipSuccess ? GM_OK : GM_ERR_DEVICE;
}

gm_status gm_lsh_info(const gm_lsh_index* index, int64_t* nstore, int32_t* k, int32_t* bands,
                      int32_t* rows) {
  if (!index) return GM_ERR_INVALID_ARG;
  if (nstore) *nstore = index->nstore;
  if (k) *k = index->k;
  if (bands) *bands = index->bands;
  if (rows) *rows = index->rows;
  return GM_OK;
}

void gm_lsh_free(gm_lsh_index* index) {
  if (!index) return;
  (void)hipFree(index->keys);
  (void)hipFree(index->ids);
  delete index;
}

}  // extern "C"
