// gm_api.hip -- the C ABI declared in include/gm.h.
//
// Host side only: argument validation (synchronous, nothing is enqueued on
// error), the per-device workspace (data-error counter), process-wide tuning
// options, and dispatch to the kernel launchers.  No call allocates on the
// steady-state path: the workspace is created by the first call on a device.
#include <atomic>
#include <map>
#include <mutex>

#include "gm.h"
#include "gm_common.h"

namespace gm {
hipError_t launch_plain(const SketchArgs& p, const PlainScratch& ps, int cus, hipStream_t stream);
int64_t plain_scratch_regs(int cus);
int64_t plain_scratch_counters(int cus);
hipError_t launch_fastgm(const SketchArgs& s, int pos_bits, double t0_scale, int map_load,
                         int republish, double seg_rest, int small_waves, int wave_lim, int32_t* list,
                         void* plan, void* big, int32_t* pool, int64_t pool_cap,
                         void* heavy, int64_t heavy_waves, void* part, int update, int cus,
                         unsigned long long* stats, hipStream_t stream);
size_t plan_state_bytes();
int64_t heavy_list_bytes();
void timing_enable(int level);
int timing_collect(int n, char (*names)[64], double* ms, long long* launches);
void timing_reset();
size_t big_info_bytes();
size_t part_scratch_bytes();
hipError_t launch_jaccard(const int32_t* a, const int32_t* b, int64_t npairs, int32_t k,
                          double* out, hipStream_t stream);
hipError_t launch_jaccard_pairs(const int32_t* store, int64_t nstore, int32_t k, const int64_t* ia,
                                const int64_t* ib, int64_t npairs, double* out,
                                unsigned long long* err, hipStream_t stream);
hipError_t launch_wcard(const double* val, int64_t nvec, int32_t k, double* out,
                        hipStream_t stream);
hipError_t launch_merge(const int32_t* in_idx, const double* in_val, int64_t r, int32_t k,
                        int32_t* out_idx, double* out_val, hipStream_t stream);
hipError_t launch_zero_u64(unsigned long long* p, hipStream_t stream);
hipError_t launch_setops(const int32_t* sa, const double* ya, const int32_t* sb, const double* yb,
                         int64_t npairs, int32_t k, double* out, hipStream_t stream);
hipError_t launch_rate_probe(int what, int64_t lanes, int32_t steps, uint64_t seed_mix,
                             double* out, hipStream_t stream);
}  // namespace gm

namespace {

constexpr int kMaxDevices = 64;

// Planner workspace of one (device, stream): the vector list and the class
// counters.  Keyed by stream so that calls on different streams never share it.
// Candidate-list pool of the big vectors (entries): 256 MiB.  A big vector
// that does not fit is walked over all of its entries instead.
constexpr int64_t kPoolCap = 64ll << 20;

struct PlanWorkspace {
  int32_t* list = nullptr;
  void* big = nullptr;   // one BigInfo per vector slot
  int64_t cap = 0;
  void* plan = nullptr;
  int32_t* pool = nullptr;
  void* heavy = nullptr;      // per-wave heavy-element lists of the FastGM walk
  int64_t heavy_waves = 0;
  void* part = nullptr;       // partial sketches of split big-vector walks
  void* plain = nullptr;      // partial registers and counters of split plain launches
};

// Resident waves per CU the heavy lists are sized for: the FastGM kernels
// need more than 128 VGPRs, so at most 3 waves per SIMD (a launch that could
// hold more is trimmed to this).
constexpr int kMaxWavesPerCu = 12;

constexpr int kStatSlots = 16;

// The data-error counter and the optional FastGM counters of each device
// live in static device memory (zero when the library is loaded), so that
// setting up a device allocates nothing.
static __device__ __align__(256) unsigned long long g_err_dev[1];
static __device__ __align__(256) unsigned long long g_stats_dev[kStatSlots];

// Scratch of gm_sketch_plain_noalloc: the partial registers and counters of
// a split plain launch, in static device memory instead of a workspace.
// kNoAllocRegs registers hold the split of one vector at any k (at most
// 2048 workgroups of 256 registers); kNoAllocCounters bounds the (vector,
// tile) pairs of a split launch.  In host code `scratch` names a host-side
// stand-in: only the address hipGetSymbolAddress returns for it is used.
constexpr int64_t kNoAllocRegs = 1ll << 19;
constexpr int64_t kNoAllocCounters = 4096;
constexpr size_t kNoAllocScratchBytes =
    static_cast<size_t>(kNoAllocRegs) * (sizeof(double) + sizeof(int32_t)) +
    2 * sizeof(int32_t) * static_cast<size_t>(kNoAllocCounters) + gm::kPlainPlanBytes;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

struct DeviceState {
  bool ready = false;
  unsigned long long* err = nullptr;
  unsigned long long* stats = nullptr;  // FastGM counters, when enabled
  void* noalloc = nullptr;              // this device's address of `scratch`
  int cus = 0;
  std::map<hipStream_t, PlanWorkspace> plans;
};

std::mutex g_mu;
DeviceState g_dev[kMaxDevices];

// Tuning / testing options (process-wide).  Each is read once per call, as
// an atomic, so a gm_set_option from another host thread (the autotuner
// beside a serving loop, say) takes effect from some call on and never
// tears a value; a call sees a mix of old and new options only while a
// change is under way.
std::atomic<int> g_pos_bits{31};
std::atomic<double> g_t0_scale{1.0};
std::atomic<int> g_map_load{14};
std::atomic<int> g_republish{8};
std::atomic<double> g_seg_rest{12.0};
std::atomic<int> g_small_waves{0};
std::atomic<int> g_wave_lim{8191};
std::atomic<bool> g_stats{false};

gm_status from_hip(hipError_t e) {
  if (e == hipSuccess) return GM_OK;
  if (e == hipErrorOutOfMemory) return GM_ERR_OUT_OF_MEMORY;
  return GM_ERR_DEVICE;
}

// State of the current device, set up on first use: the device addresses of
// the static counters and scratch (each device holds its own copies) and
// the CU count.  Allocates nothing.
gm_status device_state(DeviceState** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return GM_ERR_DEVICE;
  if (dev < 0 || dev >= kMaxDevices) return GM_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceState& st = g_dev[dev];
  if (!st.ready) {
    void* e_ptr = nullptr;
    void* s_ptr = nullptr;
    void* n_ptr = nullptr;
    hipError_t e = hipGetSymbolAddress(&e_ptr, HIP_SYMBOL(g_err_dev));
    if (e != hipSuccess) return from_hip(e);
    e = hipGetSymbolAddress(&s_ptr, HIP_SYMBOL(g_stats_dev));
    if (e != hipSuccess) return from_hip(e);
    e = hipGetSymbolAddress(&n_ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return from_hip(e);
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return from_hip(e);
    st.err = static_cast<unsigned long long*>(e_ptr);
    st.stats = static_cast<unsigned long long*>(s_ptr);
    st.noalloc = n_ptr;
    st.cus = prop.multiProcessorCount;
    st.ready = true;
  }
  *out = &st;
  return GM_OK;
}

// Planner workspace for `stream` with room for nvec vector ids.  Grows (with
// hipMalloc) only when a call needs more room than any earlier call did.
gm_status plan_workspace(DeviceState* st, hipStream_t stream, int64_t nvec, PlanWorkspace** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  PlanWorkspace& ws = st->plans[stream];
  // each piece on its own, so that a call after a failed allocation retries
  // what is missing
  if (!ws.plan) {
    hipError_t e = hipMalloc(&ws.plan, gm::plan_state_bytes());
    if (e != hipSuccess) {
      ws.plan = nullptr;
      return from_hip(e);
    }
  }
  if (!ws.pool) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, sizeof(int32_t) * static_cast<size_t>(kPoolCap));
    if (e != hipSuccess) return from_hip(e);
    ws.pool = static_cast<int32_t*>(q);
  }
  if (!ws.heavy) {
    void* q = nullptr;
    const int64_t waves = static_cast<int64_t>(st->cus) * kMaxWavesPerCu;
    hipError_t e = hipMalloc(&q, static_cast<size_t>(waves * gm::heavy_list_bytes()));
    if (e != hipSuccess) return from_hip(e);
    ws.heavy = q;
    ws.heavy_waves = waves;
  }
  if (!ws.part) {
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, gm::part_scratch_bytes());
    if (e != hipSuccess) return from_hip(e);
    ws.part = q;
  }
  if (ws.cap < nvec) {
    if (ws.list) (void)hipFree(ws.list);
    if (ws.big) (void)hipFree(ws.big);
    ws.list = nullptr;
    ws.big = nullptr;
    ws.cap = 0;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, sizeof(int32_t) * static_cast<size_t>(nvec));
    if (e != hipSuccess) return from_hip(e);
    ws.list = static_cast<int32_t*>(p);
    e = hipMalloc(&ws.big, gm::big_info_bytes() * static_cast<size_t>(nvec));
    if (e != hipSuccess) return from_hip(e);
    ws.cap = nvec;
  }
  *out = &ws;
  return GM_OK;
}

size_t plain_scratch_bytes(int cus) {
  return static_cast<size_t>(gm::plain_scratch_regs(cus)) * (sizeof(double) + sizeof(int32_t)) +
         2 * sizeof(int32_t) * static_cast<size_t>(gm::plain_scratch_counters(cus)) +
         gm::kPlainPlanBytes;
}

// Scratch of split plain launches on `stream` (created on first use, with
// its counters zeroed; the kernel leaves them at zero).
gm_status plain_workspace(DeviceState* st, hipStream_t stream, void** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  PlanWorkspace& ws = st->plans[stream];
  if (!ws.plain) {
    void* q = nullptr;
    const size_t bytes = plain_scratch_bytes(st->cus);
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) return from_hip(e);
    e = hipMemset(q, 0, bytes);
    if (e != hipSuccess) {
      (void)hipFree(q);
      return from_hip(e);
    }
    ws.plain = q;
  }
  *out = ws.plain;
  return GM_OK;
}

gm_status sketch_common(const int32_t* indices, const float* weights, const int64_t* offsets,
                        int64_t nvec, int32_t k_uniform, const int32_t* kvec,
                        const int64_t* outoff, int32_t k_max, uint64_t seed, gm_form form,
                        int32_t* out_idx, double* out_val, hipStream_t stream,
                        int update = 0, bool noalloc = false) {
  if (nvec < 0 || k_max < 1 || k_max > GM_K_MAX) return GM_ERR_INVALID_ARG;
  if (form != GM_FORM_FASTGM && form != GM_FORM_PLAIN) return GM_ERR_INVALID_ARG;
  if (nvec == 0) return GM_OK;
  if (!indices || !weights || !offsets || !out_idx || !out_val) return GM_ERR_INVALID_ARG;
  DeviceState* st = nullptr;
  gm_status s = device_state(&st);
  if (s != GM_OK) return s;
  gm::SketchArgs a;
  a.idx = indices;
  a.w = weights;
  a.off = offsets;
  a.nvec = nvec;
  a.k_uniform = k_uniform;
  a.kvec = kvec;
  a.outoff = outoff;
  a.k_max = k_max;
  a.seed_mix = gm::mix(seed);
  a.out_idx = out_idx;
  a.out_val = out_val;
  a.err = st->err;
  if (form == GM_FORM_PLAIN) {
    gm::PlainScratch ps{nullptr, gm::plain_scratch_regs(st->cus),
                        gm::plain_scratch_counters(st->cus), false};
    if (noalloc) {
      ps = gm::PlainScratch{st->noalloc, kNoAllocRegs, kNoAllocCounters, true};
    } else {
      s = plain_workspace(st, stream, &ps.base);
      if (s != GM_OK) return s;
    }
    return from_hip(gm::launch_plain(a, ps, st->cus, stream));
  }
  if (nvec > 0x7FFFFFFF) return GM_ERR_UNSUPPORTED;
  PlanWorkspace* ws = nullptr;
  s = plan_workspace(st, stream, nvec, &ws);
  if (s != GM_OK) return s;
  return from_hip(gm::launch_fastgm(a, g_pos_bits, g_t0_scale, g_map_load, g_republish,
                                    g_seg_rest, g_small_waves, g_wave_lim, ws->list, ws->plan, ws->big,
                                    ws->pool, kPoolCap, ws->heavy, ws->heavy_waves, ws->part, update,
                                    st->cus, g_stats ? st->stats : nullptr, stream));
}

}  // namespace

extern "C" {

gm_status gm_sketch(const int32_t* indices, const float* weights, const int64_t* offsets,
                    int64_t nvec, int32_t k, uint64_t seed, int32_t* out_idx, double* out_val,
                    hipStream_t stream) {
  if (k < 1 || k > GM_K_MAX) return GM_ERR_INVALID_ARG;
  return sketch_common(indices, weights, offsets, nvec, k, nullptr, nullptr, k, seed,
                       GM_FORM_FASTGM, out_idx, out_val, stream);
}

gm_status gm_sketch_update(const int32_t* indices, const float* weights, const int64_t* offsets,
                           int64_t nvec, int32_t k, uint64_t seed, int32_t* sk_idx, double* sk_val,
                           hipStream_t stream) {
  if (k < 1 || k > GM_K_MAX) return GM_ERR_INVALID_ARG;
  return sketch_common(indices, weights, offsets, nvec, k, nullptr, nullptr, k, seed,
                       GM_FORM_FASTGM, sk_idx, sk_val, stream, 1);
}

gm_status gm_sketch_plain(const int32_t* indices, const float* weights, const int64_t* offsets,
                          int64_t nvec, int32_t k, uint64_t seed, int32_t* out_idx,
                          double* out_val, hipStream_t stream) {
  if (k < 1 || k > GM_K_MAX) return GM_ERR_INVALID_ARG;
  return sketch_common(indices, weights, offsets, nvec, k, nullptr, nullptr, k, seed,
                       GM_FORM_PLAIN, out_idx, out_val, stream);
}

gm_status gm_sketch_plain_noalloc(const int32_t* indices, const float* weights,
                                  const int64_t* offsets, int64_t nvec, int32_t k, uint64_t seed,
                                  int32_t* out_idx, double* out_val, hipStream_t stream) {
  if (k < 1 || k > GM_K_MAX) return GM_ERR_INVALID_ARG;
  return sketch_common(indices, weights, offsets, nvec, k, nullptr, nullptr, k, seed,
                       GM_FORM_PLAIN, out_idx, out_val, stream, 0, true);
}

gm_status gm_sketch_batched(const int32_t* indices, const float* weights, const int64_t* offsets,
                            int64_t nvec, const int32_t* k_per_vec, const int64_t* out_offsets,
                            int32_t k_max, uint64_t seed, gm_form form, int32_t* out_idx,
                            double* out_val, hipStream_t stream) {
  if (nvec > 0 && (!k_per_vec || !out_offsets)) return GM_ERR_INVALID_ARG;
  return sketch_common(indices, weights, offsets, nvec, k_max, k_per_vec, out_offsets, k_max,
                       seed, form, out_idx, out_val, stream);
}

gm_status gm_reserve(int64_t nvec, hipStream_t stream) {
  if (nvec < 0 || nvec > 0x7FFFFFFF) return GM_ERR_INVALID_ARG;
  DeviceState* st = nullptr;
  gm_status s = device_state(&st);
  if (s != GM_OK) return s;
  PlanWorkspace* ws = nullptr;
  s = plan_workspace(st, stream, nvec > 0 ? nvec : 1, &ws);
  if (s != GM_OK) return s;
  void* pscratch = nullptr;
  return plain_workspace(st, stream, &pscratch);
}

gm_status gm_workspace_bytes(int64_t nvec, int64_t* bytes) {
  if (!bytes || nvec < 0 || nvec > 0x7FFFFFFF) return GM_ERR_INVALID_ARG;
  DeviceState* st = nullptr;
  gm_status s = device_state(&st);
  if (s != GM_OK) return s;
  const int64_t n = nvec > 0 ? nvec : 1;
  const int64_t waves = static_cast<int64_t>(st->cus) * kMaxWavesPerCu;
  *bytes = static_cast<int64_t>(gm::plan_state_bytes()) +
           static_cast<int64_t>(sizeof(int32_t)) * kPoolCap + waves * gm::heavy_list_bytes() +
           static_cast<int64_t>(gm::part_scratch_bytes()) +
           n * static_cast<int64_t>(sizeof(int32_t) + gm::big_info_bytes()) +
           static_cast<int64_t>(plain_scratch_bytes(st->cus));
  return GM_OK;
}

gm_status gm_jaccard_est(const int32_t* idx_a, const int32_t* idx_b, int64_t npairs, int32_t k,
                         double* out, hipStream_t stream) {
  if (npairs < 0 || k < 1) return GM_ERR_INVALID_ARG;
  if (npairs == 0) return GM_OK;
  if (!idx_a || !idx_b || !out) return GM_ERR_INVALID_ARG;
  return from_hip(gm::launch_jaccard(idx_a, idx_b, npairs, k, out, stream));
}

gm_status gm_jaccard_est_pairs(const int32_t* store_idx, int64_t nstore, int32_t k,
                               const int64_t* ia, const int64_t* ib, int64_t npairs, double* out,
                               hipStream_t stream) {
  if (npairs < 0 || nstore < 0 || k < 1) return GM_ERR_INVALID_ARG;
  if (npairs == 0) return GM_OK;
  if (!store_idx || !ia || !ib || !out) return GM_ERR_INVALID_ARG;
  DeviceState* st = nullptr;
  gm_status s = device_state(&st);
  if (s != GM_OK) return s;
  return from_hip(
      gm::launch_jaccard_pairs(store_idx, nstore, k, ia, ib, npairs, out, st->err, stream));
}

gm_status gm_wcard_est(const double* val, int64_t nvec, int32_t k, double* out,
                       hipStream_t stream) {
  if (nvec < 0 || k < 2) return GM_ERR_INVALID_ARG;
  if (nvec == 0) return GM_OK;
  if (!val || !out) return GM_ERR_INVALID_ARG;
  return from_hip(gm::launch_wcard(val, nvec, k, out, stream));
}

gm_status gm_rate_probe(int32_t what, int64_t lanes, int32_t steps, uint64_t seed, double* out,
                        hipStream_t stream) {
  if ((what != 0 && what != 1) || lanes < 0 || steps < 1 || steps > GM_K_MAX)
    return GM_ERR_INVALID_ARG;
  if (lanes == 0) return GM_OK;
  if (!out) return GM_ERR_INVALID_ARG;
  return from_hip(gm::launch_rate_probe(what, lanes, steps, gm::mix(seed), out, stream));
}

gm_status gm_merge(const int32_t* in_idx, const double* in_val, int64_t r, int32_t k,
                   int32_t* out_idx, double* out_val, hipStream_t stream) {
  if (r < 1 || k < 1) return GM_ERR_INVALID_ARG;
  if (!in_idx || !in_val || !out_idx || !out_val) return GM_ERR_INVALID_ARG;
  return from_hip(gm::launch_merge(in_idx, in_val, r, k, out_idx, out_val, stream));
}

gm_status gm_setops(const int32_t* idx_a, const double* val_a, const int32_t* idx_b,
                    const double* val_b, int64_t npairs, int32_t k, double* out,
                    hipStream_t stream) {
  if (npairs < 0 || k < 2) return GM_ERR_INVALID_ARG;
  if (npairs == 0) return GM_OK;
  if (!idx_a || !val_a || !idx_b || !val_b || !out) return GM_ERR_INVALID_ARG;
  return from_hip(gm::launch_setops(idx_a, val_a, idx_b, val_b, npairs, k, out, stream));
}

gm_status gm_get_data_errors(int64_t* host_count, hipStream_t stream) {
  if (!host_count) return GM_ERR_INVALID_ARG;
  DeviceState* st = nullptr;
  gm_status s = device_state(&st);
  if (s != GM_OK) return s;
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return from_hip(e);
  unsigned long long v = 0;
  e = hipMemcpy(&v, st->err, sizeof(v), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return from_hip(e);
  *host_count = static_cast<int64_t>(v);
  return GM_OK;
}

gm_status gm_reset_data_errors(hipStream_t stream) {
  DeviceState* st = nullptr;
  gm_status s = device_state(&st);
  if (s != GM_OK) return s;
  return from_hip(gm::launch_zero_u64(st->err, stream));
}

gm_status gm_set_option(gm_option opt, int64_t value) {
  switch (opt) {
    case GM_OPT_POS_BITS:
      // the packed word's low bits hold a non-negative int32 index
      if (value < 31 || value > 62) return GM_ERR_INVALID_ARG;
      g_pos_bits = static_cast<int>(value);
      return GM_OK;
    case GM_OPT_T0_SCALE_PPM:
      if (value < 1) return GM_ERR_INVALID_ARG;
      g_t0_scale = static_cast<double>(value) * 1e-6;
      return GM_OK;
    case GM_OPT_MAP_LOAD:
      if (value < 0 || value > 16) return GM_ERR_INVALID_ARG;
      g_map_load = static_cast<int>(value);
      return GM_OK;
    case GM_OPT_SEG_REST:
      if (value < 0 || value > 1000000) return GM_ERR_INVALID_ARG;
      g_seg_rest = static_cast<double>(value);
      return GM_OK;
    case GM_OPT_SMALL_WAVES:
      if (value != 0 && value != 1 && value != 2 && value != 4 && value != 8)
        return GM_ERR_INVALID_ARG;
      g_small_waves = static_cast<int>(value);
      return GM_OK;
    case GM_OPT_TIMING:
      if (value < 0 || value > 2) return GM_ERR_INVALID_ARG;
      {
        std::lock_guard<std::mutex> lock(g_mu);
        gm::timing_enable(static_cast<int>(value));
      }
      return GM_OK;
    case GM_OPT_WAVE_LIM:
      if (value != 0 && (value < 15 || value > 32767 || ((value + 1) & value) != 0))
        return GM_ERR_INVALID_ARG;
      g_wave_lim = static_cast<int>(value);
      return GM_OK;
    case GM_OPT_STATS:
      if (value != 0 && value != 1) return GM_ERR_INVALID_ARG;
      g_stats = value != 0;
      return GM_OK;
    case GM_OPT_REPUBLISH:
      if (value < 1 || value > 4096 || (value & (value - 1)) != 0) return GM_ERR_INVALID_ARG;
      g_republish = static_cast<int>(value);
      return GM_OK;
  }
  return GM_ERR_INVALID_ARG;
}

gm_status gm_get_stats(int64_t* host_counters, int32_t n, hipStream_t stream) {
  if (!host_counters || n < 1 || n > kStatSlots) return GM_ERR_INVALID_ARG;
  DeviceState* st = nullptr;
  gm_status s = device_state(&st);
  if (s != GM_OK) return s;
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return from_hip(e);
  unsigned long long v[kStatSlots];
  e = hipMemcpy(v, st->stats, sizeof(v), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return from_hip(e);
  for (int i = 0; i < n; ++i) host_counters[i] = static_cast<int64_t>(v[i]);
  return GM_OK;
}

int32_t gm_get_timing(int32_t n, char (*names)[64], double* total_ms, int64_t* launches) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (n < 0) return -1;
  std::vector<long long> l(static_cast<size_t>(n > 0 ? n : 1));
  const int m = gm::timing_collect(n, names, total_ms, l.data());
  for (int i = 0; i < m; ++i) launches[i] = l[i];
  return m;
}

void gm_reset_timing(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  gm::timing_reset();
}

gm_status gm_reset_stats(hipStream_t stream) {
  DeviceState* st = nullptr;
  gm_status s = device_state(&st);
  if (s != GM_OK) return s;
  hipError_t e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return from_hip(e);
  return from_hip(hipMemset(st->stats, 0, sizeof(unsigned long long) * kStatSlots));
}

const char* gm_status_string(gm_status status) {
  switch (status) {
    case GM_OK: return "ok";
    case GM_ERR_INVALID_ARG: return "invalid argument";
    case GM_ERR_OUT_OF_MEMORY: return "out of device memory";
    case GM_ERR_DEVICE: return "HIP device error";
    case GM_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

void gm_release_stream(hipStream_t stream) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_mu);
  DeviceState& st = g_dev[dev];
  auto it = st.plans.find(stream);
  if (it == st.plans.end()) return;
  (void)hipStreamSynchronize(stream);
  if (it->second.list) (void)hipFree(it->second.list);
  if (it->second.big) (void)hipFree(it->second.big);
  if (it->second.plan) (void)hipFree(it->second.plan);
  if (it->second.pool) (void)hipFree(it->second.pool);
  if (it->second.heavy) (void)hipFree(it->second.heavy);
  if (it->second.part) (void)hipFree(it->second.part);
  if (it->second.plain) (void)hipFree(it->second.plain);
  st.plans.erase(it);
}

void gm_release(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  int cur = 0;
  (void)hipGetDevice(&cur);
  for (int d = 0; d < kMaxDevices; ++d) {
    DeviceState& st = g_dev[d];
    if (st.plans.empty()) continue;
    (void)hipSetDevice(d);
    for (auto& kv : st.plans) {
      if (kv.second.list) (void)hipFree(kv.second.list);
      if (kv.second.big) (void)hipFree(kv.second.big);
      if (kv.second.plan) (void)hipFree(kv.second.plan);
      if (kv.second.pool) (void)hipFree(kv.second.pool);
      if (kv.second.heavy) (void)hipFree(kv.second.heavy);
      if (kv.second.part) (void)hipFree(kv.second.part);
      if (kv.second.plain) (void)hipFree(kv.second.plain);
    }
    st.plans.clear();
  }
  (void)hipSetDevice(cur);
}

}  // extern "C"
