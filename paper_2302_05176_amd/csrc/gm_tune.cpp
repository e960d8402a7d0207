// gm_tune.cpp -- autotuner for the FastGM launch options.
//
// The FastGM kernels expose a few schedule knobs that change the work split
// but never the result: waves sharing one small vector, the registers-per-
// block tiling (up to which size a vector is sketched by one wave with its
// own register set rather than by a workgroup sharing one), the per-lane
// table load before an element moves to the segment path, the expected walk
// length that sends an element there directly from its first arrival, and
// the threshold republish period.  gm_autotune times the caller's own
// batch under a coordinate descent over those knobs (HIP events on the
// caller's stream, median of `reps` runs per point), keeps the fastest
// setting, and records it in a JSON-lines cache keyed by (GPU architecture,
// k_max, log2 nvec, log2 nnz, uniform or per-vector k) so that a later call
// on a similar batch applies it without timing anything.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <sys/stat.h>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "gm.h"

namespace {

std::mutex g_tune_mu;

struct Knobs {
  int64_t small_waves, map_load, seg_rest, republish, wave_lim;
};

gm_status set_knobs(const Knobs& k) {
  gm_status s;
  if ((s = gm_set_option(GM_OPT_SMALL_WAVES, k.small_waves)) != GM_OK) return s;
  if ((s = gm_set_option(GM_OPT_MAP_LOAD, k.map_load)) != GM_OK) return s;
  if ((s = gm_set_option(GM_OPT_SEG_REST, k.seg_rest)) != GM_OK) return s;
  if ((s = gm_set_option(GM_OPT_WAVE_LIM, k.wave_lim)) != GM_OK) return s;
  return gm_set_option(GM_OPT_REPUBLISH, k.republish);
}

std::string cache_path() {
  const char* p = std::getenv("GM_TUNE_CACHE");
  if (p && *p) return p;
  const char* home = std::getenv("HOME");
  return std::string(home ? home : "/tmp") + "/.cache/gm_tune.jsonl";
}

int ilog2(int64_t x) {
  int l = 0;
  while (x > 1) {
    x >>= 1;
    ++l;
  }
  return l;
}

std::string cache_key(int32_t k_max, int64_t nvec, int64_t nnz, bool batched) {
  int dev = 0;
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
    arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  std::ostringstream os;
  os << arch << "|k" << k_max << "|v" << ilog2(nvec) << "|e" << ilog2(nnz > 0 ? nnz : 1) << "|"
     << (batched ? "kvec" : "k");
  return os.str();
}

// Very small reader for the lines this file writes:
// {"key": "...", "small_waves": a, "map_load": b, "seg_rest": c, "republish": d,
//  "wave_lim": f, "ms": e}  (a line without wave_lim has the default 8191)
bool parse_line(const std::string& line, std::string& key, Knobs& k, double& ms) {
  auto field = [&](const char* name, std::string& out) {
    const std::string pat = std::string("\"") + name + "\":";
    size_t p = line.find(pat);
    if (p == std::string::npos) return false;
    p += pat.size();
    while (p < line.size() && line[p] == ' ') ++p;
    size_t e = p;
    if (p < line.size() && line[p] == '"') {
      e = line.find('"', p + 1);
      if (e == std::string::npos) return false;
      out = line.substr(p + 1, e - p - 1);
      return true;
    }
    while (e < line.size() && line[e] != ',' && line[e] != '}') ++e;
    out = line.substr(p, e - p);
    return true;
  };
  std::string a, b, c, d, e;
  if (!field("key", key) || !field("small_waves", a) || !field("map_load", b) ||
      !field("seg_rest", c) || !field("republish", d) || !field("ms", e))
    return false;
  k.small_waves = std::atoll(a.c_str());
  k.map_load = std::atoll(b.c_str());
  k.seg_rest = std::atoll(c.c_str());
  k.republish = std::atoll(d.c_str());
  std::string f;
  k.wave_lim = field("wave_lim", f) ? std::atoll(f.c_str()) : 8191;
  ms = std::atof(e.c_str());
  return true;
}

bool cache_lookup(const std::string& key, Knobs& k, double& ms) {
  std::ifstream in(cache_path());
  std::string line, lk;
  bool hit = false;
  Knobs kk;
  double m;
  while (std::getline(in, line))
    if (parse_line(line, lk, kk, m) && lk == key) {
      k = kk;
      ms = m;
      hit = true;  // last entry wins
    }
  return hit;
}

void cache_store(const std::string& key, const Knobs& k, double ms) {
  const std::string path = cache_path();
  const size_t slash = path.rfind('/');
  if (slash != std::string::npos && slash > 0)
    (void)::mkdir(path.substr(0, slash).c_str(), 0755);  // best effort, one level
  std::ofstream out(path, std::ios::app);
  if (!out) return;
  out << "{\"key\": \"" << key << "\", \"small_waves\": " << k.small_waves
      << ", \"map_load\": " << k.map_load << ", \"seg_rest\": " << k.seg_rest
      << ", \"republish\": " << k.republish << ", \"wave_lim\": " << k.wave_lim
      << ", \"ms\": " << ms << "}\n";
}

}  // namespace

extern "C" gm_status gm_autotune(const int32_t* indices, const float* weights,
                                 const int64_t* offsets, int64_t nvec, const int32_t* k_per_vec,
                                 const int64_t* out_offsets, int32_t k_max, uint64_t seed,
                                 int32_t* out_idx, double* out_val, int32_t reps, int32_t use_cache,
                                 gm_tune_result* result, hipStream_t stream) {
  if (nvec < 1 || k_max < 1 || k_max > GM_K_MAX || reps < 1 || !offsets) return GM_ERR_INVALID_ARG;
  const bool batched = k_per_vec != nullptr;
  if (batched != (out_offsets != nullptr)) return GM_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  // nnz from the device (a tuning call may synchronise)
  int64_t ends[2] = {0, 0};
  hipError_t e = hipStreamSynchronize(stream);
  if (e == hipSuccess) e = hipMemcpy(&ends[0], offsets, sizeof(int64_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&ends[1], offsets + nvec, sizeof(int64_t), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return GM_ERR_DEVICE;
  const std::string key = cache_key(k_max, nvec, ends[1] - ends[0], batched);
  Knobs best{0, 14, 12, 8, 8191};
  double best_ms = 0.0;
  if (use_cache && cache_lookup(key, best, best_ms)) {
    gm_status s = set_knobs(best);
    if (s != GM_OK) return s;
    if (result) {
      result->small_waves = static_cast<int32_t>(best.small_waves);
      result->map_load = static_cast<int32_t>(best.map_load);
      result->seg_rest = static_cast<int32_t>(best.seg_rest);
      result->republish = static_cast<int32_t>(best.republish);
      result->wave_lim = static_cast<int32_t>(best.wave_lim);
      result->ms = best_ms;
      result->from_cache = 1;
    }
    return GM_OK;
  }
  hipEvent_t ev0, ev1;
  if (hipEventCreate(&ev0) != hipSuccess) return GM_ERR_DEVICE;
  if (hipEventCreate(&ev1) != hipSuccess) {
    (void)hipEventDestroy(ev0);
    return GM_ERR_DEVICE;
  }
  auto run_once = [&]() -> gm_status {
    if (batched)
      return gm_sketch_batched(indices, weights, offsets, nvec, k_per_vec, out_offsets, k_max, seed,
                               GM_FORM_FASTGM, out_idx, out_val, stream);
    return gm_sketch(indices, weights, offsets, nvec, k_max, seed, out_idx, out_val, stream);
  };
  auto time_knobs = [&](const Knobs& k, double& ms) -> gm_status {
    gm_status s = set_knobs(k);
    if (s != GM_OK) return s;
    if ((s = run_once()) != GM_OK) return s;  // warm-up (first use of a launch shape)
    std::vector<float> t;
    for (int r = 0; r < reps; ++r) {
      if (hipEventRecord(ev0, stream) != hipSuccess) return GM_ERR_DEVICE;
      if ((s = run_once()) != GM_OK) return s;
      if (hipEventRecord(ev1, stream) != hipSuccess) return GM_ERR_DEVICE;
      if (hipEventSynchronize(ev1) != hipSuccess) return GM_ERR_DEVICE;
      float m = 0.0f;
      if (hipEventElapsedTime(&m, ev0, ev1) != hipSuccess) return GM_ERR_DEVICE;
      t.push_back(m);
    }
    std::sort(t.begin(), t.end());
    ms = t[t.size() / 2];
    return GM_OK;
  };
  gm_status s = time_knobs(best, best_ms);
  const std::vector<int64_t> grid_waves = {0, 1, 2, 4, 8};
  const std::vector<int64_t> grid_seg = {4, 8, 12, 16, 32, 64};
  const std::vector<int64_t> grid_map = {8, 10, 12, 14, 16};
  const std::vector<int64_t> grid_rep = {4, 8, 16};
  // registers-per-block tiling: only the k <= 256 kernel has a choice (a
  // batch with per-vector k may have such vectors whatever its k_max)
  const std::vector<int64_t> grid_lim = (k_max <= 256 || batched)
                                            ? std::vector<int64_t>{0, 511, 2047, 8191, 32767}
                                            : std::vector<int64_t>{};
  for (int axis = 0; axis < 5 && s == GM_OK; ++axis) {
    const std::vector<int64_t>& grid = axis == 0   ? grid_waves
                                       : axis == 1 ? grid_seg
                                       : axis == 2 ? grid_map
                                       : axis == 3 ? grid_rep
                                                   : grid_lim;
    for (int64_t v : grid) {
      Knobs k = best;
      int64_t* field = axis == 0   ? &k.small_waves
                       : axis == 1 ? &k.seg_rest
                       : axis == 2 ? &k.map_load
                       : axis == 3 ? &k.republish
                                   : &k.wave_lim;
      if (*field == v) continue;
      *field = v;
      double ms = 0.0;
      s = time_knobs(k, ms);
      if (s != GM_OK) break;
      if (ms < best_ms) {
        best_ms = ms;
        best = k;
      }
    }
  }
  (void)hipEventDestroy(ev0);
  (void)hipEventDestroy(ev1);
  if (s != GM_OK) return s;
  s = set_knobs(best);
  if (s != GM_OK) return s;
  if (use_cache) cache_store(key, best, best_ms);
  if (result) {
    result->small_waves = static_cast<int32_t>(best.small_waves);
    result->map_load = static_cast<int32_t>(best.map_load);
    result->seg_rest = static_cast<int32_t>(best.seg_rest);
    result->republish = static_cast<int32_t>(best.republish);
    result->wave_lim = static_cast<int32_t>(best.wave_lim);
    result->ms = best_ms;
    result->from_cache = 0;
  }
  return GM_OK;
}
