// gm_serve.cpp -- continuous-batching request loop for sketch and
// similarity queries.
//
// A trace of requests (arrival time, kind, payload) is replayed open-loop:
// a request joins the pending queue once its arrival time has passed.  The
// loop keeps `slots` batches in flight, one HIP stream each, and whenever a
// slot is free it admits pending requests in arrival order while the batch
// stays within its entry and request limits and the in-flight device bytes
// (each busy slot's staging buffers and its stream's library workspace) stay
// within the budget.  A partial batch is launched once its oldest
// request has waited `max_wait_us` (or when nothing else can arrive).  Each
// batch stages its sketch requests' entries in pinned memory, copies them to
// the slot's device buffers, sketches them with gm_sketch (FastGM form), and
// answers its Jaccard queries from the device-resident store with
// gm_jaccard_est_pairs; an event marks its completion.  Requests that
// arrive while earlier batches run are admitted into other slots, so their
// work overlaps on the device.  Latency = completion time - arrival time.
// A sketch depends only on its own entries, so a request's result is the
// same alone or in any batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <thread>
#include <vector>

#include "gm.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  int32_t* d_idx = nullptr;
  float* d_w = nullptr;
  int64_t* d_off = nullptr;
  int32_t* d_out_idx = nullptr;
  double* d_out_val = nullptr;
  int64_t* d_ia = nullptr;
  int64_t* d_ib = nullptr;
  double* d_jac = nullptr;
  int32_t* h_idx = nullptr;
  float* h_w = nullptr;
  int64_t* h_off = nullptr;
  int64_t* h_ia = nullptr;
  int64_t* h_ib = nullptr;
  double* h_jac = nullptr;
  int32_t* h_out_idx = nullptr;
  double* h_out_val = nullptr;
  std::vector<int64_t> sk_reqs;  // sketch requests of the batch, in order
  std::vector<int64_t> jq_reqs;  // Jaccard requests of the batch, in order
  int64_t bytes = 0;
  bool busy = false;
};

template <class T>
hipError_t dalloc(T** p, size_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), sizeof(T) * (n ? n : 1));
}

template <class T>
hipError_t halloc(T** p, size_t n) {
  return hipHostMalloc(reinterpret_cast<void**>(p), sizeof(T) * (n ? n : 1), hipHostMallocDefault);
}

void free_slot(Slot& s) {
  if (s.stream) {
    (void)hipStreamSynchronize(s.stream);
    gm_release_stream(s.stream);
  }
  (void)hipFree(s.d_idx);
  (void)hipFree(s.d_w);
  (void)hipFree(s.d_off);
  (void)hipFree(s.d_out_idx);
  (void)hipFree(s.d_out_val);
  (void)hipFree(s.d_ia);
  (void)hipFree(s.d_ib);
  (void)hipFree(s.d_jac);
  (void)hipHostFree(s.h_idx);
  (void)hipHostFree(s.h_w);
  (void)hipHostFree(s.h_off);
  (void)hipHostFree(s.h_ia);
  (void)hipHostFree(s.h_ib);
  (void)hipHostFree(s.h_jac);
  (void)hipHostFree(s.h_out_idx);
  (void)hipHostFree(s.h_out_val);
  if (s.done) (void)hipEventDestroy(s.done);
  if (s.stream) (void)hipStreamDestroy(s.stream);
  s = Slot();
}

}  // namespace

extern "C" gm_status gm_serve_run(const gm_serve_config* cfg, const gm_request* reqs,
                                  int64_t nreq, const int32_t* host_idx, const float* host_w,
                                  const int32_t* store_idx, int64_t nstore,
                                  int32_t* out_sketch_idx, double* out_sketch_val,
                                  double* out_jaccard, double* out_done_us,
                                  gm_serve_stats* stats) {
  if (!cfg || !reqs || nreq < 0 || !out_done_us || cfg->k < 1 || cfg->k > GM_K_MAX ||
      cfg->slots < 1 || cfg->slots > 64 || cfg->max_batch_requests < 1 ||
      cfg->max_batch_entries < 1 || cfg->device_budget_bytes < 1 || cfg->max_wait_us < 0)
    return GM_ERR_INVALID_ARG;
  const int32_t k = cfg->k;
  const int64_t E = cfg->max_batch_entries;
  const int64_t R = cfg->max_batch_requests;
  // validate the trace on the host (an error enqueues nothing)
  int64_t nsk = 0;
  for (int64_t r = 0; r < nreq; ++r) {
    const gm_request& q = reqs[r];
    if (q.kind == GM_REQ_SKETCH) {
      if (!host_idx || !host_w || q.a < 0 || q.b < q.a || q.b - q.a > E) return GM_ERR_INVALID_ARG;
      ++nsk;
    } else if (q.kind == GM_REQ_JACCARD) {
      if (!store_idx || !out_jaccard) return GM_ERR_INVALID_ARG;
    } else {
      return GM_ERR_INVALID_ARG;
    }
    if (r > 0 && q.arrival_us < reqs[r - 1].arrival_us) return GM_ERR_INVALID_ARG;
  }
  // position of each sketch request among the sketch requests (output row)
  std::vector<int64_t> sk_row(static_cast<size_t>(nreq), -1);
  {
    int64_t i = 0;
    for (int64_t r = 0; r < nreq; ++r)
      if (reqs[r].kind == GM_REQ_SKETCH) sk_row[r] = i++;
  }
  // One slot's device footprint, what the budget counts per batch in flight:
  // its staging buffers (entries, offsets, outputs, query pairs and answers)
  // and the library workspace its stream holds for sketch calls of up to R
  // vectors.  (LDS needs no admission: each launch sizes its grid to what the
  // CUs hold, and launches from several slots queue for the CUs.)
  int64_t ws_bytes = 0;
  {
    const gm_status g = gm_workspace_bytes(R, &ws_bytes);
    if (g != GM_OK) return g;
  }
  const int64_t slot_bytes =
      E * 8 + (R + 1) * 8 + R * k * 12 + R * (8 + 8 + 8) + ws_bytes;
  if (slot_bytes > cfg->device_budget_bytes) return GM_ERR_INVALID_ARG;  // not even one batch fits
  int nslots = cfg->slots;
  if (nslots * slot_bytes > cfg->device_budget_bytes)
    nslots = static_cast<int>(std::max<int64_t>(1, cfg->device_budget_bytes / slot_bytes));

  std::vector<Slot> slots(static_cast<size_t>(nslots));
  gm_status status = GM_OK;
  auto fail = [&](hipError_t e) {
    status = e == hipErrorOutOfMemory ? GM_ERR_OUT_OF_MEMORY : GM_ERR_DEVICE;
  };
  for (Slot& s : slots) {
    hipError_t e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&s.done, hipEventDisableTiming);
    if (e == hipSuccess) e = dalloc(&s.d_idx, E);
    if (e == hipSuccess) e = dalloc(&s.d_w, E);
    if (e == hipSuccess) e = dalloc(&s.d_off, R + 1);
    if (e == hipSuccess) e = dalloc(&s.d_out_idx, R * k);
    if (e == hipSuccess) e = dalloc(&s.d_out_val, R * k);
    if (e == hipSuccess) e = dalloc(&s.d_ia, R);
    if (e == hipSuccess) e = dalloc(&s.d_ib, R);
    if (e == hipSuccess) e = dalloc(&s.d_jac, R);
    if (e == hipSuccess) e = halloc(&s.h_idx, E);
    if (e == hipSuccess) e = halloc(&s.h_w, E);
    if (e == hipSuccess) e = halloc(&s.h_off, R + 1);
    if (e == hipSuccess) e = halloc(&s.h_ia, R);
    if (e == hipSuccess) e = halloc(&s.h_ib, R);
    if (e == hipSuccess) e = halloc(&s.h_jac, R);
    if (e == hipSuccess) e = halloc(&s.h_out_idx, R * k);
    if (e == hipSuccess) e = halloc(&s.h_out_val, R * k);
    if (e != hipSuccess) {
      fail(e);
      break;
    }
    // the slot stream's FastGM workspace, created outside the timed loop
    gm_status g = gm_reserve(R, s.stream);
    if (g != GM_OK) {
      status = g;
      break;
    }
  }
  if (status != GM_OK) {
    for (Slot& s : slots) free_slot(s);
    return status;
  }

  gm_serve_stats st;
  std::memset(&st, 0, sizeof(st));
  std::deque<int64_t> pending;
  int64_t next = 0, completed = 0, inflight_bytes = 0;
  const auto t0 = Clock::now();
  auto now_us = [&]() {
    return std::chrono::duration<double, std::micro>(Clock::now() - t0).count();
  };
  const bool realtime = cfg->realtime != 0;

  while (completed < nreq && status == GM_OK) {
    const double now = now_us();
    // arrivals
    while (next < nreq && (!realtime || reqs[next].arrival_us <= now)) pending.push_back(next++);
    // completions
    for (Slot& s : slots) {
      if (!s.busy) continue;
      const hipError_t q = hipEventQuery(s.done);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) {
        fail(q);
        break;
      }
      const double t = now_us();
      for (size_t i = 0; i < s.sk_reqs.size(); ++i) {
        const int64_t r = s.sk_reqs[i];
        out_done_us[r] = t;
        const int64_t row = sk_row[r];
        if (out_sketch_idx)
          std::memcpy(out_sketch_idx + row * k, s.h_out_idx + i * k, sizeof(int32_t) * k);
        if (out_sketch_val)
          std::memcpy(out_sketch_val + row * k, s.h_out_val + i * k, sizeof(double) * k);
      }
      for (size_t i = 0; i < s.jq_reqs.size(); ++i) {
        const int64_t r = s.jq_reqs[i];
        out_done_us[r] = t;
        out_jaccard[r] = s.h_jac[i];
      }
      completed += static_cast<int64_t>(s.sk_reqs.size() + s.jq_reqs.size());
      inflight_bytes -= s.bytes;
      s.busy = false;
    }
    if (status != GM_OK) break;
    // admission and launch
    bool launched = false;
    for (Slot& s : slots) {
      if (s.busy || pending.empty()) continue;
      const double oldest = realtime ? now - reqs[pending.front()].arrival_us : 0.0;
      int64_t pend_entries = 0;
      for (int64_t r : pending)
        if (reqs[r].kind == GM_REQ_SKETCH) pend_entries += reqs[r].b - reqs[r].a;
      const bool more_coming = next < nreq;
      const bool full = pend_entries >= E || static_cast<int64_t>(pending.size()) >= R;
      if (!full && more_coming && oldest < cfg->max_wait_us) break;  // keep batching
      if (inflight_bytes + slot_bytes > cfg->device_budget_bytes) break;  // memory budget
      s.sk_reqs.clear();
      s.jq_reqs.clear();
      int64_t ne = 0;
      while (!pending.empty() && static_cast<int64_t>(s.sk_reqs.size() + s.jq_reqs.size()) < R) {
        const int64_t r = pending.front();
        const gm_request& q = reqs[r];
        if (q.kind == GM_REQ_SKETCH) {
          const int64_t n = q.b - q.a;
          if (ne + n > E) break;  // the next batch takes it (FIFO)
          s.h_off[s.sk_reqs.size()] = ne;
          std::memcpy(s.h_idx + ne, host_idx + q.a, sizeof(int32_t) * n);
          std::memcpy(s.h_w + ne, host_w + q.a, sizeof(float) * n);
          ne += n;
          s.sk_reqs.push_back(r);
        } else {
          s.h_ia[s.jq_reqs.size()] = q.a;
          s.h_ib[s.jq_reqs.size()] = q.b;
          s.jq_reqs.push_back(r);
        }
        pending.pop_front();
      }
      const int64_t ns = static_cast<int64_t>(s.sk_reqs.size());
      const int64_t nj = static_cast<int64_t>(s.jq_reqs.size());
      hipError_t e = hipSuccess;
      if (ns > 0) {
        s.h_off[ns] = ne;
        e = hipMemcpyAsync(s.d_idx, s.h_idx, sizeof(int32_t) * ne, hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess)
          e = hipMemcpyAsync(s.d_w, s.h_w, sizeof(float) * ne, hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess)
          e = hipMemcpyAsync(s.d_off, s.h_off, sizeof(int64_t) * (ns + 1), hipMemcpyHostToDevice,
                             s.stream);
        if (e == hipSuccess) {
          const gm_status g = gm_sketch(s.d_idx, s.d_w, s.d_off, ns, k, cfg->seed, s.d_out_idx,
                                        s.d_out_val, s.stream);
          if (g != GM_OK) {
            status = g;
            break;
          }
        }
        if (e == hipSuccess && out_sketch_idx)
          e = hipMemcpyAsync(s.h_out_idx, s.d_out_idx, sizeof(int32_t) * ns * k,
                             hipMemcpyDeviceToHost, s.stream);
        if (e == hipSuccess && out_sketch_val)
          e = hipMemcpyAsync(s.h_out_val, s.d_out_val, sizeof(double) * ns * k,
                             hipMemcpyDeviceToHost, s.stream);
      }
      if (e == hipSuccess && nj > 0) {
        e = hipMemcpyAsync(s.d_ia, s.h_ia, sizeof(int64_t) * nj, hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess)
          e = hipMemcpyAsync(s.d_ib, s.h_ib, sizeof(int64_t) * nj, hipMemcpyHostToDevice, s.stream);
        if (e == hipSuccess) {
          const gm_status g =
              gm_jaccard_est_pairs(store_idx, nstore, k, s.d_ia, s.d_ib, nj, s.d_jac, s.stream);
          if (g != GM_OK) {
            status = g;
            break;
          }
        }
        if (e == hipSuccess)
          e = hipMemcpyAsync(s.h_jac, s.d_jac, sizeof(double) * nj, hipMemcpyDeviceToHost,
                             s.stream);
      }
      if (e == hipSuccess) e = hipEventRecord(s.done, s.stream);
      if (e != hipSuccess) {
        fail(e);
        break;
      }
      s.bytes = slot_bytes;
      inflight_bytes += slot_bytes;
      st.max_inflight_bytes = std::max<int64_t>(st.max_inflight_bytes, inflight_bytes);
      s.busy = true;
      launched = true;
      ++st.batches;
      st.sketch_requests += ns;
      st.jaccard_requests += nj;
      st.entries += ne;
      int busy = 0;
      for (const Slot& o : slots) busy += o.busy ? 1 : 0;
      st.max_slots_busy = std::max<int64_t>(st.max_slots_busy, busy);
    }
    if (!launched && status == GM_OK) {
      // nothing to launch: yield briefly until the next arrival or completion
      std::this_thread::yield();
    }
  }
  st.wall_us = now_us();
  st.slots = nslots;
  st.slot_bytes = slot_bytes;
  st.workspace_bytes = ws_bytes;
  for (Slot& s : slots) free_slot(s);
  if (stats) *stats = st;
  return status;
}
