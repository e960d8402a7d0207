"""Serving driver: seeded request traces, a device sketch store, and the
native continuous-batching loop (gm_serve_run).

Trace (the serving workload): open-loop Poisson arrivals at `rate` requests
per second; one sketch request per four probability-Jaccard queries; a
sketch request carries a sparse vector with n+ ~ lognormal(ln 2000, 1.5)
clipped to [10, size_cap], distinct indices in [0, 2^24) and Exp(1) fp32
weights; a query names two rows of the device-resident store, uniform over
the store.  The store holds sketches of seeded small synthetic vectors.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _native
from . import workloads as W

REQ_DTYPE = np.dtype([("arrival_us", "<f8"), ("kind", "<i4"), ("pad", "<i4"),
                      ("a", "<i8"), ("b", "<i8")], align=True)
assert REQ_DTYPE.itemsize == 32

SKETCH, JACCARD = 0, 1


class ServeConfig(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("slots", ctypes.c_int32),
                ("max_batch_requests", ctypes.c_int32), ("realtime", ctypes.c_int32),
                ("max_batch_entries", ctypes.c_int64), ("device_budget_bytes", ctypes.c_int64),
                ("max_wait_us", ctypes.c_double), ("seed", ctypes.c_uint64)]


class ServeStats(ctypes.Structure):
    _fields_ = [("batches", ctypes.c_int64), ("sketch_requests", ctypes.c_int64),
                ("jaccard_requests", ctypes.c_int64), ("entries", ctypes.c_int64),
                ("max_inflight_bytes", ctypes.c_int64), ("max_slots_busy", ctypes.c_int64),
                ("slots", ctypes.c_int64), ("wall_us", ctypes.c_double),
                ("slot_bytes", ctypes.c_int64), ("workspace_bytes", ctypes.c_int64)]


def make_trace(nreq: int, rate: float, nstore: int, seed: int = 1005, sketch_every: int = 5,
               size_mu: float = float(np.log(2000.0)), size_sigma: float = 1.5,
               size_cap: int = 1_000_000, dim: int = 1 << 24):
    """Returns (reqs structured array, host_idx int32, host_w float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1e6 / rate, size=nreq)
    arrival = np.cumsum(gaps)
    kind = np.where(rng.random(nreq) < 1.0 / sketch_every, SKETCH, JACCARD).astype(np.int32)
    reqs = np.zeros(nreq, REQ_DTYPE)
    reqs["arrival_us"] = arrival
    reqs["kind"] = kind
    ns = int((kind == SKETCH).sum())
    sizes = np.clip(np.rint(rng.lognormal(size_mu, size_sigma, size=ns)), 10, size_cap).astype(np.int64)
    starts = np.zeros(ns + 1, np.int64)
    np.cumsum(sizes, out=starts[1:])
    idx = np.empty(int(starts[-1]), np.int32)
    w = np.empty(int(starts[-1]), np.float32)
    for i, n in enumerate(sizes):
        idx[starts[i]:starts[i + 1]] = W.distinct_sorted(rng, int(n), dim)
        w[starts[i]:starts[i + 1]] = W.exp1_weights(rng, int(n))
    si = np.nonzero(kind == SKETCH)[0]
    reqs["a"][si] = starts[:-1]
    reqs["b"][si] = starts[1:]
    ji = np.nonzero(kind == JACCARD)[0]
    reqs["a"][ji] = rng.integers(0, nstore, size=len(ji))
    reqs["b"][ji] = rng.integers(0, nstore, size=len(ji))
    return reqs, idx, w


def store_vectors(nstore: int, seed: int = 1006, nplus: int = 32, chunk: int = 200_000):
    """The store's seeded vectors, chunk by chunk: yields (first row, idx
    [m, nplus] int32, w [m, nplus] float32).  Indices are uniform in
    [0, 2^24) (a repeat inside a row is one element at its largest weight);
    weights are Exp(1) + 1e-6."""
    rng = np.random.Generator(np.random.PCG64(seed))
    for s0 in range(0, nstore, chunk):
        m = min(chunk, nstore - s0)
        idx = rng.integers(0, 1 << 24, size=(m, nplus), dtype=np.int64).astype(np.int32)
        w = rng.exponential(1.0, size=(m, nplus)).astype(np.float32) + np.float32(1e-6)
        yield s0, idx, w


def build_store(nstore: int, k: int, seed: int = 1006, nplus: int = 32, chunk: int = 200_000,
                device="cuda:0"):
    """Device [nstore, k] int32 store: FastGM sketches (sketch seed `seed`) of
    the vectors store_vectors(nstore, seed, nplus, chunk) yields."""
    import torch
    from . import sketch
    store = torch.empty((nstore, k), dtype=torch.int32, device=device)
    for s0, idx, w in store_vectors(nstore, seed, nplus, chunk):
        m = idx.shape[0]
        off = np.arange(m + 1, dtype=np.int64) * nplus
        t = lambda a: torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to(device)
        sketch(t(idx), t(w), t(off), k, seed, out_idx=store[s0:s0 + m])
    torch.cuda.synchronize()
    return store


def run(reqs, host_idx, host_w, store, k: int, seed: int = 1, slots: int = 8,
        max_batch_requests: int = 256, max_batch_entries: int | None = None,
        device_budget_bytes: int = 1 << 30, max_wait_us: float = 0.0, realtime: bool = True,
        want_sketches: bool = False):
    """Run the native loop; returns a dict of per-request arrays and stats.

    With max_wait_us = 0 a free slot takes whatever is pending at once; while
    every slot is busy, arrivals accumulate and the next free slot takes them
    as one batch.  A positive max_wait_us holds a partial batch until its
    oldest request has waited that long."""
    import torch
    L = _native.load()
    nreq = len(reqs)
    reqs = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
    sk = reqs["kind"] == SKETCH
    longest = int((reqs["b"][sk] - reqs["a"][sk]).max()) if sk.any() else 1
    if max_batch_entries is None:
        max_batch_entries = max(longest, 1 << 18)
    cfg = ServeConfig(k=k, slots=slots, max_batch_requests=max_batch_requests,
                      realtime=int(realtime), max_batch_entries=max_batch_entries,
                      device_budget_bytes=device_budget_bytes, max_wait_us=max_wait_us, seed=seed)
    hi = torch.from_numpy(np.ascontiguousarray(host_idx, np.int32)).pin_memory()
    hw = torch.from_numpy(np.ascontiguousarray(host_w, np.float32)).pin_memory()
    nsk = int(sk.sum())
    out_i = np.zeros((nsk, k), np.int32) if want_sketches else None
    out_v = np.zeros((nsk, k), np.float64) if want_sketches else None
    jac = np.full(nreq, np.nan)
    done = np.zeros(nreq)
    st = ServeStats()
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None else None
    torch.cuda.synchronize()
    rc = L.gm_serve_run(ctypes.byref(cfg), reqs.ctypes.data_as(ctypes.c_void_p), nreq,
                        ctypes.c_void_p(hi.data_ptr()), ctypes.c_void_p(hw.data_ptr()),
                        ctypes.c_void_p(store.data_ptr()), store.shape[0],
                        p(out_i), p(out_v), p(jac), p(done), ctypes.byref(st))
    _native.check(rc, "gm_serve_run")
    lat = done - reqs["arrival_us"] if realtime else done
    res = {"done_us": done, "latency_us": lat, "jaccard": jac,
           "stats": {f: getattr(st, f) for f, _ in st._fields_}}
    if want_sketches:
        res["sketch_idx"], res["sketch_val"] = out_i, out_v
    return res


def summarize(reqs, res) -> dict:
    lat = res["latency_us"]
    out = {"p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
           "throughput_req_s": len(reqs) / (res["stats"]["wall_us"] * 1e-6)}
    for name, kind in (("sketch", SKETCH), ("jaccard", JACCARD)):
        m = reqs["kind"] == kind
        if m.any():
            out[f"{name}_p50_us"] = float(np.percentile(lat[m], 50))
            out[f"{name}_p99_us"] = float(np.percentile(lat[m], 99))
    return out
