"""MI355X-native k-register Gumbel-Max sketch (FastGM and plain forms).

Thin Python binding of libgm.so: every function marshals torch device
tensors into the C ABI of ``include/gm.h`` and launches on the current torch
stream.  All arithmetic happens in the HIP kernels; there is no CPU
fallback, and a missing library raises ImportError on first use.

    import torch, paper_2302_05176_amd as gm
    s, y = gm.sketch(indices, weights, offsets, k=256, seed=1)   # FastGM form
    s0, y0 = gm.sketch(indices, weights, offsets, k=256, seed=1, form="plain")
    J = gm.jaccard_est(s[0::2], s[1::2])                           # Sec. 1, Theorem 1
    c = gm.wcard_est(y)                                            # Sec. 1, Theorem 2
"""
from __future__ import annotations

import ctypes

from . import _native
from ._native import GM_K_MAX, GMError  # noqa: F401

__all__ = ["sketch", "sketch_batched", "reserve", "autotune", "jaccard_est", "jaccard_est_pairs", "wcard_est",
           "merge", "setops", "get_data_errors", "reset_data_errors", "set_option", "release",
           "GMError", "GM_K_MAX", "library_path"]

_FORMS = {"fastgm": _native.GM_FORM_FASTGM, "plain": _native.GM_FORM_PLAIN}


def library_path() -> str:
    return _native.path()


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def sketch(indices, weights, offsets, k: int, seed: int, form: str = "fastgm",
           out_idx=None, out_val=None, stream=None):
    """Sketch CSR rows (int32 indices, fp32 weights, int64 offsets).

    Returns (s, y): int32 [nvec, k] register indices and fp64 [nvec, k] keys.
    """
    torch = _torch()
    L = _native.load()
    nvec = offsets.numel() - 1
    dev = offsets.device
    if out_idx is None:
        out_idx = torch.empty((max(nvec, 0), k), dtype=torch.int32, device=dev)
    if out_val is None:
        out_val = torch.empty((max(nvec, 0), k), dtype=torch.float64, device=dev)
    fn = L.gm_sketch if _FORMS[form] == _native.GM_FORM_FASTGM else L.gm_sketch_plain
    st = fn(_dev(indices, torch.int32, "indices"), _dev(weights, torch.float32, "weights"),
            _dev(offsets, torch.int64, "offsets"), nvec, int(k), ctypes.c_uint64(seed),
            _dev(out_idx, torch.int32, "out_idx"), _dev(out_val, torch.float64, "out_val"),
            _stream(stream))
    _native.check(st, "gm_sketch" if form == "fastgm" else "gm_sketch_plain")
    return out_idx, out_val


def empty_sketches(nvec: int, k: int, device=None):
    """Rows of empty registers (-1, +inf): the sketch of no entries."""
    torch = _torch()
    device = device or torch.device("cuda", torch.cuda.current_device())
    return (torch.full((nvec, k), -1, dtype=torch.int32, device=device),
            torch.full((nvec, k), float("inf"), dtype=torch.float64, device=device))


def sketch_update(indices, weights, offsets, k: int, seed: int, sk_idx, sk_val, stream=None):
    """Merge each row's new entries into its stored FastGM sketch in place
    (gm_sketch_update); sk_idx/sk_val are int32/fp64 [nvec, k] device tensors."""
    torch = _torch()
    L = _native.load()
    nvec = offsets.numel() - 1
    st = L.gm_sketch_update(_dev(indices, torch.int32, "indices"),
                            _dev(weights, torch.float32, "weights"),
                            _dev(offsets, torch.int64, "offsets"), nvec, int(k),
                            ctypes.c_uint64(seed), _dev(sk_idx, torch.int32, "sk_idx"),
                            _dev(sk_val, torch.float64, "sk_val"), _stream(stream))
    _native.check(st, "gm_sketch_update")
    return sk_idx, sk_val


def sketch_batched(indices, weights, offsets, k_per_vec, out_offsets, k_max: int, seed: int,
                   form: str = "fastgm", out_idx=None, out_val=None, stream=None):
    """Vectors with individual k; registers of vector v fill
    out[out_offsets[v] : out_offsets[v] + k_per_vec[v]] (flat arrays)."""
    torch = _torch()
    L = _native.load()
    nvec = offsets.numel() - 1
    dev = offsets.device
    if out_idx is None or out_val is None:
        # sizing the outputs reads the device (a sync): pass them when capturing
        total = int(out_offsets[-1].item()) if nvec > 0 else 0
        if out_idx is None:
            out_idx = torch.empty(total, dtype=torch.int32, device=dev)
        if out_val is None:
            out_val = torch.empty(total, dtype=torch.float64, device=dev)
    st = L.gm_sketch_batched(
        _dev(indices, torch.int32, "indices"), _dev(weights, torch.float32, "weights"),
        _dev(offsets, torch.int64, "offsets"), nvec, _dev(k_per_vec, torch.int32, "k_per_vec"),
        _dev(out_offsets, torch.int64, "out_offsets"), int(k_max), ctypes.c_uint64(seed),
        _FORMS[form], _dev(out_idx, torch.int32, "out_idx"),
        _dev(out_val, torch.float64, "out_val"), _stream(stream))
    _native.check(st, "gm_sketch_batched")
    return out_idx, out_val


def jaccard_est(a, b, out=None, stream=None):
    """Row-wise probability-Jaccard estimates of two [npairs, k] index sketches."""
    torch = _torch()
    L = _native.load()
    npairs, k = a.shape
    if b.shape != a.shape:
        raise ValueError("sketch shapes differ")
    if out is None:
        out = torch.empty(npairs, dtype=torch.float64, device=a.device)
    st = L.gm_jaccard_est(_dev(a, torch.int32, "a"), _dev(b, torch.int32, "b"), npairs, k,
                          _dev(out, torch.float64, "out"), _stream(stream))
    _native.check(st, "gm_jaccard_est")
    return out


def jaccard_est_pairs(store, ia, ib, out=None, stream=None):
    """Estimates for row pairs (ia[p], ib[p]) of a [nstore, k] device store."""
    torch = _torch()
    L = _native.load()
    nstore, k = store.shape
    npairs = ia.numel()
    if out is None:
        out = torch.empty(npairs, dtype=torch.float64, device=store.device)
    st = L.gm_jaccard_est_pairs(_dev(store, torch.int32, "store"), nstore, k,
                                _dev(ia, torch.int64, "ia"), _dev(ib, torch.int64, "ib"), npairs,
                                _dev(out, torch.float64, "out"), _stream(stream))
    _native.check(st, "gm_jaccard_est_pairs")
    return out


def wcard_est(val, out=None, stream=None):
    """Weighted-cardinality estimates (k-1)/sum_j y_j of [nvec, k] value sketches."""
    torch = _torch()
    L = _native.load()
    nvec, k = val.shape
    if out is None:
        out = torch.empty(nvec, dtype=torch.float64, device=val.device)
    st = L.gm_wcard_est(_dev(val, torch.float64, "val"), nvec, k,
                        _dev(out, torch.float64, "out"), _stream(stream))
    _native.check(st, "gm_wcard_est")
    return out


def merge(idx, val, stream=None):
    """Union sketch of r sketches ([r, k] idx and val) by registerwise lexicographic min."""
    torch = _torch()
    L = _native.load()
    r, k = idx.shape
    oi = torch.empty(k, dtype=torch.int32, device=idx.device)
    ov = torch.empty(k, dtype=torch.float64, device=idx.device)
    st = L.gm_merge(_dev(idx, torch.int32, "idx"), _dev(val, torch.float64, "val"), r, k,
                    _dev(oi, torch.int32, "out_idx"), _dev(ov, torch.float64, "out_val"),
                    _stream(stream))
    _native.check(st, "gm_merge")
    return oi, ov


SETOPS = ("union", "intersection", "a_minus_b", "b_minus_a", "jaccard_w")


def setops(idx_a, val_a, idx_b, val_b, out=None, stream=None):
    """Weighted cardinalities of set pairs from their [npairs, k] sketches
    (gm_setops): returns fp64 [npairs, 5] = union, intersection, A minus B,
    B minus A, weighted Jaccard (columns named in SETOPS)."""
    torch = _torch()
    L = _native.load()
    npairs, k = idx_a.shape
    for t in (val_a, idx_b, val_b):
        if tuple(t.shape) != (npairs, k):
            raise ValueError("sketch shapes differ")
    if out is None:
        out = torch.empty((npairs, 5), dtype=torch.float64, device=idx_a.device)
    st = L.gm_setops(_dev(idx_a, torch.int32, "idx_a"), _dev(val_a, torch.float64, "val_a"),
                     _dev(idx_b, torch.int32, "idx_b"), _dev(val_b, torch.float64, "val_b"),
                     npairs, k, _dev(out, torch.float64, "out"), _stream(stream))
    _native.check(st, "gm_setops")
    return out


class LshIndex:
    """Banding LSH index over a device sketch store (gm_lsh_build): band b is
    registers b*rows .. b*rows+rows-1; a stored row is a candidate for a query
    when some band's indices are all equal and non-negative.  Holds a
    reference to the store, which queries read."""

    def __init__(self, store, bands: int, rows: int, stream=None):
        torch = _torch()
        L = _native.load()
        nstore, k = store.shape
        h = ctypes.c_void_p()
        st = L.gm_lsh_build(_dev(store, torch.int32, "store"), nstore, k, bands, rows,
                            ctypes.byref(h), _stream(stream))
        _native.check(st, "gm_lsh_build")
        self._h = h
        self.store = store
        self.k, self.bands, self.rows = k, bands, rows

    def query(self, queries, max_cand: int = 64, stream=None):
        """Candidates of [nq, k] query sketches: (cand [nq, max_cand] int32, the
        smallest candidate rows in ascending order; count [nq] int32, the number
        of distinct candidates, -1 past 2048 band matches)."""
        torch = _torch()
        L = _native.load()
        nq = queries.shape[0]
        if queries.shape[1] != self.k:
            raise ValueError("queries must have the index's k registers")
        cand = torch.full((nq, max(max_cand, 1)), -1, dtype=torch.int32, device=queries.device)
        count = torch.empty(nq, dtype=torch.int32, device=queries.device)
        st = L.gm_lsh_query(self._h, _dev(queries, torch.int32, "queries"), nq, max_cand,
                            _dev(cand, torch.int32, "cand"), _dev(count, torch.int32, "count"),
                            _stream(stream))
        _native.check(st, "gm_lsh_query")
        return cand[:, :max_cand], count

    def close(self):
        if self._h:
            _native.load().gm_lsh_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rate_probe(what: str, lanes: int, steps: int, seed: int = 1, out=None, stream=None):
    """Issue-rate probe (gm_rate_probe): `lanes` lanes each draw `steps` FastGM
    arrivals (what="arrivals") or plain keys (what="keys"); returns the
    per-lane results (fp64, on the current device)."""
    torch = _torch()
    L = _native.load()
    if out is None:
        out = torch.empty(lanes, dtype=torch.float64, device=torch.device("cuda", torch.cuda.current_device()))
    st = L.gm_rate_probe({"arrivals": 0, "keys": 1}[what], lanes, steps, seed,
                         _dev(out, torch.float64, "out"), _stream(stream))
    _native.check(st, "gm_rate_probe")
    return out


def autotune(indices, weights, offsets, k_max: int, seed: int, k_per_vec=None, out_offsets=None,
             out_idx=None, out_val=None, reps: int = 3, use_cache: bool = True, stream=None) -> dict:
    """Time this batch under the FastGM schedule options, apply the fastest
    (process-wide) and return it (gm_autotune; outputs are overwritten)."""
    torch = _torch()
    L = _native.load()
    nvec = offsets.numel() - 1
    dev = offsets.device
    batched = k_per_vec is not None
    if out_idx is None or out_val is None:
        total = int(out_offsets[-1].item()) if batched else nvec * k_max
        out_idx = torch.empty(total, dtype=torch.int32, device=dev)
        out_val = torch.empty(total, dtype=torch.float64, device=dev)
    res = _native.TuneResult()
    st = L.gm_autotune(_dev(indices, torch.int32, "indices"), _dev(weights, torch.float32, "weights"),
                       _dev(offsets, torch.int64, "offsets"), nvec,
                       _dev(k_per_vec, torch.int32, "k_per_vec") if batched else None,
                       _dev(out_offsets, torch.int64, "out_offsets") if batched else None,
                       int(k_max), ctypes.c_uint64(seed), _dev(out_idx, torch.int32, "out_idx"),
                       _dev(out_val, torch.float64, "out_val"), int(reps), int(bool(use_cache)),
                       ctypes.byref(res), _stream(stream))
    _native.check(st, "gm_autotune")
    return {f: getattr(res, f) for f, _ in res._fields_}


def reserve(nvec: int, stream=None) -> None:
    """Create the FastGM workspace for `stream` up front (before graph capture)."""
    _native.check(_native.load().gm_reserve(int(nvec), _stream(stream)), "gm_reserve")


def workspace_bytes(nvec: int) -> int:
    """Device bytes of one stream's library workspace for calls of up to nvec
    vectors (gm_workspace_bytes)."""
    n = ctypes.c_int64(0)
    _native.check(_native.load().gm_workspace_bytes(int(nvec), ctypes.byref(n)), "gm_workspace_bytes")
    return int(n.value)


def get_data_errors(stream=None) -> int:
    L = _native.load()
    n = ctypes.c_int64(0)
    _native.check(L.gm_get_data_errors(ctypes.byref(n), _stream(stream)), "gm_get_data_errors")
    return int(n.value)


def reset_data_errors(stream=None) -> None:
    L = _native.load()
    _native.check(L.gm_reset_data_errors(_stream(stream)), "gm_reset_data_errors")


def set_option(name: str, value: int) -> None:
    """Tuning/testing knobs of gm_set_option: pos_bits, t0_scale_ppm, map_load, republish,
    stats, seg_rest."""
    L = _native.load()
    _native.check(L.gm_set_option(_native.OPTIONS[name], int(value)), f"gm_set_option({name})")


def get_stats(stream=None) -> dict:
    """FastGM work counters accumulated while set_option("stats", 1) was on."""
    L = _native.load()
    n = len(_native.STATS)
    buf = (ctypes.c_int64 * n)()
    _native.check(L.gm_get_stats(buf, n, _stream(stream)), "gm_get_stats")
    return dict(zip(_native.STATS, list(buf)))


def get_timing() -> dict:
    """Per-kernel HIP-event totals of launches made while set_option("timing", 1 or 2):
    {kernel name: (total ms, launches)}."""
    L = _native.load()
    n = 64
    names = (ctypes.c_char * 64 * n)()
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    m = L.gm_get_timing(n, names, ms, cnt)
    return {bytes(names[i]).split(b"\0")[0].decode(): (ms[i], cnt[i]) for i in range(max(m, 0))}


def reset_timing() -> None:
    _native.load().gm_reset_timing()


def reset_stats(stream=None) -> None:
    _native.check(_native.load().gm_reset_stats(_stream(stream)), "gm_reset_stats")


def reset_options() -> None:
    for name, v in (("pos_bits", 31), ("t0_scale_ppm", 1_000_000), ("map_load", 14),
                    ("republish", 8), ("stats", 0), ("seg_rest", 12),
                    ("small_waves", 0), ("timing", 0), ("wave_lim", 8191)):
        set_option(name, v)


def release() -> None:
    _native.load().gm_release()
