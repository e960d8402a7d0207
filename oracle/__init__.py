"""CPU oracle for the k-register Gumbel-Max sketch (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does; it
shares no code with it.  The arithmetic lives in ``gm_oracle.c`` (plain C,
fp64, compiled with contraction off); this module only marshals numpy arrays.
Each wrapped function names the passage of the paper it follows in the C
source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

FORM_PLAIN = 0      # Eq. (1)/(2) by definition, O(k n+)
FORM_FULL = 1       # FastGM form, every arrival (no pruning)
FORM_ALG1 = 2       # Algorithm 1 (FastSearch + FastPrune)
FORM_STREAM = 3     # Algorithm 2 (Stream-FastGM)


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (no GPU toolchain involved)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fno-fast-math",
            "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        u64, i32, i64, dbl, p = (ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64,
                                 ctypes.c_double, ctypes.c_void_p)
        L.gmo_sm64.argtypes, L.gmo_sm64.restype = [u64], u64
        L.gmo_unif.argtypes, L.gmo_unif.restype = [u64], dbl
        L.gmo_neglog.argtypes, L.gmo_neglog.restype = [dbl], dbl
        L.gmo_exp1.argtypes, L.gmo_exp1.restype = [u64], dbl
        L.gmo_prefix.argtypes, L.gmo_prefix.restype = [u64, i32], u64
        L.gmo_randint.argtypes, L.gmo_randint.restype = [u64, i32, i32], i32
        L.gmo_element_arrivals.argtypes = [u64, i32, ctypes.c_float, i32, p, p]
        L.gmo_element_arrivals.restype = None
        L.gmo_sketch.argtypes = [ctypes.c_int, p, p, p, i64, i32, u64, p, p, p]
        L.gmo_sketch.restype = ctypes.c_int
        L.gmo_needed_arrivals.argtypes = [p, p, p, i64, i32, u64, p, p]
        L.gmo_needed_arrivals.restype = None
        L.gmo_release_counts.argtypes = [p, i64, dbl, p]
        L.gmo_release_counts.restype = None
        L.gmo_jaccard.argtypes, L.gmo_jaccard.restype = [p, p, i32], dbl
        L.gmo_wcard.argtypes, L.gmo_wcard.restype = [p, i32], dbl
        L.gmo_merge.argtypes = [p, p, i64, i32, p, p]
        L.gmo_merge.restype = None
        L.gmo_setops.argtypes = [p, p, p, p, i32, p]
        L.gmo_setops.restype = None
        L.gmo_jp_brute.argtypes = [p, p, i64, p, p, i64]
        L.gmo_jp_brute.restype = dbl
        L.gmo_set_threads.argtypes, L.gmo_set_threads.restype = [ctypes.c_int], None
        L.gmo_get_threads.argtypes, L.gmo_get_threads.restype = [], ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def set_threads(n: int) -> None:
    lib().gmo_set_threads(int(n))


def get_threads() -> int:
    return int(lib().gmo_get_threads())


# -- draw specification ------------------------------------------------------

def sm64(z: int) -> int:
    return int(lib().gmo_sm64(ctypes.c_uint64(z & 0xFFFFFFFFFFFFFFFF)))


def unif(x: int) -> float:
    return float(lib().gmo_unif(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def neglog(u: float) -> float:
    return float(lib().gmo_neglog(float(u)))


def exp1(x: int) -> float:
    return float(lib().gmo_exp1(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def prefix(seed: int, index: int) -> int:
    return int(lib().gmo_prefix(ctypes.c_uint64(seed), int(index)))


def randint(x: int, z: int, k: int) -> int:
    return int(lib().gmo_randint(ctypes.c_uint64(x), int(z), int(k)))


def element_arrivals(seed: int, index: int, weight: float, k: int):
    """All k FastGM arrivals of one element: (times t_1..t_k, 0-based servers)."""
    t = np.empty(k, np.float64)
    c = np.empty(k, np.int32)
    lib().gmo_element_arrivals(ctypes.c_uint64(seed), int(index), float(weight), int(k),
                               _ptr(t), _ptr(c))
    return t, c


# -- sketches ----------------------------------------------------------------

def _csr(indices, weights, offsets):
    idx = np.ascontiguousarray(indices, dtype=np.int32)
    w = np.ascontiguousarray(weights, dtype=np.float32)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    return idx, w, off


def sketch(indices, weights, offsets, k: int, seed: int, form: int = FORM_STREAM,
           return_work: bool = False):
    """Sketch every CSR row; returns (s: int32[nvec,k], y: float64[nvec,k])."""
    idx, w, off = _csr(indices, weights, offsets)
    nvec = len(off) - 1
    s = np.empty((nvec, k), np.int32)
    y = np.empty((nvec, k), np.float64)
    work = np.zeros(max(nvec, 1), np.int64)
    rc = lib().gmo_sketch(int(form), _ptr(idx), _ptr(w), _ptr(off), nvec, int(k),
                          ctypes.c_uint64(seed), _ptr(s), _ptr(y), _ptr(work))
    if rc != 0:
        raise ValueError("oracle rejected arguments")
    if return_work:
        return s, y, work[:nvec]
    return s, y


def needed_arrivals(indices, weights, offsets, k: int, seed: int, y) -> np.ndarray:
    """A*: arrivals any exact pruned FastGM run must emit, per vector."""
    idx, w, off = _csr(indices, weights, offsets)
    nvec = len(off) - 1
    yy = np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros(max(nvec, 1), np.int64)
    lib().gmo_needed_arrivals(_ptr(idx), _ptr(w), _ptr(off), nvec, int(k),
                              ctypes.c_uint64(seed), _ptr(yy), _ptr(out))
    return out[:nvec]


def release_counts(v, R: float) -> np.ndarray:
    vv = np.ascontiguousarray(v, dtype=np.float64)
    out = np.empty(len(vv), np.int64)
    lib().gmo_release_counts(_ptr(vv), len(vv), float(R), _ptr(out))
    return out


# -- estimators --------------------------------------------------------------

def jaccard(a, b) -> float:
    aa = np.ascontiguousarray(a, dtype=np.int32)
    bb = np.ascontiguousarray(b, dtype=np.int32)
    return float(lib().gmo_jaccard(_ptr(aa), _ptr(bb), len(aa)))


def wcard(y) -> float:
    yy = np.ascontiguousarray(y, dtype=np.float64)
    return float(lib().gmo_wcard(_ptr(yy), len(yy)))


def merge(s, y):
    """Sketch of a union from r sketches of its parts (Sec. 2.3): arrays of
    shape (r, k); returns (s, y) of shape (k,)."""
    ss = np.ascontiguousarray(s, dtype=np.int32)
    yy = np.ascontiguousarray(y, dtype=np.float64)
    r, k = ss.shape
    so = np.empty(k, np.int32)
    yo = np.empty(k, np.float64)
    lib().gmo_merge(_ptr(ss), _ptr(yy), r, k, _ptr(so), _ptr(yo))
    return so, yo


SETOPS = ("union", "intersection", "a_minus_b", "b_minus_a", "jaccard_w")


def setops(sa, ya, sb, yb) -> np.ndarray:
    """Weighted cardinalities of two sets from their sketches (k registers
    each): [union, intersection, |A\\B|, |B\\A|, J_W] (see gmo_setops)."""
    sa = np.ascontiguousarray(sa, dtype=np.int32)
    sb = np.ascontiguousarray(sb, dtype=np.int32)
    ya = np.ascontiguousarray(ya, dtype=np.float64)
    yb = np.ascontiguousarray(yb, dtype=np.float64)
    out = np.empty(5, np.float64)
    lib().gmo_setops(_ptr(sa), _ptr(ya), _ptr(sb), _ptr(yb), len(sa), _ptr(out))
    return out


def jp_brute(ia, wa, ib, wb) -> float:
    ia = np.ascontiguousarray(ia, dtype=np.int32)
    ib = np.ascontiguousarray(ib, dtype=np.int32)
    wa = np.ascontiguousarray(wa, dtype=np.float64)
    wb = np.ascontiguousarray(wb, dtype=np.float64)
    return float(lib().gmo_jp_brute(_ptr(ia), _ptr(wa), len(ia), _ptr(ib), _ptr(wb), len(ib)))


def jp_sorted(ia, wa, ib, wb) -> float:
    """J_P in O(n log n): for i in both supports, sum_l max(u_l/u_i, v_l/v_i)
    splits at the ratio u_l/v_l = u_i/v_i, so sort the union by u/v and use
    prefix sums (Sec. 1 closed form, rearranged)."""
    ia = np.asarray(ia, np.int64)
    ib = np.asarray(ib, np.int64)
    wa = np.asarray(wa, np.float64)
    wb = np.asarray(wb, np.float64)
    keys = np.union1d(ia[wa > 0], ib[wb > 0])
    u = np.zeros(len(keys))
    v = np.zeros(len(keys))
    u[np.searchsorted(keys, ia[wa > 0])] = wa[wa > 0]
    v[np.searchsorted(keys, ib[wb > 0])] = wb[wb > 0]
    # ratio u/v in [0, inf]; l with u_l/u_i >= v_l/v_i  <=>  u_l/v_l >= u_i/v_i
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(v > 0, u / np.where(v > 0, v, 1.0), np.inf)
    order = np.argsort(ratio, kind="stable")
    rs, us, vs = ratio[order], u[order], v[order]
    # suffix sums of u over ratio >= r, prefix sums of v over ratio < r
    su = np.concatenate([np.cumsum(us[::-1])[::-1], [0.0]])
    pv = np.concatenate([[0.0], np.cumsum(vs)])
    jp = 0.0
    for p in range(len(rs)):
        if us[p] > 0 and vs[p] > 0:
            first = np.searchsorted(rs, rs[p], side="left")
            den = su[first] / us[p] + pv[first] / vs[p]
            jp += 1.0 / den
    return jp
