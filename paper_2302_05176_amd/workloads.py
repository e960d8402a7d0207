"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds input generation only (numpy PCG64 streams); none of the
sketch arithmetic lives here, so both the HIP path and the oracle can be fed
from it.  The paper's real datasets (document term vectors and rating
vectors, Table 1) are not available; these stand in for them:

* ``single``   one vector, n+ = 1000, weights Uniform(0,1] (the synthetic
               UNI(0,1) vectors of the Jaccard-task experiments, Sec. 4.1).
* ``batch``    sparse document-like vectors, n+ ~ lognormal(ln 500, 1)
               clipped to [10, 50000], indices distinct in [0, 2^20), weights
               Exp(1) (the EXP(1) variant of Sec. 4.1).
* ``pairs``    vector pairs sharing a chosen fraction of their support.
* ``stream``   one long vector with half Uniform(0,1] and half Pareto(1.5)
               weights (the weighted-cardinality task, Sec. 4.4).
* ``uneven``   very uneven batch: n+ ~ truncated Zipf(1.2) on [10, 1e5],
               per-vector k from {64, 256, 1024, 4096}, weights
               lognormal(0, 2).
* ``mixed``    small adversarial batches for parity tests (empty vectors,
               single elements, zero weights, duplicates, heavy elements).

All CSR arrays are (indices int32, weights float32, offsets int64).
"""
from __future__ import annotations

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def distinct_sorted(rng: np.random.Generator, n: int, dim: int) -> np.ndarray:
    """n distinct sorted integers drawn uniformly from [0, dim)."""
    if n > dim:
        raise ValueError("n > dim")
    if n * 4 > dim:
        return np.sort(rng.choice(dim, size=n, replace=False)).astype(np.int64)
    out = np.unique(rng.integers(0, dim, size=n + n // 8 + 8))
    while len(out) < n:
        out = np.unique(np.concatenate([out, rng.integers(0, dim, size=n - len(out) + 8)]))
    if len(out) > n:
        out = np.sort(rng.choice(out, size=n, replace=False))
    return out


def _pack(rows_idx, rows_w):
    lens = np.array([len(r) for r in rows_idx], np.int64)
    off = np.zeros(len(lens) + 1, np.int64)
    np.cumsum(lens, out=off[1:])
    idx = np.concatenate(rows_idx).astype(np.int32) if len(rows_idx) else np.zeros(0, np.int32)
    w = np.concatenate(rows_w).astype(np.float32) if len(rows_w) else np.zeros(0, np.float32)
    return idx, w, off


def exp1_weights(rng, n):
    w = rng.exponential(1.0, size=n).astype(np.float32)
    while True:
        bad = w <= 0
        if not bad.any():
            return w
        w[bad] = rng.exponential(1.0, size=int(bad.sum())).astype(np.float32)


def single(nplus: int = 1000, dim: int = 1 << 20, seed: int = 1001):
    """One vector, distinct sorted indices, weights float32(1 - U[0,1)) in (0, 1]."""
    rng = _rng(seed)
    idx = distinct_sorted(rng, nplus, dim)
    w = (1.0 - rng.random(nplus)).astype(np.float32)
    return _pack([idx], [w])


def batch_sizes(nvec: int, seed: int = 1002, mu: float = np.log(500.0), sigma: float = 1.0,
                lo: int = 10, hi: int = 50000) -> np.ndarray:
    rng = _rng(seed)
    n = np.rint(rng.lognormal(mu, sigma, size=nvec)).astype(np.int64)
    return np.clip(n, lo, hi)


def batch(nvec: int = 10000, dim: int = 1 << 20, seed: int = 1002, sizes=None):
    """Document-like batch: lognormal n+, distinct indices, Exp(1) weights."""
    if sizes is None:
        sizes = batch_sizes(nvec, seed)
    rng = _rng(seed + 7919)
    rows_i, rows_w = [], []
    for n in sizes:
        rows_i.append(distinct_sorted(rng, int(n), dim))
        rows_w.append(exp1_weights(rng, int(n)))
    return _pack(rows_i, rows_w)


def pairs(npairs: int = 5000, dim: int = 1 << 20, seed: int = 1012,
          fractions=(0.0, 0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9),
          equal_shared_weights: bool = False):
    """Vector pairs (a_p, b_p) as one CSR batch ordered a_0, b_0, a_1, b_1, ...

    Pair p shares round(f * min(n_a, n_b)) indices, f = fractions[p % len];
    the rest of each support is disjoint.  Returns (idx, w, off, f_per_pair).
    """
    rng = _rng(seed)
    sizes = batch_sizes(2 * npairs, seed + 1)
    rows_i, rows_w, fr = [], [], []
    for p in range(npairs):
        f = fractions[p % len(fractions)]
        na, nb = int(sizes[2 * p]), int(sizes[2 * p + 1])
        shared = int(round(f * min(na, nb)))
        pool = distinct_sorted(rng, na + nb - shared, dim)
        pool = rng.permutation(pool)
        sh = pool[:shared]
        a = np.sort(np.concatenate([sh, pool[shared:shared + na - shared]]))
        b = np.sort(np.concatenate([sh, pool[shared + na - shared:]]))
        wa = exp1_weights(rng, na)
        wb = exp1_weights(rng, nb)
        if equal_shared_weights and shared:
            ia = np.searchsorted(a, sh)
            ib = np.searchsorted(b, sh)
            wb[ib] = wa[ia]
        rows_i += [a, b]
        rows_w += [wa, wb]
        fr.append(f)
    idx, w, off = _pack(rows_i, rows_w)
    return idx, w, off, np.array(fr)


def stream(nplus: int = 10_000_000, dim: int = (1 << 31) - 1, seed: int = 1003):
    """One long vector: first half Uniform(0,1], second half 1 + Pareto(1.5)."""
    rng = _rng(seed)
    idx = distinct_sorted(rng, nplus, dim)
    h = nplus // 2
    w = np.empty(nplus, np.float32)
    w[:h] = (1.0 - rng.random(h)).astype(np.float32)
    w[h:] = (1.0 + rng.pareto(1.5, size=nplus - h)).astype(np.float32)
    return _pack([idx], [w])


def zipf_sizes(nvec: int, seed: int, s: float = 1.2, lo: int = 10, hi: int = 100000):
    """Truncated discrete Zipf: P(n) proportional to n^-s on [lo, hi]."""
    rng = _rng(seed)
    n = np.arange(lo, hi + 1, dtype=np.float64)
    p = n ** (-s)
    cdf = np.cumsum(p)
    cdf /= cdf[-1]
    return (lo + np.searchsorted(cdf, rng.random(nvec), side="right")).astype(np.int64)


def uneven(nvec: int = 100000, dim: int = 1 << 24, seed: int = 1004,
           ks=(64, 256, 1024, 4096), size_cap: int | None = None):
    """Uneven batch: Zipf(1.2) n+, per-vector k, lognormal(0, 2) weights.

    Returns (idx, w, off, k_per_vec int32)."""
    sizes = zipf_sizes(nvec, seed)
    if size_cap is not None:
        sizes = np.minimum(sizes, size_cap)
    rng = _rng(seed + 104729)
    kk = rng.choice(np.asarray(ks, np.int32), size=nvec)
    rows_i, rows_w = [], []
    for n in sizes:
        rows_i.append(distinct_sorted(rng, int(n), dim))
        w = rng.lognormal(0.0, 2.0, size=int(n)).astype(np.float32)
        w[w <= 0] = np.float32(1e-30)
        rows_w.append(w)
    idx, w, off = _pack(rows_i, rows_w)
    return idx, w, off, kk.astype(np.int32)


def mixed(seed: int = 7, nvec: int = 64, dim: int = 1 << 20, max_n: int = 3000):
    """Adversarial small batch for parity: empty rows, single elements, zero
    weights, duplicated entries, one dominant element, tiny and huge
    weights, unsorted indices."""
    rng = _rng(seed)
    rows_i, rows_w = [], []
    for v in range(nvec):
        kind = v % 8
        if kind == 0:
            n = 0
            i = np.zeros(0, np.int64)
            w = np.zeros(0, np.float32)
        elif kind == 1:
            i = distinct_sorted(rng, 1, dim)
            w = np.array([rng.exponential()], np.float32) + np.float32(1e-3)
        elif kind == 2:
            n = int(rng.integers(2, 40))
            i = distinct_sorted(rng, n, dim)
            w = exp1_weights(rng, n)
            w[rng.random(n) < 0.3] = 0.0
        elif kind == 3:
            n = int(rng.integers(5, 200))
            i = distinct_sorted(rng, n, dim)
            w = exp1_weights(rng, n)
            dup = rng.integers(0, n, size=max(1, n // 4))
            i = np.concatenate([i, i[dup]])
            w = np.concatenate([w, w[dup]])
        elif kind == 4:
            n = int(rng.integers(3, 100))
            i = distinct_sorted(rng, n, dim)
            w = exp1_weights(rng, n) * np.float32(1e-3)
            w[0] = np.float32(1e3)
        elif kind == 5:
            n = int(rng.integers(100, max_n))
            i = rng.permutation(distinct_sorted(rng, n, dim))
            w = rng.lognormal(0.0, 2.0, size=n).astype(np.float32)
        elif kind == 6:
            n = int(rng.integers(10, 500))
            i = distinct_sorted(rng, n, dim)
            w = (1.0 - rng.random(n)).astype(np.float32)
            w[: n // 2] *= np.float32(1e-30)
        else:
            n = int(rng.integers(500, max_n))
            i = distinct_sorted(rng, n, dim)
            w = exp1_weights(rng, n)
        rows_i.append(np.asarray(i, np.int64))
        rows_w.append(np.asarray(w, np.float32))
    return _pack(rows_i, rows_w)


def sites(idx, w, off, nsites: int = 3, seed: int = 1020, reweight: bool = False):
    """Spread every vector's entries over `nsites` overlapping sites: each entry
    goes to a random non-empty subset of them.  With `reweight` each copy gets
    its own weight (the entry's weight times a factor drawn from [0.25, 4)).

    Returns two CSR triples: the site vectors (rows v*nsites .. v*nsites +
    nsites - 1 belong to vector v) and the union vectors, which hold every
    index of v once with the largest weight any site gives it."""
    rng = _rng(seed)
    site_i, site_w, uni_i, uni_w = [], [], [], []
    for v in range(len(off) - 1):
        ii = np.asarray(idx[off[v]:off[v + 1]])
        ww = np.asarray(w[off[v]:off[v + 1]], np.float32)
        mask = rng.integers(1, 1 << nsites, size=len(ii))
        best = np.zeros(len(ii), np.float32)
        for p in range(nsites):
            sel = ((mask >> p) & 1) == 1
            wp = ww[sel]
            if reweight:
                wp = (wp * rng.uniform(0.25, 4.0, size=wp.size)).astype(np.float32)
            site_i.append(ii[sel])
            site_w.append(wp)
            best[sel] = np.maximum(best[sel], wp)
        uni_i.append(ii)
        uni_w.append(best)
    return _pack(site_i, site_w), _pack(uni_i, uni_w)
