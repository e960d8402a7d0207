"""Banding LSH over Gumbel-Max sketches -- CPU oracle (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module; the product library shares no code with
it.

Sec. 1 of the paper: a register s_j(v) of the sketch maps similar vectors to
the same element with probability J_P (the expected fraction of equal
registers), so the registers can key a locality-sensitive index for
sub-linear similarity search, in the way of the LSH schemes the paper cites.
The index bands the k registers: band b is registers b*rows .. b*rows+rows-1,
and a stored sketch is a candidate for a query when every index of at least
one band agrees.  An empty (-1) or poisoned (-2) register never agrees, as in
the Jaccard estimate.  With the registers independent, a pair at J_P = J is
a candidate with probability 1 - (1 - J^rows)^bands.

Written as the plain definition: exact tuples in a dictionary, no hashing.
"""
from __future__ import annotations

import numpy as np


def band_key(sketch_idx, b: int, rows: int):
    """The indices of band b as a tuple, or None when one is negative."""
    t = tuple(int(x) for x in sketch_idx[b * rows:(b + 1) * rows])
    return None if min(t) < 0 else t


def build(store, bands: int, rows: int):
    """For every band, a dictionary from band tuple to the stored rows with it."""
    store = np.asarray(store)
    assert bands * rows <= store.shape[1]
    tables = [dict() for _ in range(bands)]
    for i in range(store.shape[0]):
        for b in range(bands):
            key = band_key(store[i], b, rows)
            if key is not None:
                tables[b].setdefault(key, []).append(i)
    return tables


def candidates(store, queries, bands: int, rows: int, tables=None):
    """Sorted distinct candidate rows of the store for every query."""
    if tables is None:
        tables = build(store, bands, rows)
    out = []
    for q in np.asarray(queries):
        found = set()
        for b in range(bands):
            key = band_key(q, b, rows)
            if key is not None:
                found.update(tables[b].get(key, ()))
        out.append(np.array(sorted(found), dtype=np.int64))
    return out


def band_matches(store, query, bands: int, rows: int, tables=None) -> int:
    """Number of (band, stored row) agreements of one query, duplicates across
    bands counted."""
    if tables is None:
        tables = build(store, bands, rows)
    n = 0
    for b in range(bands):
        key = band_key(query, b, rows)
        if key is not None:
            n += len(tables[b].get(key, ()))
    return n


def collision_probability(J: float, bands: int, rows: int) -> float:
    """Probability that a pair at Jaccard J shares a band, registers independent."""
    return 1.0 - (1.0 - J ** rows) ** bands
