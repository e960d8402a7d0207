"""Pins of the LSH oracle (oracle/lsh.py) against what the paper and the
mathematics fix, on sketches made by the C oracle.

* Sec. 1: a register of two sketches agrees with probability J_P, and the
  registers are independent (Eq. (1)-(2) with independent a_{i,j}; the FastGM
  form draws the same joint distribution, Sec. 2.2).  So a pair shares one of
  `bands` bands of `rows` registers with probability 1 - (1 - J_P^rows)^bands.
  A band of the wrong width, or overlapping bands, moves the rate by many
  standard errors.
* Special cases: equal sketches always collide; disjoint supports (J_P = 0)
  never; empty and poisoned registers never agree.
"""
import math

import numpy as np
import pytest

from oracle import lsh as L


def _pair(orc, rng, n=40, shared=30):
    ia = np.sort(rng.choice(1000, n, replace=False))
    ib = np.concatenate([ia[:shared], np.sort(rng.choice(np.arange(1000, 2000), n - shared,
                                                         replace=False))])
    wa = rng.exponential(size=n).astype(np.float32)
    wb = rng.exponential(size=n).astype(np.float32)
    wb[:shared] = wa[:shared]
    jp = orc.jp_sorted(ia, wa.astype(np.float64), ib, wb.astype(np.float64))
    idx = np.concatenate([ia, ib]).astype(np.int32)
    w = np.concatenate([wa, wb])
    off = np.array([0, n, 2 * n], np.int64)
    return idx, w, off, jp


@pytest.mark.parametrize("form", [0, 3])
def test_band_collision_rate_follows_s_curve(orc, form):
    rng = np.random.default_rng(21)
    idx, w, off, jp = _pair(orc, rng)
    assert 0.45 < jp < 0.65
    bands, rows, k = 8, 4, 32
    trials = 600
    hits = 0
    for seed in range(1, trials + 1):
        s, _ = orc.sketch(idx, w, off, k, seed, form=form)
        hits += len(L.candidates(s[:1], s[1:], bands, rows)[0]) == 1
    p = L.collision_probability(jp, bands, rows)
    se = math.sqrt(p * (1 - p) / trials)
    assert abs(hits / trials - p) < 4.5 * se
    # the test can tell a band one register wider or narrower
    for r2 in (rows - 1, rows + 1):
        assert abs(L.collision_probability(jp, bands, r2) - p) > 9 * se


def test_equal_and_disjoint_vectors(orc):
    rng = np.random.default_rng(22)
    ia = np.sort(rng.choice(500, 30, replace=False)).astype(np.int32)
    ib = (np.sort(rng.choice(500, 30, replace=False)) + 1000).astype(np.int32)
    wa = rng.exponential(size=30).astype(np.float32)
    idx = np.concatenate([ia, ia, ib]).astype(np.int32)
    w = np.concatenate([wa, wa * np.float32(4.0), wa])     # a scaled copy: J_P = 1
    off = np.array([0, 30, 60, 90], np.int64)
    for seed in range(1, 51):
        s, _ = orc.sketch(idx, w, off, 48, seed, form=3)
        c = L.candidates(s[:1], s[1:], 12, 4)
        assert list(c[0]) == [0]          # equal up to scale: every band agrees
        assert list(c[1]) == []           # disjoint: no register can agree
        assert L.band_matches(s[:1], s[1], 12, 4) == 12


def test_empty_and_poisoned_registers_never_agree():
    k, bands, rows = 16, 4, 4
    store = np.array([[-1] * k, [-2] * k, list(range(k)), [5] * 4 + [-1] * 12], np.int32)
    q = np.array([[-1] * k, [-2] * k, list(range(k)), [5] * 4 + [-1] * 12, [5] * k], np.int32)
    c = L.candidates(store, q, bands, rows)
    assert [list(x) for x in c] == [[], [], [2], [3], [3]]
    assert L.collision_probability(0.0, bands, rows) == 0.0
    assert L.collision_probability(1.0, bands, rows) == 1.0
