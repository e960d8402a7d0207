"""Oracle self-consistency: the FastGM forms agree, and the invariances the
paper states hold bit-exactly.

* Pruning never changes the sketch (Sec. 1 queue model, Sec. 2.2 FastPrune):
  the unpruned FastGM form == Algorithm 1 == Algorithm 2, bit for bit.
* A non-negative vector and its rescaling have the same sketch (Sec. 2.5):
  scaling by 2^m keeps indices and scales values by exactly 2^-m.
* Mergeability (Sec. 2.3): sketch(A u B) == registerwise lexicographic min
  of sketch(A) and sketch(B), for disjoint parts and for sites whose sets
  overlap.  An element's arrivals and permutation depend on its index only
  and its keys fall as its weight grows, so when sites give one element
  different weights the merge is the sketch of the largest.
* Entry order and duplicated stream elements do not matter (Sec. 3).
* The plain form's register j depends on (i, j) only, so a k-register plain
  sketch is the prefix of a larger one.
* A single element fills every register once: its k arrivals visit each
  server exactly once (Fisher-Yates permutation, Sec. 2.2).
"""
import numpy as np
import pytest

from paper_2302_05176_amd import workloads as W

FORMS_FAST = (1, 2, 3)


def _bits(y):
    return np.ascontiguousarray(y).view(np.uint64)


def _same(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(_bits(a[1]), _bits(b[1]))


@pytest.mark.parametrize("k", [1, 2, 3, 7, 8, 64, 256])
def test_fastgm_forms_agree(orc, k):
    idx, w, off = W.mixed(seed=100 + k, nvec=40, max_n=1500 if k < 256 else 600)
    res = [orc.sketch(idx, w, off, k, 1234 + k, form=f) for f in FORMS_FAST]
    assert _same(res[0], res[1])
    assert _same(res[0], res[2])


def test_fastgm_forms_agree_heavy_single_and_sizes(orc):
    rows_i, rows_w = [], []
    rng = np.random.default_rng(3)
    for n in [1, 2, 3, 5, 17, 100, 2000]:
        rows_i.append(np.sort(rng.choice(1 << 20, n, replace=False)))
        w = rng.exponential(size=n).astype(np.float32) + np.float32(1e-6)
        w[0] = 50.0 * w.sum()          # one dominant element walks most of its queue
        rows_w.append(w)
    idx, w, off = W._pack(rows_i, rows_w)
    for k in (8, 64, 512):
        res = [orc.sketch(idx, w, off, k, 9, form=f) for f in FORMS_FAST]
        assert _same(res[0], res[1]) and _same(res[0], res[2])


def test_pruned_forms_emit_at_least_needed_arrivals(orc):
    idx, w, off = W.batch(nvec=60, seed=33)
    k = 128
    s, y, full = orc.sketch(idx, w, off, k, 5, form=1, return_work=True)
    need = orc.needed_arrivals(idx, w, off, k, 5, y)
    _, _, a1 = orc.sketch(idx, w, off, k, 5, form=2, return_work=True)
    _, _, a2 = orc.sketch(idx, w, off, k, 5, form=3, return_work=True)
    assert np.all(a1 >= need) and np.all(a2 >= need)
    assert np.all(full == k * np.diff(off))
    assert np.all(need < full)


def test_empty_zero_and_poisoned_vectors(orc):
    idx = np.array([5, 6, 7, 8, 9, 10, 11], np.int32)
    w = np.array([0, 0, 1.0, np.nan, 2.0, -1.0, np.inf], np.float32)
    off = np.array([0, 0, 2, 3, 4, 5, 6, 7], np.int64)
    for form in (0, 1, 2, 3):
        s, y = orc.sketch(idx, w, off, 16, 1, form=form)
        assert np.all(s[0] == -1) and np.all(np.isinf(y[0]))     # empty row
        assert np.all(s[1] == -1) and np.all(np.isinf(y[1]))     # zero weights only
        assert np.all(s[2] == 7) and np.all(np.isfinite(y[2]))   # one element fills all
        for r in (3, 5, 6):                                      # NaN, negative, inf weight
            assert np.all(s[r] == -2) and np.all(np.isnan(y[r]))
        assert np.all(s[4] == 9)
    # negative index poisons
    s, y = orc.sketch(np.array([-3], np.int32), np.array([1.0], np.float32),
                      np.array([0, 1], np.int64), 4, 1, form=3)
    assert np.all(s == -2)


@pytest.mark.parametrize("form", [0, 1])
def test_power_of_two_scaling(orc, form):
    idx, w, off = W.mixed(seed=21, nvec=24, max_n=800)
    k = 64
    s0, y0 = orc.sketch(idx, w, off, k, 77, form=form)
    for m in (-3, 5):
        s1, y1 = orc.sketch(idx, w * np.float32(2.0 ** m), off, k, 77, form=form)
        assert np.array_equal(s0, s1)
        fin = np.isfinite(y0)
        assert np.array_equal(_bits(y1[fin]), _bits(y0[fin] * 2.0 ** -m))


@pytest.mark.parametrize("form", [0, 3])
def test_split_and_merge(orc, form):
    idx, w, off = W.batch(nvec=8, seed=41)
    k = 128
    s, y = orc.sketch(idx, w, off, k, 3, form=form)
    # split each vector into 3 interleaved parts, sketch separately, merge
    rows_i, rows_w = [], []
    for v in range(8):
        a, b = off[v], off[v + 1]
        for part in range(3):
            rows_i.append(idx[a:b][part::3])
            rows_w.append(w[a:b][part::3])
    pi, pw, po = W._pack(rows_i, rows_w)
    ps, py = orc.sketch(pi, pw, po, k, 3, form=form)
    ps = ps.reshape(8, 3, k)
    py = py.reshape(8, 3, k)
    ms = ps[:, 0].copy()
    my = py[:, 0].copy()
    for part in (1, 2):
        better = (py[:, part] < my) | ((py[:, part] == my) & (ps[:, part] < ms))
        my = np.where(better, py[:, part], my)
        ms = np.where(better, ps[:, part], ms)
    assert np.array_equal(ms, s)
    assert np.array_equal(_bits(my), _bits(y))


def _merge_rows(s, y, nsites):
    """Registerwise lexicographic (value, index) min over each group of rows."""
    k = s.shape[1]
    s = s.reshape(-1, nsites, k)
    y = y.reshape(-1, nsites, k)
    ms, my = s[:, 0].copy(), y[:, 0].copy()
    for p in range(1, nsites):
        better = (y[:, p] < my) | ((y[:, p] == my) & (s[:, p] < ms))
        my = np.where(better, y[:, p], my)
        ms = np.where(better, s[:, p], ms)
    return ms, my


@pytest.mark.parametrize("reweight", [False, True])
@pytest.mark.parametrize("form", [0, 3])
def test_merge_of_overlapping_sites(orc, form, reweight):
    idx, w, off = W.batch(nvec=10, seed=43)
    (si, sw, so), (ui, uw, uo) = W.sites(idx, w, off, nsites=3, seed=44, reweight=reweight)
    k = 64
    union = orc.sketch(ui, uw, uo, k, 12, form=form)
    merged = _merge_rows(*orc.sketch(si, sw, so, k, 12, form=form), 3)
    assert _same(merged, union)
    if not reweight:
        assert _same(union, orc.sketch(idx, w, off, k, 12, form=form))


@pytest.mark.parametrize("form", [0, 1, 3])
def test_order_and_duplicate_invariance(orc, form):
    idx, w, off = W.batch(nvec=6, seed=55)
    k = 64
    s, y = orc.sketch(idx, w, off, k, 8, form=form)
    rng = np.random.default_rng(0)
    rows_i, rows_w = [], []
    for v in range(6):
        a, b = off[v], off[v + 1]
        ii, ww = idx[a:b], w[a:b]
        dup = rng.integers(0, b - a, size=(b - a) // 3)
        ii = np.concatenate([ii, ii[dup]])
        ww = np.concatenate([ww, ww[dup]])
        perm = rng.permutation(len(ii))
        rows_i.append(ii[perm])
        rows_w.append(ww[perm])
    pi, pw, po = W._pack(rows_i, rows_w)
    s2, y2 = orc.sketch(pi, pw, po, k, 8, form=form)
    assert np.array_equal(s, s2) and np.array_equal(_bits(y), _bits(y2))


def test_plain_prefix_property(orc):
    idx, w, off = W.batch(nvec=5, seed=66)
    s1, y1 = orc.sketch(idx, w, off, 256, 4, form=0)
    s2, y2 = orc.sketch(idx, w, off, 64, 4, form=0)
    assert np.array_equal(s1[:, :64], s2)
    assert np.array_equal(_bits(y1[:, :64]), _bits(y2))


@pytest.mark.parametrize("k", [1, 5, 64, 1000])
def test_single_element_visits_every_server_once(orc, k):
    t, c = orc.element_arrivals(99, 123456, 0.37, k)
    assert np.array_equal(np.sort(c), np.arange(k))
    assert np.all(np.diff(t) >= 0)                      # ascending arrival times
    idx = np.array([123456], np.int32)
    w = np.array([0.37], np.float32)
    off = np.array([0, 1], np.int64)
    for form in FORMS_FAST:
        s, y = orc.sketch(idx, w, off, k, 99, form=form)
        assert np.all(s[0] == 123456)
        # register c holds the arrival routed to server c
        assert np.array_equal(_bits(y[0][c]), _bits(t))


def test_fastgm_form_differs_from_plain_form(orc):
    """Both are valid Gumbel-Max sketches but of different draws (the FastGM
    key of (i, j) is an order statistic routed by the permutation)."""
    idx, w, off = W.single(nplus=200)
    s0, y0 = orc.sketch(idx, w, off, 128, 1, form=0)
    s1, y1 = orc.sketch(idx, w, off, 128, 1, form=1)
    assert not np.array_equal(_bits(y0), _bits(y1))
