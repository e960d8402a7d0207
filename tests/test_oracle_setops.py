"""Oracle pins for the merge (Sec. 2.3), the estimators' empty and poisoned
conventions (Sec. 1; readings Q8 and Q18), and the two-set weighted
cardinality algebra (Sec. 1 estimator on merged sketches; the Lemiesz
algebra the paper uses in Sec. 4.5).

What fixes each expected value, outside the function under test:
* merge: the sketch the oracle computes for the union vector itself
  (mergeability, Sec. 2.3), for parts that are empty or poisoned too;
* Jaccard of an empty sketch: J_P by its closed form (sum over the common
  positive elements) is 0 when either vector is empty, and Theorem 1's
  variance J_P (1 - J_P)/k is then 0, so the estimate must be exactly 0;
* weighted cardinality of an empty vector: sum of its weights, 0;
* set algebra: J_W of two sets with fixed object weights equals J_P (both
  closed forms of Sec. 1), the union equals the estimator on the sketch of
  the union vector, disjoint sets share no register, a set with itself
  shares every register, and the estimates are unbiased over sketch seeds.
"""
import numpy as np
import pytest

from paper_2302_05176_amd import workloads as W


def _bits(y):
    return np.ascontiguousarray(y).view(np.uint64)


def _row(orc, ii, ww, k, seed, form=3):
    s, y = orc.sketch(np.asarray(ii, np.int32), np.asarray(ww, np.float32),
                      np.array([0, len(ii)], np.int64), k, seed, form=form)
    return s[0], y[0]


@pytest.mark.parametrize("form", [0, 3])
def test_merge_equals_sketch_of_union_with_empty_and_poisoned_parts(orc, form):
    idx, w, off = W.batch(nvec=3, seed=71)
    k = 96
    parts = [(idx[off[v]:off[v + 1]], w[off[v]:off[v + 1]]) for v in range(3)]
    parts.insert(1, (np.zeros(0, np.int32), np.zeros(0, np.float32)))      # empty site
    rows = [_row(orc, ii, ww, k, 5, form) for ii, ww in parts]
    ms, my = orc.merge(np.stack([r[0] for r in rows]), np.stack([r[1] for r in rows]))
    us, uy = _row(orc, np.concatenate([p[0] for p in parts]),
                  np.concatenate([p[1] for p in parts]), k, 5, form)
    assert np.array_equal(ms, us) and np.array_equal(_bits(my), _bits(uy))
    # only empty parts: the union is empty
    e = _row(orc, [], [], k, 5, form)
    es, ey = orc.merge(np.stack([e[0], e[0]]), np.stack([e[1], e[1]]))
    assert np.all(es == -1) and np.all(np.isinf(ey))
    # a part holding an invalid entry: the union holds it too, and the
    # oracle poisons the union's sketch
    bad_i = np.array([7, 8], np.int32)
    bad_w = np.array([1.0, np.nan], np.float32)
    b = _row(orc, bad_i, bad_w, k, 5, form)
    ps, py = orc.merge(np.stack([rows[0][0], b[0]]), np.stack([rows[0][1], b[1]]))
    us, uy = _row(orc, np.concatenate([parts[0][0], bad_i]),
                  np.concatenate([parts[0][1], bad_w]), k, 5, form)
    assert np.all(us == -2) and np.array_equal(ps, us) and np.all(np.isnan(py))


def test_jaccard_of_empty_and_poisoned_sketches(orc):
    k = 64
    idx, w, off = W.batch(nvec=1, seed=72)
    a = _row(orc, idx, w, k, 3)
    e = _row(orc, [], [], k, 3)
    z = _row(orc, [5, 6], [0.0, 0.0], k, 3)           # zero weights only: empty too
    p = _row(orc, [5, 6], [1.0, -1.0], k, 3)          # poisoned
    assert np.all(p[0] == -2)
    for x, y, ix, wx, iy, wy in ((e, e, [], [], [], []), (e, a, [], [], idx, w),
                                 (z, z, [5, 6], [0.0, 0.0], [5, 6], [0.0, 0.0]),
                                 (a, z, idx, w, [5, 6], [0.0, 0.0])):
        jp = orc.jp_brute(ix, wx, iy, wy)
        assert jp == 0.0
        assert orc.jaccard(x[0], y[0]) == jp
    # a poisoned sketch holds no element: it matches nothing, itself included
    assert orc.jaccard(p[0], p[0]) == 0.0
    assert orc.jaccard(p[0], a[0]) == 0.0
    # and a filled sketch with itself matches everywhere (J_P(v, v) = 1)
    assert orc.jaccard(a[0], a[0]) == 1.0 == pytest.approx(orc.jp_brute(idx, w, idx, w), abs=1e-12)


def test_wcard_of_empty_and_poisoned_sketches(orc):
    k = 64
    e = _row(orc, [], [], k, 3)
    assert orc.wcard(e[1]) == 0.0                      # sum of no weights
    p = _row(orc, [5], [np.inf], k, 3)
    assert np.isnan(orc.wcard(p[1]))


def _set_pair(rng, n_a, n_b, shared, dim=1 << 22):
    """Two sets with fixed per-object weights: objects in both carry the same
    weight on both sides."""
    pool = rng.permutation(W.distinct_sorted(rng, n_a + n_b - shared, dim))
    wts = W.exp1_weights(rng, len(pool))
    a = np.arange(0, n_a)
    b = np.concatenate([np.arange(0, shared), np.arange(n_a, n_a + n_b - shared)])
    return (pool[a], wts[a]), (pool[b], wts[b])


def test_jw_equals_jp_for_sets(orc):
    rng = np.random.default_rng(5)
    for shared in (0, 7, 40, 120):
        (ia, wa), (ib, wb) = _set_pair(rng, 120, 90, min(shared, 90))
        common = np.intersect1d(ia, ib)
        wmap = dict(zip(ia.tolist(), wa.astype(np.float64).tolist()))
        wmap.update(dict(zip(ib.tolist(), wb.astype(np.float64).tolist())))
        jw = sum(wmap[i] for i in common.tolist()) / sum(wmap.values())
        assert orc.jp_brute(ia, wa, ib, wb) == pytest.approx(jw, rel=1e-12, abs=1e-15)


@pytest.mark.parametrize("form", [0, 3])
def test_setops_identities(orc, form):
    rng = np.random.default_rng(6)
    k = 128
    (ia, wa), (ib, wb) = _set_pair(rng, 300, 200, 80)
    sa, ya = _row(orc, ia, wa, k, 9, form)
    sb, yb = _row(orc, ib, wb, k, 9, form)
    out = orc.setops(sa, ya, sb, yb)
    # the union is the estimator on the sketch of the union vector (Sec. 2.3)
    ui = np.concatenate([ia, ib])
    uw = np.concatenate([wa, wb])
    us, uy = _row(orc, ui, uw, k, 9, form)
    assert out[0] == orc.wcard(uy)
    # the three parts cover the union: fractions sum to one
    assert out[1] + out[2] + out[3] == pytest.approx(out[0], rel=4e-16 * 4)
    assert 0.0 < out[4] < 1.0
    # swapping the sets swaps the complements
    rev = orc.setops(sb, yb, sa, ya)
    assert rev[0] == out[0] and rev[1] == out[1] and rev[2] == out[3] and rev[3] == out[2]
    # a set with itself: all intersection
    same = orc.setops(sa, ya, sa, ya)
    assert same[0] == orc.wcard(ya) and same[1] == same[0] and same[4] == 1.0
    assert same[2] == 0.0 and same[3] == 0.0
    # disjoint sets share no register
    (ic, wc), _ = _set_pair(rng, 150, 1, 0)
    ic = ic + (1 << 23)                                # outside both supports
    sc, yc = _row(orc, ic, wc, k, 9, form)
    dis = orc.setops(sa, ya, sc, yc)
    assert dis[1] == 0.0 and dis[4] == 0.0
    # against an empty set: everything is A's
    se, ye = _row(orc, [], [], k, 9, form)
    ea = orc.setops(sa, ya, se, ye)
    assert ea[0] == orc.wcard(ya) and ea[2] == ea[0] and ea[1] == 0.0 and ea[3] == 0.0
    # two empty sets: zeros; a poisoned one: NaN everywhere
    assert np.all(orc.setops(se, ye, se, ye) == 0.0)
    sp, yp = _row(orc, [3], [-1.0], k, 9, form)
    assert np.all(np.isnan(orc.setops(sa, ya, sp, yp)))


@pytest.mark.parametrize("form", [0, 3])
def test_setops_unbiased(orc, form):
    """Each estimate is unbiased (Theorem 2 for the union; the winner's
    identity is independent of the register values for the parts).  Over
    200 sketch seeds at k = 256 the mean is within 4 standard errors."""
    rng = np.random.default_rng(8)
    k, nseeds = 256, 200
    (ia, wa), (ib, wb) = _set_pair(rng, 400, 300, 150)
    wa64, wb64 = wa.astype(np.float64), wb.astype(np.float64)
    common = np.isin(ia, ib)
    true = np.array([wa64.sum() + wb64[~np.isin(ib, ia)].sum(), wa64[common].sum(),
                     wa64[~common].sum(), wb64[~np.isin(ib, ia)].sum(), 0.0])
    true[4] = true[1] / true[0]
    # both sets in one oracle call per seed
    idx = np.concatenate([ia, ib]).astype(np.int32)
    w = np.concatenate([wa, wb]).astype(np.float32)
    off = np.array([0, len(ia), len(ia) + len(ib)], np.int64)
    est = []
    for seed in range(1, nseeds + 1):
        s, y = orc.sketch(idx, w, off, k, seed, form=form)
        est.append(orc.setops(s[0], y[0], s[1], y[1]))
    est = np.array(est)
    mean = est.mean(0)
    se = est.std(0, ddof=1) / np.sqrt(nseeds)
    assert np.all(np.abs(mean - true) <= 4.0 * se + 1e-12), (mean, true, se)
    # J_W: binomial variance J (1 - J) / k, as Theorem 1 states for J_P
    var = est[:, 4].var(ddof=1)
    jv = true[4] * (1 - true[4]) / k
    assert 0.6 * jv < var < 1.5 * jv
