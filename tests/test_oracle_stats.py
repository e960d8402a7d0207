"""Statistical pins of the oracle against the paper's closed forms.

Seeds are fixed, so each check is deterministic; thresholds are set at
p > 1e-4 (or 4-5 standard errors) so a correct implementation passes with
a wide margin while a dropped term, a wrong sign or a transposed operand
fails.

* Gumbel-Max trick (Sec. 1): P(s_j(v) = i) = v_i / sum(v), both forms.
* Lemiesz sketch (Sec. 1): y_j ~ EXP(c), sum_j y_j ~ Gamma(k, c).
* Time analysis (Sec. 2.5): y* = max_j y_j of the normalised vector has
  CDF (1 - e^-x)^k, mean H_k and variance sum 1/m^2.
* Theorem 1 (Sec. 2.4): E[J_hat] = J_P and Var = J_P (1 - J_P) / k.
* Theorem 2 (Sec. 2.4): E[c_hat] = c; the exact variance of (k-1)/Gamma(k, c)
  is c^2/(k-2), which is below the paper's 2/k approximation.
* Eq. (7)-(8) (Renyi): O_z has mean H_k - H_{k-z}; k O_1 ~ Exp(1).
* Fisher-Yates (Sec. 2.2): the server of step z is uniform.
* Release heuristic (Sec. 2.1 worked example): R = 17, R_i printed.
* Complexity (Sec. 2.5): arrivals needed ~ k H_k + n+.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

from paper_2302_05176_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
FIG1_V = np.array([0.3, 0.1, 0.05, 0.05, 0.2, 0.07, 0.1, 0.03])


def H(k):
    return sum(1.0 / m for m in range(1, k + 1))


def _fig1():
    idx = np.arange(1, 9, dtype=np.int32)
    w = FIG1_V.astype(np.float32)
    off = np.array([0, 8], np.int64)
    return idx, w, off


def test_worked_example_release_counts(orc):
    g = {}
    for ln in open(os.path.join(GOLDEN, "fig1_worked_example.txt")):
        if ln.strip() and not ln.startswith("#"):
            key, *vals = ln.split()
            g[key] = [float(x) for x in vals]
    v = np.array(g["v"])
    k = int(g["k"][0])
    R = math.ceil(k * math.log(k))
    assert R == int(g["R"][0])
    Ri = orc.release_counts(v, R)
    assert list(Ri) == [int(x) for x in g["R_i"]]
    assert Ri.sum() == int(g["sum"][0])


@pytest.mark.parametrize("form", [0, 3])
def test_argmax_distribution_matches_weights(orc, form):
    idx, w, off = _fig1()
    k = 64
    counts = np.zeros(8)
    for seed in range(1, 301):
        s, _ = orc.sketch(idx, w, off, k, seed, form=form)
        counts += np.bincount(s[0] - 1, minlength=8)
    p = w.astype(np.float64) / w.astype(np.float64).sum()
    pv = stats.chisquare(counts, counts.sum() * p).pvalue
    assert pv > 1e-4, (counts, pv)


def _vec():
    idx, w, off = W.batch(nvec=1, seed=90, sizes=np.array([300]))
    return idx, w, off, float(w.astype(np.float64).sum())


@pytest.mark.parametrize("form", [0, 3])
def test_register_values_exponential_and_gamma(orc, form):
    idx, w, off, S = _vec()
    k = 64
    regs, sums, ymax = [], [], []
    for seed in range(1, 301):
        _, y = orc.sketch(idx, w, off, k, seed, form=form)
        regs.append(y[0] * S)
        sums.append(y[0].sum() * S)
        ymax.append(y[0].max() * S)
    regs = np.concatenate(regs)
    assert stats.kstest(regs, "expon").pvalue > 1e-4
    assert stats.kstest(sums, stats.gamma(k).cdf).pvalue > 1e-4
    cdf = lambda x: (1.0 - np.exp(-np.asarray(x))) ** k
    assert stats.kstest(ymax, cdf).pvalue > 1e-4
    hk = H(k)
    sd = math.sqrt(sum(1.0 / m ** 2 for m in range(1, k + 1)))
    assert abs(np.mean(ymax) - hk) < 5 * sd / math.sqrt(len(ymax))


@pytest.mark.parametrize("k", [16, 128])
def test_weighted_cardinality_unbiased(orc, k):
    idx, w, off, S = _vec()
    est = []
    for seed in range(1, 401):
        _, y = orc.sketch(idx, w, off, k, seed, form=3)
        est.append(orc.wcard(y[0]))
    r = np.array(est) / S
    n = len(r)
    assert abs(r.mean() - 1.0) < 4.0 * math.sqrt(1.0 / ((k - 2) * n))
    var = r.var(ddof=1)
    assert 0.75 < var * (k - 2) < 1.3
    assert var < 2.0 / k            # Theorem 2's approximation is an upper bound here


def test_jp_closed_form_properties(orc):
    rng = np.random.default_rng(4)
    for _ in range(20):
        ia = np.sort(rng.choice(60, 25, replace=False))
        ib = np.sort(rng.choice(60, 30, replace=False))
        wa = rng.exponential(size=25)
        wb = rng.exponential(size=30)
        assert abs(orc.jp_brute(ia, wa, ib, wb) - orc.jp_sorted(ia, wa, ib, wb)) < 1e-12
        assert abs(orc.jp_brute(ia, wa, ia, 3.5 * wa) - 1.0) < 1e-12      # scale invariant
        # sets: J_P reduces to |A n B| / |A u B|
        j = len(np.intersect1d(ia, ib)) / len(np.union1d(ia, ib))
        assert abs(orc.jp_brute(ia, np.ones(25), ib, np.ones(30)) - j) < 1e-12
    assert orc.jp_brute([1, 2], [1.0, 2.0], [3, 4], [1.0, 1.0]) == 0.0


@pytest.mark.parametrize("form", [0, 3])
def test_jaccard_estimator_theorem1(orc, form):
    rng = np.random.default_rng(8)
    n = 40
    ia = np.sort(rng.choice(1000, n, replace=False))
    ib = np.concatenate([ia[:25], np.sort(rng.choice(np.arange(1000, 2000), n - 25, replace=False))])
    wa = rng.exponential(size=n).astype(np.float32)
    wb = rng.exponential(size=n).astype(np.float32)
    wb[:25] = wa[:25] * np.float32(1.5) + rng.exponential(size=25).astype(np.float32) * np.float32(0.2)
    jp = orc.jp_sorted(ia, wa.astype(np.float64), ib, wb.astype(np.float64))
    idx = np.concatenate([ia, ib]).astype(np.int32)
    w = np.concatenate([wa, wb])
    off = np.array([0, n, 2 * n], np.int64)
    k = 64
    est = []
    for seed in range(1, 401):
        s, _ = orc.sketch(idx, w, off, k, seed, form=form)
        est.append(orc.jaccard(s[0], s[1]))
    est = np.array(est)
    sd = math.sqrt(jp * (1 - jp) / k)
    assert 0.05 < jp < 0.95
    assert abs(est.mean() - jp) < 4.0 * sd / math.sqrt(len(est))
    assert 0.75 < est.var(ddof=1) / sd ** 2 < 1.3


def test_renyi_order_statistics(orc):
    k = 32
    T = np.array([orc.element_arrivals(5, i, 1.0, k)[0] for i in range(3000)])
    # weight 1 gives r = 1 exactly, so t_z = O_z
    for z in (1, 8, 16, 32):
        mean = H(k) - H(k - z)
        sd = math.sqrt(sum(1.0 / m ** 2 for m in range(k - z + 1, k + 1)))
        assert abs(T[:, z - 1].mean() - mean) < 4.5 * sd / math.sqrt(len(T)), z
    assert stats.kstest(k * T[:, 0], "expon").pvalue > 1e-4
    # increments are independent exponentials with rate k - z + 1
    inc = (T[:, 10] - T[:, 9]) * (k - 10)
    assert stats.kstest(inc, "expon").pvalue > 1e-4


def test_fisher_yates_server_uniform(orc):
    k = 16
    C = np.array([orc.element_arrivals(17, i, 2.0, k)[1] for i in range(4000)])
    for z in (0, 7, 14):
        counts = np.bincount(C[:, z], minlength=k)
        assert stats.chisquare(counts).pvalue > 1e-4
    # every row is a permutation
    assert np.all(np.sort(C, axis=1) == np.arange(k))


def test_needed_arrivals_close_to_k_Hk_plus_n(orc):
    idx, w, off = W.batch(nvec=1, seed=91, sizes=np.array([2000]))
    k = 64
    tot = []
    for seed in range(1, 41):
        s, y = orc.sketch(idx, w, off, k, seed, form=3)
        tot.append(orc.needed_arrivals(idx, w, off, k, seed, y)[0])
    want = k * H(k) + 2000
    assert abs(np.mean(tot) / want - 1.0) < 0.05
