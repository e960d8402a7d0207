"""Pins of the oracle's draw arithmetic against values fixed outside it.

* splitmix64: published known-answer outputs (golden file).
* U(x): the exact rational (n + 1/2) 2^-53 rounded once (Python Fraction).
* neglog: within 1 ulp of a 64-bit-mantissa logarithm; exact and +0 at 1.
* RandInt: range and uniformity (chi-square); Lemire bias bound.
* ln 2 split used by neglog: checked against a 50-digit ln 2.
"""
import math
import os
from decimal import Decimal, getcontext
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M64 = (1 << 64) - 1


def test_splitmix64_known_answers(orc):
    rows = [ln.split() for ln in open(os.path.join(GOLDEN, "splitmix64_kat.txt"))
            if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for n, state, out in rows:
        assert orc.sm64(int(state, 16)) == int(out, 16), (n, state)


def test_unif_is_exact_rounding(orc):
    rng = np.random.default_rng(11)
    xs = [0, M64, (1 << 63), ((1 << 53) - 1) << 11, ((1 << 52) + 1) << 11,
          ((1 << 52) - 1) << 11, 1 << 11, 2047]
    xs += [int(v) for v in rng.integers(0, 1 << 63, size=2000, dtype=np.uint64)]
    xs += [int(v) << 1 | 1 for v in rng.integers(0, 1 << 62, size=2000, dtype=np.uint64)]
    for x in xs:
        n = x >> 11
        want = float(Fraction(2 * n + 1, 1 << 54))
        assert orc.unif(x) == want, hex(x)
    assert orc.unif(0) == 2.0 ** -54
    assert orc.unif(M64) == 1.0           # (2^53 - 1) + 0.5 rounds to even 2^53
    assert 0.0 < orc.unif(12345) <= 1.0


def _ulp_err(r, u):
    ref = -np.log(np.longdouble(u))
    if ref == 0:
        return 0.0 if r == 0 else math.inf
    return float(abs(np.longdouble(r) - ref) / np.longdouble(np.spacing(np.float64(ref))))


def test_neglog_accuracy(orc):
    rng = np.random.default_rng(5)
    us = [orc.unif(int(x)) for x in rng.integers(0, 1 << 63, size=20000, dtype=np.uint64)]
    us += list(rng.random(20000) * 0.999 + 1e-3)
    us += [2.0 ** -n for n in range(0, 55)]
    us += [math.sqrt(0.5), math.nextafter(math.sqrt(0.5), 1), math.nextafter(math.sqrt(0.5), 0),
           math.nextafter(1.0, 0), 0.5, 0.75, 2.0 ** -54, math.nextafter(2.0 ** -54, 1)]
    worst = max(_ulp_err(orc.neglog(float(u)), u) for u in us)
    assert worst <= 1.0, worst


def test_neglog_special_values(orc):
    r = orc.neglog(1.0)
    assert r == 0.0 and math.copysign(1.0, r) == 1.0   # +0, never -0
    ln2 = math.log(2.0)
    for n in range(1, 55):
        v = orc.neglog(2.0 ** -n)
        assert abs(v - n * ln2) <= np.spacing(n * ln2), n
    # Exp(1) variate of the all-ones draw is +0 (U = 1)
    e = orc.exp1(M64)
    assert e == 0.0 and math.copysign(1.0, e) == 1.0
    # smallest uniform gives 54 ln 2
    assert abs(orc.exp1(0) - 54 * ln2) <= 2 * np.spacing(54 * ln2)


def test_ln2_split_constants():
    """neglog splits ln 2 as HI + LO; HI has 21 trailing zero bits so e*HI is
    exact for |e| < 2^11, and HI + LO equals ln 2 to far below an ulp."""
    hi = float.fromhex("0x1.62e42fee00000p-1")
    lo = float.fromhex("0x1.a39ef35793c76p-33")
    getcontext().prec = 60
    ln2 = Decimal(2).ln()
    m, _ = math.frexp(hi)
    assert int(m * 2 ** 53) % (1 << 21) == 0
    err = abs(Decimal(hi) + Decimal(lo) - ln2)
    assert err < Decimal(2) ** -80
    assert float(ln2 - Decimal(hi)) == lo


def test_randint_range_and_uniformity(orc):
    for (z, k) in [(1, 1), (1, 2), (3, 7), (1, 64), (200, 256), (4096, 4096), (1, 4096)]:
        span = k - z + 1
        n = max(2000, 60 * span) if span <= 64 else 40000
        draws = np.array([orc.randint(orc.sm64(i * 7 + z), z, k) for i in range(n)])
        assert draws.min() >= z and draws.max() <= k
        if span > 1:
            counts = np.bincount(draws - z, minlength=span)
            if span <= 64:
                p = stats.chisquare(counts).pvalue
                assert p > 1e-4, (z, k, p)
            else:
                # spread check for wide ranges: every decile of the range is hit evenly
                dec = np.bincount((draws - z) * 10 // span, minlength=10)
                assert stats.chisquare(dec).pvalue > 1e-4


def test_randint_bias_bound():
    """Multiply-high on the top 32 bits maps 2^32 inputs onto `span` outputs;
    each output receives floor or ceil of 2^32/span inputs, so the relative
    bias is below span / 2^32 (< 1e-6 for span <= 4096)."""
    for span in (1, 3, 7, 100, 4096):
        # count of 32-bit h with (h*span)>>32 == c is ceil((c+1) 2^32/span) - ceil(c 2^32/span)
        lo = min(-(-((c + 1) << 32) // span) - (-(-(c << 32) // span)) for c in range(min(span, 64)))
        hi = max(-(-((c + 1) << 32) // span) - (-(-(c << 32) // span)) for c in range(min(span, 64)))
        assert hi - lo <= 1
        assert (hi - lo) / (2 ** 32 / span) < span / 2 ** 32 + 1e-12


def test_prefix_and_tags_are_distinct(orc):
    # element prefixes depend on the seed and the index; tags give independent draws
    a = orc.prefix(1, 5)
    assert a != orc.prefix(2, 5) and a != orc.prefix(1, 6)
    assert a == orc.sm64(orc.sm64(1) ^ 5)
    # index is taken as its 32-bit pattern
    assert orc.prefix(1, 2**31 - 1) == orc.sm64(orc.sm64(1) ^ (2**31 - 1))
