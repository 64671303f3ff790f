"""Pins of the oracle's random-number, logarithm, spacing and drive-table functions
against values fixed outside the oracle (published vectors, the paper's worked
example, libm, scipy)."""
import json
import math
import os

import numpy as np
import pytest
import scipy.stats

import oracle

# Known-answer vectors published with the Random123 library for Philox4x32 with 10
# rounds: (counter words, key words) -> output words; tests/golden/philox4x32_10_kat.json.
def _kat():
    with open(os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.json")) as f:
        vec = json.load(f)["vectors"]
    return [([int(x, 16) for x in v["counter"]], [int(x, 16) for x in v["key"]],
             [int(x, 16) for x in v["output"]]) for v in vec]


PHILOX_KAT = _kat()


@pytest.mark.parametrize("ctr,key,expected", PHILOX_KAT)
def test_philox_known_answers(ctr, key, expected):
    assert list(oracle.philox4x32_10(ctr, key)) == expected


def test_philox_words_uniform():
    # 4 x 20000 words: mean of u32/2^32 ~ 1/2, and each byte value equally likely
    words = np.concatenate([oracle.philox4x32_10([i, 7, 0, 1], [5, 9]) for i in range(20000)])
    u = words.astype(np.float64) / 2**32
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / len(u))
    counts = np.bincount((words & 0xFF).astype(np.int64), minlength=256)
    chi2 = ((counts - len(words) / 256) ** 2 / (len(words) / 256)).sum()
    assert chi2 < scipy.stats.chi2.ppf(1 - 1e-6, 255)


def test_neg_log_matches_libm():
    rng = np.random.default_rng(0)
    grid = (rng.integers(0, 2**24, size=4000) + 1).astype(np.float64) * 2.0**-24
    edge = [1.0, 2.0**-24, 0.5, 1 - 2.0**-24, math.sqrt(0.5), math.nextafter(math.sqrt(0.5), 0),
            math.nextafter(math.sqrt(0.5), 1), 0.75, 0.999, 1e-300, 0.3]
    for u in list(grid) + list(rng.random(2000) + 1e-300) + edge:
        got = oracle.neg_log(u)
        ref = -math.log(u)
        assert abs(got - ref) <= 2 * math.ulp(ref) + 1e-300, (u, got, ref)
    assert oracle.neg_log(1.0) == 0.0


def test_fig2_worked_example():
    """Fig. 2: n = 6 sorted distinct integers from [0, 100) out of the uniforms (a); the
    printed rows are in tests/golden/fig2_worked_example.json."""
    with open(os.path.join(os.path.dirname(__file__), "golden", "fig2_worked_example.json")) as f:
        fx = json.load(f)
    a = fx["a_uniforms"]
    b_printed = fx["b_neg_log"]
    c_printed = fx["c_exclusive_sum"]
    d_printed = fx["d_normalised"]
    e_printed = fx["e_scaled_rounded"]
    g_printed = fx["g_result"]
    n = fx["n"]
    lo, hi = fx["range"]
    # (a) -> (b): -log, to the two printed decimals
    for u, b in zip(a, b_printed):
        assert abs(oracle.neg_log(u) - b) <= 0.0051
    # (b) -> (c): exclusive running sum; uses the first n+1 draws, the last is unused
    S, x = oracle.spacing_core(a[: n + 1], spare=(hi - lo) - n)
    c = S.astype(np.float64) * 2.0**-24
    assert len(c) == n + 2
    assert np.all(np.abs(c - np.array(c_printed)) <= 0.011)
    # (c) -> (d): normalise by the total; positions 3 and 4 of the printed row are
    # inconsistent with (c) (2.32/3.88 = 0.598, 2.53/3.88 = 0.652), the rest agree
    d = c / c[-1]
    for k in (0, 1, 2, 5, 6, 7):
        assert abs(d[k] - d_printed[k]) <= 0.01
    # (d) -> (e) and (e) -> (g) on the printed numbers: scale by b - n = 94, round,
    # then add 0..n-1
    assert [round(94 * v) for v in d_printed] == e_printed
    assert [e_printed[k + 1] + k for k in range(n)] == g_printed
    # the exact pipeline: equal to the printed (e) and (g) wherever (d) is consistent
    e_exact = x - np.arange(n)
    assert list(e_exact) == [19, 20, 56, 61, 62, 85]
    assert list(x) == [19, 21, 58, 64, 66, 90]
    for k in (0, 1, 5):
        assert e_exact[k] == e_printed[k + 1] and x[k] == g_printed[k]


def test_spacing_core_properties():
    rng = np.random.default_rng(1)
    for n, spare in [(1, 0), (5, 0), (5, 1), (100, 10), (300, 100000), (64, 3)]:
        for _ in range(20):
            u = (rng.integers(0, 2**24, size=n + 1) + 1) * 2.0**-24
            S, x = oracle.spacing_core(u, spare)
            assert np.all(np.diff(S.astype(np.int64)) >= 0)
            assert np.all(np.diff(x) >= 1)
            assert x[0] >= 0 and x[-1] <= n + spare - 1
            if spare == 0:
                assert list(x) == list(range(n))


def test_spacing_core_all_gaps_zero():
    S, x = oracle.spacing_core([1.0] * 6, spare=10)
    assert list(S) == [0] * 7 and list(x) == list(range(5))


@pytest.mark.parametrize("n,p", [(1000, 0.002), (1000, 0.001), (100, 0.3), (5, 0.5), (10000, 0.0002)])
def test_binom_table_matches_scipy(n, p):
    tbl = oracle.binom_table(n, p)
    assert tbl[-1] == 2**32
    assert np.all(np.diff(tbl.astype(np.float64)) >= 0)
    for j, v in enumerate(tbl[:-1]):
        ref = scipy.stats.binom.cdf(j, n, p) * 2.0**32
        assert abs(float(v) - ref) <= 2.0 + 1e-9 * ref, (j, v, ref)
    # truncation: the mass beyond the table is below the 2^-32 resolution
    assert scipy.stats.binom.sf(len(tbl) - 1, n, p) < 2.0**-32


def test_binom_table_degenerate():
    assert list(oracle.binom_table(0, 0.3)) == [2**32]
    assert list(oracle.binom_table(1000, 0.0)) == [2**32]
    assert list(oracle.binom_table(3, 1.0)) == [0, 0, 0, 2**32]
