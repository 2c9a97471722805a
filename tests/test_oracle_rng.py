"""Pins of the oracle's random-number layer (counter-based generator, exact
uniform conversions, integer ball sampler) against published values and
distribution laws.  The paper names no generator; the Philox4x32-10 choice and
its stream layout are the contract's reading (design notes)."""
import math
import os

import numpy as np
import pytest
from scipy import stats

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(oracle):
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        got = oracle.philox(ctr, key)
        assert [int(x) for x in got] == want


def test_philox_words_uniform(oracle):
    # 4 x 20000 words over 16 equal bins: chi-square
    words = np.concatenate([oracle.philox((i, 7, 3, 9), (1, 2)) for i in range(20000)])
    counts = np.bincount(words >> 28, minlength=16)
    chi2, p = stats.chisquare(counts)
    assert p > 1e-4


def test_philox_counter_sensitivity(oracle):
    base = oracle.philox((1, 2, 3, 4), (5, 6))
    for i in range(4):
        c = [1, 2, 3, 4]
        c[i] ^= 1
        assert not np.array_equal(oracle.philox(c, (5, 6)), base)
    assert not np.array_equal(oracle.philox((1, 2, 3, 4), (5, 7)), base)


def test_ball_candidate_grid_and_acceptance(oracle):
    rng = np.random.default_rng(3)
    n = 40000
    acc = 0
    radii = []
    for _ in range(n):
        wa, wb = (int(x) for x in rng.integers(0, 2**32, size=2))
        ok, m = oracle.ball_candidate(wa, wb)
        assert all(v % 2 != 0 and abs(v) < 2**21 for v in m)
        r2 = sum(v * v for v in m)
        assert ok == (r2 < 2**42)
        if ok:
            acc += 1
            radii.append(math.sqrt(r2) / 2**21)
    p = acc / n
    # acceptance = volume of the unit ball / volume of the cube = pi/6
    assert abs(p - math.pi / 6) < 4 * math.sqrt(p * (1 - p) / n)
    # uniform in the ball: P(|o| < r) = r^3
    ks = stats.kstest(np.array(radii), lambda r: np.clip(r, 0, 1) ** 3)
    assert ks.pvalue > 1e-4


def test_ball_candidate_extremes(oracle):
    ok, m = oracle.ball_candidate(0, 0)
    assert m == (-(2**21) + 1,) * 3 and not ok
    # all-ones fields -> m = 2^21 - 1 on every axis, outside the ball
    ok, m = oracle.ball_candidate(0xFFFFFFFF, 0x7FFFFFFF)
    assert m == (2**21 - 1,) * 3 and not ok
    # f = 2^20 on every axis -> m = +1 (the grid point nearest the centre)
    v = (1 << 20) | (1 << 41) | (1 << 62)
    ok, m = oracle.ball_candidate(v & 0xFFFFFFFF, v >> 32)
    assert ok and m == (1, 1, 1)
