"""Pins of the oracle's random-number contract and acceptance thresholds."""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import oracle as O
from tests.conftest import read_golden
import workloads as W


def test_philox_known_answers():
    """Philox4x32-10 against the published known-answer vectors."""
    rows = read_golden("philox4x32_10_kat.txt")
    assert len(rows) == 3
    for row in rows:
        v = [int(x, 16) for x in row]
        out = O.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_metropolis_uniform_is_uniform():
    """The 32-bit Metropolis uniform: chi^2 over 64 bins of its top and low bits."""
    seed = W.seed_for(99)
    n = 1 << 14
    u = np.array([O.metropolis_u32(seed, 3, 1, h & 1, h) for h in range(n)], np.uint64)
    for vals in ((u >> 26), (u & 63)):
        counts = np.bincount(vals.astype(np.int64), minlength=64)
        chi2 = ((counts - n / 64) ** 2 / (n / 64)).sum()
        # 63 degrees of freedom: mean 63, sd ~11.2; 6 sd bound
        assert chi2 < 63 + 6 * math.sqrt(2 * 63)
    # head and tail halves come from independent draws: no correlation
    head = (u >> 16).astype(np.float64)
    tail = (u & 0xFFFF).astype(np.float64)
    corr = np.corrcoef(head, tail)[0, 1]
    assert abs(corr) < 5 / math.sqrt(n)


def test_metropolis_uniform_depends_on_every_key():
    seed = W.seed_for(7)
    base = O.metropolis_u32(seed, 5, 2, 0, 123)
    assert O.metropolis_u32(seed + 1, 5, 2, 0, 123) != base
    assert O.metropolis_u32(seed + (1 << 32), 5, 2, 0, 123) != base
    assert O.metropolis_u32(seed, 6, 2, 0, 123) != base
    assert O.metropolis_u32(seed, 5, 3, 0, 123) != base
    assert O.metropolis_u32(seed, 5, 2, 1, 123) != base
    assert O.metropolis_u32(seed, 5, 2, 0, 124) != base


def _exact_threshold(beta: float, m: int) -> Decimal:
    getcontext().prec = 50
    return Decimal(2) ** 32 * (Decimal(-4 * m) * Decimal(beta)).exp()


BETAS = [0.0, 0.05, 0.30, W.BETA_C_2D, 0.50, 0.693] + list(W.geometric_ladder(0.8, 2.0, 32)) + \
    list(W.geometric_ladder(0.5, 2.0, 16))


@pytest.mark.parametrize("dim", [2, 3])
def test_thresholds_match_50_digit_exp(dim):
    """thr[m] = floor(2^32 exp(-4 m beta)) agrees with 50-digit arithmetic, and no
    value lies within 1e-6 of an integer (so a 1-ulp libm difference cannot move it)."""
    for beta in BETAS:
        thr = O.thresholds(beta, dim)
        assert int(thr[0]) == 1 << 32
        for m in range(1, dim + 1):
            x = _exact_threshold(beta, m)
            assert int(thr[m]) == int(x), (beta, m)
            frac = x - int(x)
            if beta > 0:
                assert 1e-6 < frac < 1 - 1e-6, (beta, m, frac)


def test_threshold_limits():
    thr = O.thresholds(1e3, 3)
    assert [int(v) for v in thr] == [1 << 32, 0, 0, 0]
    thr = O.thresholds(0.0, 2)
    assert [int(v) for v in thr] == [1 << 32] * 3
