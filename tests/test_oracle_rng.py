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


_ROCRAND_PROBE = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
// rocRAND's Philox4x32-10 engine on the host: key = seed, counter words
// (0, 1) = block index, (2, 3) = subsequence; prints the block's four words.
int main() {
    unsigned long long seed, sub, blk;
    while (scanf("%llu %llu %llu", &seed, &sub, &blk) == 3) {
        rocrand_device::philox4x32_10_engine e(seed, sub, 4ull * blk);
        unsigned a = e(), b = e(), c = e(), d = e();
        printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
"""


def test_philox_matches_rocrand(tmp_path):
    """The oracle's Philox4x32-10 against rocRAND's engine (an independent
    implementation, compiled for the host from the ROCm headers) on counters
    that use all four words and keys that use both halves."""
    import os
    import shutil
    import subprocess

    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers or hipcc not available")
    src = tmp_path / "probe.cpp"
    src.write_text(_ROCRAND_PROBE)
    exe = tmp_path / "probe"
    subprocess.run([hipcc, "-O1", str(src), "-o", str(exe)], check=True, capture_output=True)
    rng = np.random.default_rng(1101)
    cases = []
    for k in range(64):
        seed = int(rng.integers(0, 1 << 63)) * 2 + (k & 1)
        ctr = [int(x) for x in rng.integers(0, 1 << 32, 4, dtype=np.uint64)]
        ctr[1] &= (1 << 30) - 1  # keeps 4 * block below 2^64
        cases.append((seed, ctr))
    cases.append((W.seed_for(2), [5, 17, 3, 2 * 3 + 1]))  # a Metropolis head draw
    lines = "".join(f"{s} {c[2] | (c[3] << 32)} {c[0] | (c[1] << 32)}\n" for s, c in cases)
    out = subprocess.run([str(exe)], input=lines, check=True, capture_output=True, text=True).stdout.split("\n")
    for (seed, ctr), line in zip(cases, out):
        want = [int(x) for x in line.split()]
        got = [int(x) for x in O.philox(ctr, [seed & 0xFFFFFFFF, seed >> 32])]
        assert got == want, (seed, ctr)
