"""Pins of the oracle's random-number study (Sec. 3.3, Table 1): the LCGs
with and without skip-ahead and the lagged Fibonacci generators driving the
double checkerboard.

The generators are checked against plain Python big-integer arithmetic in
another formulation (global sequences by iteration, skip-ahead by the closed
form a^M and c (a^M - 1) / (a - 1) of Eqs. 4-5, the Fibonacci sequence as an
unbounded list instead of a ring), the stream layout and the update against
a site-by-site Python model of the tiled sweep, and the physics on the 4x4
lattice against exact enumeration for the generators the paper finds sound.
"""
import math

import numpy as np
import pytest

from oracle import exact as X
from oracle import oracle as O
from tests import philox_ref as P
import workloads as W

SEED = W.seed_for(90)
LCG32 = (1664525, 1013904223, 2 ** 32)
LCG64 = (2862933555777941757, 1442695040888963407, 2 ** 64)
LAGS = {O.GEN_FIB521: (521, 353), O.GEN_FIB1279: (1279, 861)}


def test_lcg32_is_the_numerical_recipes_quick_generator():
    """From x = 0 the recursion gives the values printed for this generator
    (Numerical Recipes' quick generator), and Hull-Dobell holds (full period)."""
    a, c, m = LCG32
    x, got = 0, []
    for _ in range(6):
        x = (a * x + c) % m
        got.append(x)
    assert got == [0x3C6EF35F, 0x47502932, 0xD1CCF6E9, 0xAAF95334, 0x6252E503, 0x9F2EC686]
    for a, c, m in (LCG32, LCG64):
        assert c % 2 == 1 and (a - 1) % 4 == 0


def _x0(gen, rep):
    w = P.seeded(SEED, [0, 0, rep, 16])
    return w[0] if gen == O.GEN_LCG32 else (w[1] << 32) | w[0]


def _global(gen, rep, n):
    """x_n of the skip-ahead global sequence by the closed form of Eq. 4."""
    a, c, m = LCG32 if gen == O.GEN_LCG32 else LCG64
    an = pow(a, n, m)
    cn = (c * ((pow(a, n, m * (a - 1)) - 1) // (a - 1))) % m
    return (an * _x0(gen, rep) + cn) % m


@pytest.mark.parametrize("gen", [O.GEN_LCG32, O.GEN_LCG64])
def test_skip_ahead_streams_interleave_the_global_sequence(gen):
    """Stream j starts at x_j; after n sweeps of k hits (4 k n numbers per
    stream) it holds x_{j + 4 k n M} (M = L^2/4 streams)."""
    L, T, k, n, rep = 16, 4, 2, 3, 5
    M = L * L // 4
    st = O.rng_init(gen, L, T, SEED, rep)
    assert [int(v) for v in st] == [_global(gen, rep, j) for j in range(M)]
    s = O.init_spins(2, L, SEED, rep)
    O.dcb_run_rng(L, T, k, None, s, 0.4, gen, st, n)
    assert [int(v) for v in st] == [_global(gen, rep, j + 4 * k * n * M) for j in range(M)]


@pytest.mark.parametrize("gen", [O.GEN_LCG32_RANDOM, O.GEN_LCG64_RANDOM])
def test_random_seeded_streams(gen):
    """Each stream starts at its own Philox seed and steps by Eq. 3 itself."""
    L, T, k, n, rep = 8, 2, 1, 5, 1
    a, c, m = LCG32 if gen == O.GEN_LCG32_RANDOM else LCG64
    st = O.rng_init(gen, L, T, SEED, rep)
    want = []
    for j in range(L * L // 4):
        w = P.seeded(SEED, [j, 1, rep, 16])
        x = w[0] if gen == O.GEN_LCG32_RANDOM else (w[1] << 32) | w[0]
        assert int(st[j]) == x
        for _ in range(4 * k * n):
            x = (a * x + c) % m
        want.append(x)
    O.dcb_run_rng(L, T, k, None, O.init_spins(2, L, SEED, rep), 0.4, gen, st, n)
    assert [int(v) for v in st] == want


@pytest.mark.parametrize("gen", [O.GEN_FIB521, O.GEN_FIB1279])
def test_lagged_fibonacci_ring(gen):
    """Generator q: initial words from Philox, then x_n = x_{n-r} + x_{n-s}
    mod 2^32; after n sweeps its ring holds the last r numbers (word i the
    number with index = i mod r) and the count mod r."""
    r, s_lag = LAGS[gen]
    L, T, k, n, rep = 16, 4, 3, 2, 2
    Q = (L // T) ** 2 // 2
    st = O.rng_init(gen, L, T, SEED, rep)
    O.dcb_run_rng(L, T, k, None, O.init_spins(2, L, SEED, rep), 0.3, gen, st, n)
    produced = 4 * k * n * (T * T // 2)
    for q in range(Q):
        xs = [P.seeded(SEED, [q * r + i, 2, rep, 16])[0] for i in range(r)]
        for _ in range(produced):
            xs.append((xs[-r] + xs[-s_lag]) % 2 ** 32)
        ring = st[q * (r + 1):(q + 1) * (r + 1)]
        total = r + produced
        assert int(ring[r]) == total % r
        for idx in range(total - r, total):
            assert int(ring[idx % r]) == xs[idx], (q, idx)


def _model_run(L, T, k, J, s, beta, draw, n):
    """Site-by-site model of the study sweep: tile colour 0 then 1, k hits,
    colour 0 then 1, every site of the round drawing draw(q, p) in position
    order; flip iff dE <= 0 or u < floor(2^32 exp(-beta dE)) (the oracle's
    integer table, pinned elsewhere)."""
    thr = O.thresholds(beta, 2)
    B = L // T
    s = s.astype(np.int64).copy()
    Jx = np.ones(L * L, np.int64) if J is None else J[:L * L].astype(np.int64)
    Jy = np.ones(L * L, np.int64) if J is None else J[L * L:].astype(np.int64)
    for _ in range(n):
        for tc in (0, 1):
            for by in range(B):
                for bx in range(B):
                    if (bx + by) & 1 != tc:
                        continue
                    q = by * (B // 2) + bx // 2
                    for _ in range(k):
                        for c in (0, 1):
                            for v in range(T):
                                for u in range(T):
                                    x, y = bx * T + u, by * T + v
                                    if (x + y) & 1 != c:
                                        continue
                                    uu = draw(q, v * (T // 2) + u // 2)
                                    i = y * L + x
                                    xr, xl = y * L + (x + 1) % L, y * L + (x - 1) % L
                                    yu, yd = ((y + 1) % L) * L + x, ((y - 1) % L) * L + x
                                    h = Jx[i] * s[xr] + Jx[xl] * s[xl] + Jy[i] * s[yu] + Jy[yd] * s[yd]
                                    d = 2 * s[i] * h
                                    if d <= 0 or uu < int(thr[d // 4]):
                                        s[i] = -s[i]
    return s


@pytest.mark.parametrize("gen,ea", [(O.GEN_LCG32, False), (O.GEN_LCG64_RANDOM, True), (O.GEN_FIB521, True)])
def test_study_sweep_follows_the_site_model(gen, ea):
    L, T, k, n, rep, beta = 8, 4, 2, 3, 3, 0.38
    J = O.init_couplings(2, L, SEED, 1) if ea else None
    st = O.rng_init(gen, L, T, SEED, rep)
    model_state = [int(v) for v in st]
    M = L * L // 4
    if gen in LAGS:
        r, s_lag = LAGS[gen]
        Q = (L // T) ** 2 // 2
        seqs = [[model_state[q * (r + 1) + i] for i in range(r)] for q in range(Q)]

        def draw(q, p):
            xs = seqs[q]
            xs.append((xs[-r] + xs[-s_lag]) % 2 ** 32)
            return xs[-1]
    else:
        a, c, m = LCG32 if gen in (O.GEN_LCG32, O.GEN_LCG32_RANDOM) else LCG64
        skip = gen in (O.GEN_LCG32, O.GEN_LCG64)
        xs = list(model_state)
        P2 = T * T // 2

        def draw(q, p):
            j = q * P2 + p
            out = xs[j]
            steps = M if skip else 1
            for _ in range(steps):
                xs[j] = (a * xs[j] + c) % m
            return out if m == 2 ** 32 else out >> 32
    s0 = O.init_spins(2, L, SEED, rep)
    want = _model_run(L, T, k, J, s0, beta, draw, n)
    got = s0.copy()
    O.dcb_run_rng(L, T, k, J, got, beta, gen, st, n)
    assert np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("gen", [O.GEN_LCG64_RANDOM, O.GEN_FIB521])
def test_sound_generators_reproduce_the_4x4_enumeration(gen):
    """4x4 Ising at beta = 0.4 with 2x2 tiles: the time averages of E and E^2
    from the study sweep agree with exact enumeration within 4.5 standard
    errors (binned)."""
    L, T, k, beta = 4, 2, 1, 0.4
    E_all, M_all = X.enumerate_states(2, L)
    ex = X.boltzmann_averages(E_all, M_all, beta)
    st = O.rng_init(gen, L, T, SEED, 0)
    s = O.init_spins(2, L, SEED, 0)
    O.dcb_run_rng(L, T, k, None, s, beta, gen, st, 200)
    E = O.energy(2, L, None, s)
    n_bins, per_bin, every = 50, 400, 5
    bins_e, bins_e2 = [], []
    for _ in range(n_bins):
        acc_e = acc_e2 = 0.0
        for _ in range(per_bin):
            E += O.dcb_run_rng(L, T, k, None, s, beta, gen, st, every)
            acc_e += E
            acc_e2 += E * E
        bins_e.append(acc_e / per_bin)
        bins_e2.append(acc_e2 / per_bin)
    for got, want in ((bins_e, ex["E"]), (bins_e2, ex["E2"])):
        m = np.mean(got)
        err = np.std(got, ddof=1) / math.sqrt(n_bins)
        assert abs(m - want) < 4.5 * err, (gen, m, want, err)
