"""Pins of the oracle's Heisenberg (O(3)) sweep, Eq. (10) with uniform proposals."""
import math

import numpy as np
import pytest

from oracle import exact as X
from oracle import oracle as O
import workloads as W
from tests import npref

SEED = W.seed_for(43)


def test_random_start_uniform_on_sphere():
    """z uniform on [-1, 1] and azimuth uniform: moments of the uniform sphere."""
    s = O.init_heis(3, 24, SEED, 0)
    n = len(s)
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-15)
    sd = math.sqrt(1.0 / (3 * n))
    assert np.all(np.abs(s.mean(axis=0)) < 5 * sd)
    assert np.all(np.abs((s ** 2).mean(axis=0) - 1 / 3) < 5 * math.sqrt(4 / 45 / n))
    assert abs((s[:, 0] * s[:, 1]).mean()) < 5 * math.sqrt(1 / 15 / n)
    # projection on any axis is uniform on [-1, 1] (Archimedes): histogram test
    counts = np.histogram(s[:, 0], bins=20, range=(-1, 1))[0]
    chi2 = ((counts - n / 20) ** 2 / (n / 20)).sum()
    assert chi2 < 19 + 6 * math.sqrt(38)


def test_infinite_temperature_accepts_every_proposal():
    """At beta = 0 every move is accepted: after a sweep all spins are fresh
    proposals (uniform on the sphere, unit norm)."""
    L = 16
    s = O.init_heis(3, L, SEED, 1)
    n_acc = O.heis_sweep(3, L, s, 0.0, SEED, 1, 0, 0)
    assert n_acc == L ** 3
    s0 = O.init_heis(3, L, SEED, 1)
    assert np.all(np.abs(s - s0).max(axis=1) > 0)
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-15)
    assert np.all(np.abs(s.mean(axis=0)) < 5 * math.sqrt(1 / (3 * L ** 3)))


@pytest.mark.parametrize("dim,L,beta", [(3, 8, 0.5), (3, 8, 2.0), (2, 16, 1.2)])
def test_acceptance_rate_matches_closed_form(dim, L, beta):
    """Per half-sweep from a fixed state the number of accepted moves averages
    sum_i P(a_i, |h_i|) with P the exact acceptance of a uniform proposal."""
    s0 = O.init_heis(dim, L, SEED, 2)
    h = npref.heis_field(dim, L, s0)
    a = (s0 * h).sum(axis=1)
    H = np.linalg.norm(h, axis=1)
    P = X.heis_acceptance_probability(a, H, beta)
    col = npref.colours(dim, L)
    trials = 600
    for c in (0, 1):
        mine = col == c
        acc = 0
        for t in range(trials):
            s = s0.copy()
            acc += O.heis_half_sweep(dim, L, s, beta, SEED, 2, t, c)
            assert np.array_equal(s[~mine], s0[~mine])
        p = P[mine]
        mean = trials * p.sum()
        var = trials * (p * (1 - p)).sum()
        assert abs(acc - mean) < 4.5 * math.sqrt(var), (c, acc, mean)


@pytest.mark.parametrize("dim,L", [(3, 12), (2, 32)])
def test_high_temperature_tree_energy(dim, L):
    """At beta = 0.05 the energy per site is -d L(beta) up to O(L(beta)^4)."""
    beta = 0.05
    means = []
    for r in range(6):
        s = O.init_heis(dim, L, SEED, 10 + r)
        series = []
        for t in range(300):
            O.heis_sweep(dim, L, s, beta, SEED, 10 + r, t, 16)
            if t >= 10:
                series.append(O.heis_energy(dim, L, s) / L ** dim)
        means.append(np.mean(series))
    m, err = np.mean(means), np.std(means, ddof=1) / math.sqrt(len(means))
    assert abs(m - X.heis_tree_energy(beta, dim)) < 4.5 * err + 1e-5


def test_renormalisation_schedule():
    L = 8
    s = O.init_heis(3, L, SEED, 3)
    s *= 1.5
    O.heis_sweep(3, L, s, 0.0, SEED, 3, 14, 16)        # t = 14: not a renorm sweep
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-15)  # all replaced at beta=0
    s = O.init_heis(3, L, SEED, 3) * 1.5
    O.heis_sweep(3, L, s, 1e6, SEED, 3, 14, 16)        # only downhill moves, no renorm
    norms = np.linalg.norm(s, axis=1)
    kept = np.isclose(norms, 1.5)
    assert np.all(kept | np.isclose(norms, 1.0)) and kept.sum() > len(s) // 4
    O.heis_sweep(3, L, s, 1e6, SEED, 3, 15, 16)        # (15 + 1) % 16 == 0: renorm
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-15)


def test_energy_closed_forms():
    L = 8
    n = np.array([0.6, 0.0, 0.8])
    s = np.tile(n, (L ** 3, 1)).copy()
    assert O.heis_energy(3, L, s) == pytest.approx(-3 * L ** 3, rel=1e-14)
    assert np.allclose(O.heis_magnetisation(3, L, s), L ** 3 * n, rtol=1e-14)
    col = npref.colours(3, L)
    s[col == 1] *= -1
    assert O.heis_energy(3, L, s) == pytest.approx(3 * L ** 3, rel=1e-14)
    assert np.allclose(O.heis_magnetisation(3, L, s), 0.0, atol=1e-12)


def test_resume_identity():
    L = 8
    a = O.init_heis(3, L, SEED, 4)
    b = a.copy()
    O.heis_run(3, L, a, 0.7, SEED, 4, 0, 40, 16)
    O.heis_run(3, L, b, 0.7, SEED, 4, 0, 17, 16)
    O.heis_run(3, L, b, 0.7, SEED, 4, 17, 23, 16)
    assert np.array_equal(a, b)
