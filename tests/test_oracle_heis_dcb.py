"""Pins of the oracle's double-checkerboard sweep of the 2D Heisenberg model
(orc_heis_dcb_run): its reductions to the plain sweep (itself pinned in
test_oracle_heis.py), the draw numbering of the hits, beta = 0, and the
sampled distribution at high temperature."""
import math

import numpy as np
import pytest

from oracle import exact as X
from oracle import oracle as O
import workloads as W

SEED = W.seed_for(81)


def test_single_tile_single_hit_is_the_plain_sweep():
    L = 16
    a = O.init_heis(2, L, SEED, 0)
    b = a.copy()
    na = O.heis_dcb_run(L, L, 1, a, 0.9, SEED, 0, 13, 6, renorm_every=16)
    nb = O.heis_run(2, L, b, 0.9, SEED, 0, 13, 6, 16)
    assert na == nb and np.array_equal(a, b)


def test_single_tile_k_hits_are_k_plain_sweeps():
    """Hit j of sweep t draws as plain sweep t*k + j."""
    L, k = 16, 3
    a = O.init_heis(2, L, SEED, 1)
    b = a.copy()
    na = O.heis_dcb_run(L, L, k, a, 1.3, SEED, 1, 4, 3, renorm_every=0)
    nb = O.heis_run(2, L, b, 1.3, SEED, 1, 4 * k, 3 * k, 0)
    assert na == nb and np.array_equal(a, b)


def test_palindromic_odd_sweep_runs_colour_1_first():
    L = 16
    a = O.init_heis(2, L, SEED, 2)
    b = a.copy()
    O.heis_dcb_run(L, L, 1, a, 0.7, SEED, 2, 5, 1, palindromic=True, renorm_every=0)
    O.heis_half_sweep(2, L, b, 0.7, SEED, 2, 5, 1)
    O.heis_half_sweep(2, L, b, 0.7, SEED, 2, 5, 0)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("T,k,pal", [(4, 3, False), (8, 2, True), (16, 1, False)])
def test_beta_zero_keeps_the_last_hits_proposals(T, k, pal):
    """At beta = 0 every move is accepted, so after sweep t every site holds
    the proposal of hit k - 1: whatever the tiling, the state equals a plain
    sweep t*k + k - 1 at beta = 0 from any start."""
    L, t = 16, 3
    a = O.init_heis(2, L, SEED, 3)
    n = O.heis_dcb_run(L, T, k, a, 0.0, SEED, 3, t, 1, palindromic=pal, renorm_every=0)
    assert n == k * L * L
    b = O.init_heis(2, L, SEED, 4) * 0.5  # any start
    O.heis_run(2, L, b, 0.0, SEED, 3, t * k + k - 1, 1, 0)
    assert np.array_equal(a, b)


def test_tiling_changes_the_chain():
    L = 16
    a = O.init_heis(2, L, SEED, 5)
    b = a.copy()
    O.heis_dcb_run(L, 8, 1, a, 1.0, SEED, 5, 0, 1)
    O.heis_dcb_run(L, L, 1, b, 1.0, SEED, 5, 0, 1)
    assert not np.array_equal(a, b)


@pytest.mark.parametrize("T,k,pal", [(8, 3, False), (4, 2, True)])
def test_high_temperature_tree_energy(T, k, pal):
    """At beta = 0.05 the energy per site is -2 L(beta) up to O(L(beta)^4)."""
    L, beta = 32, 0.05
    means = []
    for r in range(6):
        s = O.init_heis(2, L, SEED, 20 + r)
        series = []
        for t in range(120):
            O.heis_dcb_run(L, T, k, s, beta, SEED, 20 + r, t, 1, palindromic=pal)
            if t >= 5:
                series.append(O.heis_energy(2, L, s) / L ** 2)
        means.append(np.mean(series))
    m, err = np.mean(means), np.std(means, ddof=1) / math.sqrt(len(means))
    assert abs(m - X.heis_tree_energy(beta, 2)) < 4.5 * err + 1e-5


@pytest.mark.parametrize("cap", [0.05, 0.6, 2.0])
def test_small_step_proposals_fill_the_cap_uniformly(cap):
    """beta = 0, one hit: every spin moves to a uniform point of the cap
    1 - s.s' <= cap around its old direction (uniform in the cosine and the
    azimuth), and stays a unit vector."""
    L = 32
    s0 = O.init_heis(2, L, SEED, 30)
    s = s0.copy()
    n = O.heis_dcb_run(L, 16, 1, s, 0.0, SEED, 30, 0, 1, renorm_every=0, cap=cap)
    assert n == L * L
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-14)
    w = 1.0 - (s * s0).sum(axis=1)  # 1 - cos(angle)
    assert w.min() >= -1e-14 and w.max() <= cap + 1e-12
    counts = np.histogram(w / cap, bins=16, range=(0, 1))[0]
    chi2 = ((counts - L * L / 16) ** 2 / (L * L / 16)).sum()
    assert chi2 < 15 + 6 * math.sqrt(30)
    # azimuth about the old direction: the component along any fixed
    # perpendicular direction averages to zero
    perp = np.cross(s0, np.array([0.3, -0.5, 0.8]))
    perp /= np.linalg.norm(perp, axis=1, keepdims=True)
    proj = (s * perp).sum(axis=1)
    sd = math.sqrt((cap - cap * cap / 3) / 2 / (L * L))  # E[w (2 - w)] / 2 over w uniform in [0, cap]
    assert abs(proj.mean()) < 5 * sd


@pytest.mark.parametrize("cap", [0.3, 1.0])
def test_small_step_high_temperature_tree_energy(cap):
    """The small-step chain samples the same distribution: e = -2 L(beta) at
    beta = 0.05."""
    L, beta = 32, 0.05
    means = []
    for r in range(6):
        s = O.init_heis(2, L, SEED, 40 + r)
        series = []
        for t in range(160):
            O.heis_dcb_run(L, 16, 2, s, beta, SEED, 40 + r, t, 1, cap=cap)
            if t >= 20:
                series.append(O.heis_energy(2, L, s) / L ** 2)
        means.append(np.mean(series))
    m, err = np.mean(means), np.std(means, ddof=1) / math.sqrt(len(means))
    assert abs(m - X.heis_tree_energy(beta, 2)) < 4.5 * err + 1e-5


def test_small_step_low_temperature_matches_uniform_proposals():
    """beta = 2 on 16^2: the long-run energy with small steps (cap 0.2) and
    with uniform proposals agree within their errors."""
    L, beta = 16, 2.0
    res = {}
    for cap in (0.0, 0.2):
        means = []
        for r in range(8):
            s = O.init_heis(2, L, SEED, 60 + r)
            series = []
            for t in range(400):
                O.heis_dcb_run(L, 8, 2, s, beta, SEED, 60 + r, t, 1, cap=cap)
                if t >= 100 and t % 4 == 0:
                    series.append(O.heis_energy(2, L, s) / L ** 2)
            means.append(np.mean(series))
        res[cap] = (np.mean(means), np.std(means, ddof=1) / math.sqrt(len(means)))
    (m0, e0), (m1, e1) = res[0.0], res[0.2]
    assert abs(m0 - m1) < 4.5 * math.hypot(e0, e1), res
