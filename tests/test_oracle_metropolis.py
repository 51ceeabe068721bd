"""Pins of the oracle's checkerboard Metropolis sweep (Ising / EA, 2D / 3D).

Every check compares the oracle with something it does not compute itself:
the Metropolis probability of Eq. (2), exact enumeration, Onsager/Yang,
the high-temperature series, or an exact symmetry of the definition.
"""
import math

import numpy as np
import pytest

from oracle import exact as X
from oracle import oracle as O
import workloads as W
from tests import npref

SEED = W.seed_for(42)


def _couplings(model, dim, L, q=0):
    return O.init_couplings(dim, L, SEED, q) if model == W.MODEL_EA else None


@pytest.mark.parametrize("model,dim,L,beta", [
    (W.MODEL_ISING, 2, 16, 0.3), (W.MODEL_EA, 2, 16, 0.45),
    (W.MODEL_ISING, 3, 8, 0.2), (W.MODEL_EA, 3, 8, 0.35)])
@pytest.mark.parametrize("colour", [0, 1])
def test_flip_probabilities_follow_metropolis(model, dim, L, beta, colour):
    """From a fixed state, one half-sweep flips each site of the colour
    independently with probability min(1, exp(-beta dE)) (Eq. 2); sites of the
    other colour never change."""
    J = _couplings(model, dim, L)
    s0 = O.init_spins(dim, L, SEED, 3)
    h = npref.local_field(dim, L, J, s0)
    dE = 2 * s0.astype(np.int64) * h
    col = npref.colours(dim, L)
    trials = 3000
    flips = np.zeros(s0.size, np.int64)
    for t in range(trials):
        s = s0.copy()
        got = O.half_sweep(dim, L, J, s, beta, SEED, 3, t, colour)
        changed = s != s0
        assert not np.any(changed & (col != colour))
        assert got == int(dE[changed].sum())
        flips += changed
    mine = col == colour
    assert np.all(flips[mine & (dE <= 0)] == trials)
    for m in range(1, dim + 1):
        sel = mine & (dE == 4 * m)
        if not sel.any():
            continue
        n = sel.sum() * trials
        p = math.exp(-beta * 4 * m)
        z = (flips[sel].sum() - n * p) / math.sqrt(n * p * (1 - p))
        assert abs(z) < 4.5, (m, z)


@pytest.mark.parametrize("model,dim", [(W.MODEL_ISING, 2), (W.MODEL_EA, 2), (W.MODEL_ISING, 3), (W.MODEL_EA, 3)])
def test_infinite_temperature_flips_every_spin(model, dim):
    L = 6 if dim == 3 else 10
    J = _couplings(model, dim, L)
    s = O.init_spins(dim, L, SEED, 0)
    s0 = s.copy()
    for t in range(5):
        O.sweep(dim, L, J, s, 0.0, SEED, 0, t)
        assert np.array_equal(s, s0 * (-1) ** (t + 1))


@pytest.mark.parametrize("dim", [2, 3])
def test_zero_temperature_closed_forms(dim):
    L = 8
    N = L ** dim
    big = 1e3  # exp(-4 * big) underflows: thresholds are all 0
    up = np.ones(N, np.int8)
    s = up.copy()
    assert O.sweep(dim, L, None, s, big, SEED, 0, 0) == 0 and np.all(s == 1)
    # one overturned spin of colour 0 flips back in the first half-sweep
    s = up.copy()
    s[0] = -1
    assert O.sweep(dim, L, None, s, big, SEED, 0, 0) == -4 * dim and np.all(s == 1)
    # Neel state: every colour-0 spin has dE = -4d and flips; afterwards the
    # colour-1 spins sit in an aligned state with dE = +4d and stay
    col = npref.colours(dim, L)
    s = np.where(col == 0, 1, -1).astype(np.int8)
    dE = O.sweep(dim, L, None, s, big, SEED, 0, 0)
    assert np.all(s == -1) and dE == -(N // 2) * 4 * dim


def _series_stats(dim, L, J, beta, reps, sweeps, burn, cold=False):
    Es, Ms = [], []
    for r in range(reps):
        s = np.ones(L ** dim, np.int8) if cold else O.init_spins(dim, L, SEED, r)
        E, M = O.run_series(dim, L, J, s, beta, SEED, r, 0, sweeps)
        Es.append(E[burn:].astype(np.float64))
        Ms.append(M[burn:].astype(np.float64))
    return np.array(Es), np.array(Ms)


def _mean_err(per_rep):
    """Mean over independent replicas of their time averages, with its error."""
    m = per_rep.mean(axis=1)
    return m.mean(), m.std(ddof=1) / math.sqrt(len(m))


@pytest.mark.parametrize("beta", [0.3, X.BETA_C_2D, 0.6])
def test_4x4_ising_matches_enumeration(beta):
    E_all, M_all = X.enumerate_states(2, 4)
    ex = X.boltzmann_averages(E_all, M_all, beta)
    Es, Ms = _series_stats(2, 4, None, beta, reps=96, sweeps=2000, burn=100)
    for key, vals in (("E", Es), ("E2", Es ** 2), ("absM", np.abs(Ms)), ("M2", Ms ** 2)):
        mean, err = _mean_err(vals)
        assert abs(mean - ex[key]) < 4.5 * err, (key, mean, ex[key], err)


def test_4x4_spin_glass_matches_enumeration():
    J = O.init_couplings(2, 4, SEED, 11)
    E_all, M_all = X.enumerate_states(2, 4, J)
    for beta in (0.4, 1.0):
        ex = X.boltzmann_averages(E_all, M_all, beta)
        Es, Ms = _series_stats(2, 4, J, beta, reps=96, sweeps=2000, burn=100)
        for key, vals in (("E", Es), ("E2", Es ** 2), ("M2", Ms ** 2)):
            mean, err = _mean_err(vals)
            assert abs(mean - ex[key]) < 4.5 * err, (beta, key, mean, ex[key], err)


def test_onsager_energy_high_temperature():
    """L = 64 at beta = 0.3: finite-size corrections are exponentially small."""
    L, beta = 64, 0.30
    Es, _ = _series_stats(2, L, None, beta, reps=8, sweeps=400, burn=50)
    mean, err = _mean_err(Es / L ** 2)
    assert abs(mean - X.onsager_energy(beta)) < 4.5 * err + 1e-4


def test_yang_magnetisation_cold_start():
    """L = 64 at beta = 0.5 from the aligned state stays in the ordered phase."""
    L, beta = 64, 0.50
    Es, Ms = _series_stats(2, L, None, beta, reps=8, sweeps=400, burn=50, cold=True)
    mean_m, err_m = _mean_err(np.abs(Ms) / L ** 2)
    mean_e, err_e = _mean_err(Es / L ** 2)
    assert abs(mean_m - X.yang_magnetisation(beta)) < 4.5 * err_m + 2e-4
    assert abs(mean_e - X.onsager_energy(beta)) < 4.5 * err_e + 2e-4


def test_3d_high_temperature_series():
    L, beta = 12, 0.05
    Es, _ = _series_stats(3, L, None, beta, reps=8, sweeps=600, burn=20)
    mean, err = _mean_err(Es / L ** 3)
    t = math.tanh(beta)
    assert abs(mean - X.ising_highT_energy(beta, 3)) < 4.5 * err + 200 * t ** 5


# ---------------------------------------------------------------- invariants
@pytest.mark.parametrize("model,dim,L", [(W.MODEL_ISING, 2, 12), (W.MODEL_EA, 2, 12),
                                         (W.MODEL_ISING, 3, 6), (W.MODEL_EA, 3, 6)])
def test_incremental_energy_and_resume(model, dim, L):
    J = _couplings(model, dim, L)
    s = O.init_spins(dim, L, SEED, 5)
    E0 = O.energy(dim, L, J, s)
    assert E0 == npref.energy(dim, L, J, s)
    a = s.copy()
    dE = O.run(dim, L, J, a, 0.6, SEED, 5, 0, 30)
    assert O.energy(dim, L, J, a) == E0 + dE
    assert (E0 + dE) % 4 == E0 % 4
    b = s.copy()
    dE1 = O.run(dim, L, J, b, 0.6, SEED, 5, 0, 13)
    dE2 = O.run(dim, L, J, b, 0.6, SEED, 5, 13, 17)
    assert np.array_equal(a, b) and dE1 + dE2 == dE


@pytest.mark.parametrize("model,dim,L", [(W.MODEL_ISING, 2, 12), (W.MODEL_EA, 3, 6)])
def test_global_flip_symmetry(model, dim, L):
    J = _couplings(model, dim, L)
    s = O.init_spins(dim, L, SEED, 2)
    a, b = s.copy(), (-s).astype(np.int8)
    O.run(dim, L, J, a, 0.5, SEED, 2, 0, 20)
    O.run(dim, L, J, b, 0.5, SEED, 2, 0, 20)
    assert np.array_equal(b, -a)


@pytest.mark.parametrize("dim,L", [(2, 12), (3, 6)])
def test_gauge_symmetry(dim, L):
    """(eps_i s_i, eps_i J_ij eps_j) evolves to eps_i times the original
    trajectory: dE is gauge invariant and the draws are keyed by site."""
    N = L ** dim
    J = O.init_couplings(dim, L, SEED, 4)
    s = O.init_spins(dim, L, SEED, 6)
    eps = O.init_spins(dim, L, SEED + 1, 0)
    Jg = J.reshape(dim, N).copy()
    g = npref.as_grid(dim, L, eps)
    for mu in range(dim):
        nb = np.roll(g, -1, axis=npref.axis_of(dim, mu)).reshape(-1)
        Jg[mu] = J.reshape(dim, N)[mu] * eps * nb
    Jg = Jg.reshape(-1)
    a, b = s.copy(), (s * eps).astype(np.int8)
    assert O.energy(dim, L, J, a) == O.energy(dim, L, Jg, b)
    O.run(dim, L, J, a, 0.7, SEED, 6, 0, 20)
    O.run(dim, L, Jg, b, 0.7, SEED, 6, 0, 20)
    assert np.array_equal(b, a * eps)


@pytest.mark.parametrize("dim,L", [(2, 12), (3, 6)])
def test_all_plus_couplings_equal_ferromagnet(dim, L):
    J = np.ones(dim * L ** dim, np.int8)
    s = O.init_spins(dim, L, SEED, 1)
    a, b = s.copy(), s.copy()
    O.run(dim, L, J, a, 0.4, SEED, 1, 0, 15)
    O.run(dim, L, None, b, 0.4, SEED, 1, 0, 15)
    assert np.array_equal(a, b)


def test_couplings_are_bimodal_half_half():
    J = O.init_couplings(3, 16, SEED, 0)
    n = J.size
    assert set(np.unique(J)) == {-1, 1}
    assert abs((J == 1).sum() - n / 2) < 5 * math.sqrt(n / 4)


def test_random_start_is_half_half():
    s = O.init_spins(2, 128, SEED, 0)
    assert set(np.unique(s)) == {-1, 1}
    assert abs(int(s.sum())) < 5 * math.sqrt(s.size)
