"""Pins of the oracle's parallel-tempering step (Sec. 6, Eq. 12)."""
import math

import numpy as np
import pytest

from oracle import exact as X
from oracle import oracle as O
import workloads as W

SEED = W.seed_for(44)


def _chain(dim, L, n_temps, r0, J=None):
    spins = np.stack([O.init_spins(dim, L, SEED, r0 + k) for k in range(n_temps)])
    E = np.array([O.energy(dim, L, J, spins[k]) for k in range(n_temps)], np.int64)
    return spins, E, np.arange(n_temps, dtype=np.int32)


def test_equal_temperatures_accept_every_swap():
    """x = 0 for equal betas: every attempt is accepted, so the permutation
    follows the deterministic even/odd transposition walk."""
    n = 6
    spins, E, sot = _chain(2, 8, n, 0)
    beta = np.full(n, 0.4)
    acc = np.zeros(n, np.uint64)
    expect = list(range(n))
    for t in range(9):
        O.pt_run(2, 8, None, spins, beta, sot, E, SEED, 0, 0, t, 1, acc)
        for k in range(t & 1, n - 1, 2):
            expect[k], expect[k + 1] = expect[k + 1], expect[k]
        assert list(sot) == expect
    assert int(acc.sum()) == sum(len(range(t & 1, n - 1, 2)) for t in range(9))


def test_sweeps_per_step_numbering():
    """Step t with m sweeps per exchange: every slot gets the plain sweeps
    t*m .. t*m + m - 1 at its temperature (equal temperatures: every swap is
    accepted, so the permutation is the transposition walk)."""
    n, L, m, t = 4, 8, 3, 5
    spins, E, sot = _chain(2, L, n, 40)
    ref = spins.copy()
    beta = np.full(n, 0.45)
    O.pt_run(2, L, None, spins, beta, sot, E, SEED, 0, 40, t, 1, sweeps_per_step=m)
    for slot in range(n):
        O.run(2, L, None, ref[slot], 0.45, SEED, 40 + slot, t * m, m)
    assert np.array_equal(spins, ref)
    assert list(sot) == [0, 2, 1, 3]  # t odd: the pair (1, 2) exchanges
    for k in range(n):
        assert E[k] == O.energy(2, L, None, spins[k])


def test_energy_tracking_and_permutation_validity():
    J = O.init_couplings(2, 8, SEED, 3)
    n = 8
    spins, E, sot = _chain(2, 8, n, 16, J)
    beta = W.geometric_ladder(0.5, 2.0, n)
    O.pt_run(2, 8, J, spins, beta, sot, E, SEED, 2, 16, 0, 200)
    assert sorted(sot) == list(range(n))
    for k in range(n):
        assert E[k] == O.energy(2, 8, J, spins[k])


@pytest.mark.parametrize("m", [1, 3])
def test_swap_rate_matches_exact_double_sum(m):
    """For two temperatures on the 4x4 Ising model the mean acceptance of a
    swap attempt is sum_{E1,E2} P_b1(E1) P_b2(E2) min(1, exp((b2-b1)(E2-E1))),
    whatever the number m of sweeps between exchange rounds."""
    b1, b2 = 0.30, 0.45
    E_all, M_all = X.enumerate_states(2, 4)
    lev, cnt = X.density_of_states(E_all)

    def p(b):
        w = cnt * np.exp(-b * (lev - lev.min()))
        return w / w.sum()

    P1, P2 = p(b1), p(b2)
    x = (b2 - b1) * (lev[None, :] - lev[:, None])
    exact = float((P1[:, None] * P2[None, :] * np.minimum(1.0, np.exp(x))).sum())
    beta = np.array([b1, b2])
    rates = []
    for q in range(64):
        spins, E, sot = _chain(2, 4, 2, 2 * q)
        O.pt_run(2, 4, None, spins, beta, sot, E, SEED, q, 2 * q, 0, 100, sweeps_per_step=m)   # equilibrate
        acc = np.zeros(2, np.uint64)
        O.pt_run(2, 4, None, spins, beta, sot, E, SEED, q, 2 * q, 100, 2000, acc, sweeps_per_step=m)
        rates.append(float(acc[0]) / 1000.0)   # pair 0 is attempted on even steps
    m, err = np.mean(rates), np.std(rates, ddof=1) / math.sqrt(len(rates))
    assert abs(m - exact) < 4.5 * err, (m, exact, err)


def test_uniform_occupancy():
    """The stationary law is symmetric in the slot labels: in the long run each
    slot spends the same fraction of time at every temperature."""
    n = 4
    beta = np.array([0.2, 0.3, 0.4, 0.5])
    occ = np.zeros((n, n))
    for q in range(24):
        spins, E, sot = _chain(2, 4, n, 4 * q)
        for t in range(1500):
            O.pt_run(2, 4, None, spins, beta, sot, E, SEED, q, 4 * q, t, 1)
            if t >= 100:
                occ[sot, np.arange(n)] += 1
    frac = occ / occ.sum(axis=1, keepdims=True)
    assert np.all(np.abs(frac - 1.0 / n) < 0.03), frac


def test_swap_uniform_is_53_bit_uniform():
    u = np.array([O.swap_u53(SEED, k % 31, k // 31, 7) for k in range(20000)])
    assert np.all((u >= 0) & (u < 1))
    assert abs(u.mean() - 0.5) < 5 * math.sqrt(1 / 12 / len(u))
    # 53 significant bits: scaled by 2^53 every value is an integer
    assert np.all(np.floor(u * 2.0 ** 53) == u * 2.0 ** 53)


@pytest.mark.planted_tie
def test_near_tie_audit_counts_a_planted_tie():
    """The audit sees an exchange whose exp(x) lies within 2^-40 of its
    uniform: two frozen slots (all spins up at beta >= 8, where every
    threshold is 0) with energies chosen so that x = ln(u53) up to rounding."""
    n, L, t, q = 2, 4, 0, 5
    u = O.swap_u53(SEED, 0, t, q)
    D = 100
    b0 = 8.0
    b1 = b0 - math.log(u) / D                        # x = (b1 - b0) * (E_B - E_A) = ln(u) when E_B - E_A = -D
    spins = np.ones((n, L * L), np.int8)
    E = np.array([0, -D], np.int64)
    sot = np.arange(n, dtype=np.int32)
    O.pt_audit(reset=True)
    O.pt_run(2, L, None, spins, np.array([b0, b1]), sot, E, SEED, q, 0, t, 1)
    audit = O.pt_audit(reset=True)
    assert audit["attempts"] == 1 and audit["near_ties"] == 1 and audit["min_gap"] < 2.0 ** -40
    assert list(E) == [0, -D]                        # frozen: no flip was accepted
    # one step later (odd step: no pair of two slots is attempted)
    O.pt_run(2, L, None, spins, np.array([b0, b1]), sot, E, SEED, q, 0, t + 1, 1)
    assert O.pt_audit(reset=True)["attempts"] == 0


def test_near_tie_audit_on_a_ladder():
    """A 4x4 ladder of 8 temperatures over 1000 steps: hundreds of attempts
    with x < 0, none within 2^-40 (the audit fixture asserts that too)."""
    n = 8
    spins, E, sot = _chain(2, 4, n, 0)
    beta = np.ascontiguousarray(W.geometric_ladder(0.5, 2.0, n))
    O.pt_audit(reset=True)
    O.pt_run(2, 4, None, spins, beta, sot, E, SEED, 0, 0, 0, 1000)
    audit = O.pt_audit()
    assert audit["attempts"] > 150 and audit["near_ties"] == 0 and audit["min_gap"] > 2.0 ** -40
