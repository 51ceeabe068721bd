"""Pins of the exact references themselves (enumeration, Kaufman, Onsager)."""
import math

import numpy as np
import pytest

from oracle import exact as X
from tests.conftest import read_golden


@pytest.mark.parametrize("beta", [0.1, 0.3, X.BETA_C_2D, 0.6, 1.0])
def test_kaufman_equals_enumeration_4x4(beta):
    E, M = X.enumerate_states(2, 4)
    a = X.boltzmann_averages(E, M, beta)
    k = X.kaufman_thermo(beta, 4)
    N = 16
    assert k["lnZ_per_site"] == pytest.approx(a["lnZ"] / N, rel=1e-13)
    assert k["e"] == pytest.approx(-a["E"] / N, rel=1e-12)
    assert k["C"] == pytest.approx(beta * beta * (a["E2"] - a["E"] ** 2) / N, rel=1e-10, abs=1e-12)


def test_enumeration_ground_states_and_levels():
    E, M = X.enumerate_states(2, 4)
    assert E.min() == -32 and (E == -32).sum() == 2          # all up / all down
    assert E.max() == 32 and (E == 32).sum() == 2            # the two Neel states
    assert np.all(E % 4 == 0)
    assert (1 << 16) == len(E)


def test_kaufman_reproduces_table1():
    """Table 1 (row "exact"): e = -E/N and C_V for L = 1024 at beta = 0.4.

    The printed values agree with the exact finite-size result to 3e-9; the
    exact value also equals Onsager's infinite-lattice energy to 1e-12 since
    the correlation length at beta = 0.4 is a few lattice spacings."""
    (L, beta, e, C), = read_golden("table1_exact.txt")
    k = X.kaufman_thermo(float(beta), int(L))
    assert abs(k["e"] - float(e)) < 1e-8
    assert abs(k["C"] - float(C)) < 1e-8
    assert abs(-k["e"] - X.onsager_energy(float(beta))) < 1e-12


def test_onsager_special_values():
    assert X.onsager_energy(X.BETA_C_2D) == pytest.approx(-math.sqrt(2.0), abs=1e-12)
    # beta -> infinity: ground state energy -2 per spin; beta -> 0: -2 tanh(beta)
    assert X.onsager_energy(5.0) == pytest.approx(-2.0, abs=1e-8)
    assert X.onsager_energy(1e-4) == pytest.approx(-2 * math.tanh(1e-4), rel=1e-6)
    assert X.yang_magnetisation(0.4) == 0.0
    assert X.yang_magnetisation(5.0) == pytest.approx(1.0, abs=1e-15)
    assert X.yang_magnetisation(X.BETA_C_2D + 1e-9) < 0.2


@pytest.mark.parametrize("beta", [0.02, 0.05])
def test_highT_series_matches_onsager_in_2d(beta):
    """The t^3 series (plaquette count d(d-1)/2) is checked in 2D against Onsager."""
    t = math.tanh(beta)
    assert X.ising_highT_energy(beta, 2) == pytest.approx(X.onsager_energy(beta), abs=20 * t ** 5)


def test_heis_acceptance_limits():
    # a = -H (spin anti-aligned with its field): every proposal lowers E
    assert X.heis_acceptance_probability(np.array([-2.0]), np.array([2.0]), 1.5)[0] == pytest.approx(1.0)
    # beta -> 0 limit
    assert X.heis_acceptance_probability(np.array([0.3]), np.array([1.0]), 1e-9)[0] == pytest.approx(1.0, abs=1e-6)
    # numeric integral check of the closed form
    a, H, beta = 0.7, 1.3, 0.9
    b = np.linspace(-H, H, 200001)
    f = np.minimum(1.0, np.exp(-beta * (a - b)))
    num = np.trapezoid(f, b) / (2 * H)
    assert X.heis_acceptance_probability(np.array([a]), np.array([H]), beta)[0] == pytest.approx(num, abs=1e-8)
