"""Pins of the oracle's double-checkerboard sweep with multi-hit updates
(Sec. 3.2, Sec. 3.4): single-tile and single-hit special cases reduce to
the plain checkerboard sweep, beta = 0 has a closed form, and runs on a
4 x 4 lattice with 2 x 2 tiles reproduce the enumerated averages (each hit
is a Metropolis update that keeps the Boltzmann distribution)."""
import math

import numpy as np
import pytest

from oracle import exact as X
from oracle import oracle as O
import workloads as W

SEED = W.seed_for(70)


@pytest.mark.parametrize("ea", [False, True])
def test_single_tile_single_hit_is_the_plain_sweep(ea):
    L = 16
    J = O.init_couplings(2, L, SEED, 2) if ea else None
    a = O.init_spins(2, L, SEED, 2)
    b = a.copy()
    da = O.run(2, L, J, a, 0.6, SEED, 2, 7, 5)
    db = O.dcb_run(L, L, 1, J, b, 0.6, SEED, 2, 7, 5)
    assert np.array_equal(a, b) and da == db


def test_single_tile_k_hits_are_k_plain_sweeps():
    """One tile, k hits per sweep: sweeps t0 .. t0+n-1 are the plain sweeps
    t0*k .. (t0+n)*k - 1 (hit j of sweep t draws as plain sweep t*k + j)."""
    L, k, t0, n = 16, 3, 4, 2
    J = O.init_couplings(2, L, SEED, 5)
    a = O.init_spins(2, L, SEED, 5)
    b = a.copy()
    da = O.run(2, L, J, a, 0.9, SEED, 5, t0 * k, n * k)
    db = O.dcb_run(L, L, k, J, b, 0.9, SEED, 5, t0, n)
    assert np.array_equal(a, b) and da == db


def test_palindromic_odd_sweep_runs_colour_1_first():
    L, t = 16, 9  # odd sweep
    J = O.init_couplings(2, L, SEED, 6)
    a = O.init_spins(2, L, SEED, 6)
    b = a.copy()
    da = O.half_sweep(2, L, J, a, 0.7, SEED, 6, t, 1)
    da += O.half_sweep(2, L, J, a, 0.7, SEED, 6, t, 0)
    db = O.dcb_run(L, L, 1, J, b, 0.7, SEED, 6, t, 1, palindromic=True)
    assert np.array_equal(a, b) and da == db


@pytest.mark.parametrize("T,k,pal", [(4, 1, False), (4, 3, True), (8, 2, False)])
def test_beta_zero_flips_every_attempt(T, k, pal):
    """At beta = 0 every attempt is accepted: after n sweeps every spin has
    flipped n*k times, whatever the tiling."""
    L, n = 16, 3
    J = O.init_couplings(2, L, SEED, 7)
    s0 = O.init_spins(2, L, SEED, 7)
    s = s0.copy()
    O.dcb_run(L, T, k, J, s, 0.0, SEED, 7, 0, n, palindromic=pal)
    assert np.array_equal(s, s0 * (-1) ** (n * k))


def test_tiling_changes_the_chain():
    """With several tiles the update order differs from the plain sweep."""
    L = 16
    a = O.init_spins(2, L, SEED, 8)
    b = a.copy()
    O.run(2, L, None, a, 0.44, SEED, 8, 0, 3)
    O.dcb_run(L, 8, 1, None, b, 0.44, SEED, 8, 0, 3)
    assert not np.array_equal(a, b)


@pytest.mark.parametrize("ea,k,pal", [(False, 1, False), (True, 3, False), (True, 2, True)])
def test_4x4_tiled_runs_match_enumeration(ea, k, pal):
    """4 x 4 lattice, 2 x 2 tiles (B = 2): time and replica averages of E,
    E^2 and M^2 against the enumeration, within 4.5 standard errors."""
    L, T, beta, reps, sweeps, burn = 4, 2, 0.6, 48, 1500, 100
    J = O.init_couplings(2, L, SEED, 9) if ea else None
    E_all, M_all = X.enumerate_states(2, L, J)
    ex = X.boltzmann_averages(E_all, M_all, beta)
    per = {"E": [], "E2": [], "M2": []}
    for r in range(reps):
        s = O.init_spins(2, L, SEED, 100 + r)
        E0 = O.energy(2, L, J, s)
        Es, Ms = [], []
        e = E0
        for t in range(sweeps):
            e += O.dcb_run(L, T, k, J, s, beta, SEED, 100 + r, t, 1, palindromic=pal)
            if t >= burn:
                Es.append(e)
                Ms.append(O.magnetisation(2, L, s))
        assert e == O.energy(2, L, J, s)
        Es = np.array(Es, np.float64)
        Ms = np.array(Ms, np.float64)
        per["E"].append(Es.mean())
        per["E2"].append((Es ** 2).mean())
        per["M2"].append((Ms ** 2).mean())
    for key, vals in per.items():
        vals = np.array(vals)
        err = vals.std(ddof=1) / math.sqrt(len(vals))
        assert abs(vals.mean() - ex[key]) < 4.5 * err, (key, vals.mean(), ex[key], err)


# ---------------------------------------------------------------- 3D --
@pytest.mark.parametrize("ea", [False, True])
def test_3d_single_tile_single_hit_is_the_plain_sweep(ea):
    L = 8
    J = O.init_couplings(3, L, SEED, 5) if ea else None
    a = O.init_spins(3, L, SEED, 5)
    b = a.copy()
    da = O.run(3, L, J, a, 0.3, SEED, 5, 4, 3)
    db = O.dcb_run(L, L, 1, J, b, 0.3, SEED, 5, 4, 3, dim=3)
    assert np.array_equal(a, b) and da == db


def test_3d_single_tile_k_hits_are_k_plain_sweeps():
    L, k = 8, 3
    a = O.init_spins(3, L, SEED, 6)
    b = a.copy()
    O.run(3, L, None, a, 0.25, SEED, 6, 2 * k, 2 * k)
    O.dcb_run(L, L, k, None, b, 0.25, SEED, 6, 2, 2, dim=3)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("T,k,pal", [(4, 2, False), (2, 3, True)])
def test_3d_beta_zero_flips_every_attempt(T, k, pal):
    L, n = 8, 2
    s = O.init_spins(3, L, SEED, 7)
    s0 = s.copy()
    O.dcb_run(L, T, k, None, s, 0.0, SEED, 7, 0, n, palindromic=pal, dim=3)
    assert np.array_equal(s, s0 * (-1) ** (n * k))


def test_3d_tiling_changes_the_chain():
    L = 8
    a = O.init_spins(3, L, SEED, 8)
    b = a.copy()
    O.dcb_run(L, 4, 1, None, a, 0.3, SEED, 8, 0, 1, dim=3)
    O.dcb_run(L, L, 1, None, b, 0.3, SEED, 8, 0, 1, dim=3)
    assert not np.array_equal(a, b)


@pytest.mark.parametrize("T,k", [(4, 2), (2, 4)])
def test_3d_high_temperature_energy(T, k):
    """beta = 0.1 (t^5 corrections below 1e-5): the tiled multi-hit chain
    samples the energy of the high-temperature series."""
    L, beta = 8, 0.1
    means = []
    for r in range(8):
        s = O.init_spins(3, L, SEED, 20 + r)
        series = []
        for t in range(150):
            O.dcb_run(L, T, k, None, s, beta, SEED, 20 + r, t, 1, dim=3)
            if t >= 10:
                series.append(O.energy(3, L, None, s) / L ** 3)
        means.append(np.mean(series))
    m, err = np.mean(means), np.std(means, ddof=1) / math.sqrt(len(means))
    assert abs(m - X.ising_highT_energy(beta, 3)) < 4.5 * err + 2e-5
