"""Pins of the oracle's energy / magnetisation measurement (Eqs. 1, 11)."""
import numpy as np
import pytest

from oracle import oracle as O
import workloads as W
from tests import npref

SEED = W.seed_for(45)


@pytest.mark.parametrize("dim,L", [(2, 6), (2, 10), (3, 4), (3, 6)])
def test_closed_form_states(dim, L):
    N = L ** dim
    up = np.ones(N, np.int8)
    assert O.energy(dim, L, None, up) == -dim * N and O.magnetisation(dim, L, up) == N
    neel = np.where(npref.colours(dim, L) == 0, 1, -1).astype(np.int8)
    assert O.energy(dim, L, None, neel) == dim * N and O.magnetisation(dim, L, neel) == 0
    one = up.copy()
    one[N // 2 + 1] = -1
    assert O.energy(dim, L, None, one) == -dim * N + 4 * dim
    assert O.magnetisation(dim, L, one) == N - 2


@pytest.mark.parametrize("dim,L", [(2, 8), (3, 6)])
def test_spin_glass_energy_is_gauge_invariant(dim, L):
    N = L ** dim
    J = O.init_couplings(dim, L, SEED, 1)
    s = O.init_spins(dim, L, SEED, 2)
    eps = O.init_spins(dim, L, SEED, 3)
    Jg = J.reshape(dim, N).copy()
    g = npref.as_grid(dim, L, eps)
    for mu in range(dim):
        Jg[mu] *= eps * np.roll(g, -1, axis=npref.axis_of(dim, mu)).reshape(-1)
    assert O.energy(dim, L, J, s) == O.energy(dim, L, Jg.reshape(-1), (s * eps).astype(np.int8))
    # the state s = (product of couplings' signs) can be satisfied on a
    # ferromagnetic gauge: J_ij = eps_i eps_j has ground state s = eps
    Jf = np.ones_like(J).reshape(dim, N)
    for mu in range(dim):
        Jf[mu] = eps * np.roll(g, -1, axis=npref.axis_of(dim, mu)).reshape(-1)
    assert O.energy(dim, L, Jf.reshape(-1), eps) == -dim * N
