"""Small numpy helpers for the pin tests: local fields and energies written with
array shifts (an independent formulation from the oracle's site loops)."""
import numpy as np


def as_grid(dim, L, a):
    return a.reshape((L,) * dim)


def axis_of(dim, mu):
    """Array axis of lattice direction mu (mu = 0 is x, the fastest index)."""
    return dim - 1 - mu


def local_field(dim, L, J, s):
    """h_i = sum_mu [J(i,mu) s(i+e_mu) + J(i-e_mu,mu) s(i-e_mu)], flat int array."""
    g = as_grid(dim, L, s.astype(np.int64))
    h = np.zeros_like(g)
    for mu in range(dim):
        ax = axis_of(dim, mu)
        Jm = np.ones_like(g) if J is None else as_grid(dim, L, J.reshape(dim, -1)[mu].astype(np.int64))
        h += Jm * np.roll(g, -1, axis=ax)                       # bond (i, i+e_mu)
        h += np.roll(Jm, 1, axis=ax) * np.roll(g, 1, axis=ax)   # bond (i-e_mu, i)
    return h.reshape(-1)


def colours(dim, L):
    idx = np.indices((L,) * dim).sum(axis=0)
    return (idx & 1).reshape(-1)


def energy(dim, L, J, s):
    return int(-(s.astype(np.int64) * local_field(dim, L, J, s)).sum() // 2)


def heis_field(dim, L, s):
    g = s.reshape((L,) * dim + (3,))
    h = np.zeros_like(g)
    for mu in range(dim):
        ax = axis_of(dim, mu)
        h += np.roll(g, -1, axis=ax) + np.roll(g, 1, axis=ax)
    return h.reshape(-1, 3)
