"""Exact reference results used to pin the oracle (TEST INFRASTRUCTURE ONLY).

Nothing here shares code with the oracle's C file or the GPU library; every
result is computed from its own closed form or by brute force:

* ``enumerate_states``: all 2^N states of a small periodic Ising / +-J lattice
  (Eqs. 1 and 11), giving E and M of every state.
* ``onsager_energy`` / ``yang_magnetisation``: infinite-lattice 2D Ising
  closed forms (the exact transition point is quoted in Sec. 3.4).
* ``kaufman_*``: exact finite-size partition function of the L x L torus
  (Kaufman 1949, Ferdinand and Fisher 1969), the source of the exact
  reference values printed in Table 1.
* ``ising_highT_energy`` / ``heis_tree_energy``: leading high-temperature
  behaviour of the Ising and O(3) models on the simple (hyper)cubic lattice.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

BETA_C_2D = 0.5 * math.log(1.0 + math.sqrt(2.0))


# ----------------------------------------------------------------------
# brute-force enumeration
# ----------------------------------------------------------------------
def bonds(dim: int, L: int):
    """(i, j, mu) for every bond i -> i + e_mu of the periodic lattice."""
    out = []
    shape = (L,) * dim
    for coord in itertools.product(range(L), repeat=dim):
        # coord is (z, y, x) ordering -> site index with x fastest
        i = int(np.ravel_multi_index(coord, shape))
        for mu in range(dim):
            c2 = list(coord)
            axis = dim - 1 - mu  # mu = 0 is x (last axis)
            c2[axis] = (c2[axis] + 1) % L
            j = int(np.ravel_multi_index(tuple(c2), shape))
            out.append((i, j, mu))
    return out


def enumerate_states(dim: int, L: int, J: np.ndarray | None = None):
    """E and M of all 2^N states; state bit i = 1 means s_i = -1.

    J (optional) is int8 [dim][N]: J[mu][i] is the bond i -> i + e_mu.
    """
    N = L ** dim
    assert N <= 24, "enumeration only for tiny lattices"
    states = np.arange(1 << N, dtype=np.int64)
    spins = 1 - 2 * ((states[:, None] >> np.arange(N)[None, :]) & 1)  # [2^N, N] of +-1
    E = np.zeros(1 << N, np.int64)
    for i, j, mu in bonds(dim, L):
        jij = 1 if J is None else int(J.reshape(dim, N)[mu, i])
        E -= jij * spins[:, i] * spins[:, j]
    M = spins.sum(axis=1)
    return E, M


def boltzmann_averages(E: np.ndarray, M: np.ndarray, beta: float):
    """<E>, <E^2>, <|M|>, <M^2> and Z for the enumerated states."""
    Ef = E.astype(np.float64)
    w = np.exp(-beta * (Ef - Ef.min()))
    Z = w.sum()
    p = w / Z
    return {
        "E": float((p * Ef).sum()),
        "E2": float((p * Ef * Ef).sum()),
        "absM": float((p * np.abs(M)).sum()),
        "M2": float((p * M.astype(np.float64) ** 2).sum()),
        "lnZ": float(np.log(Z) - beta * Ef.min()),
    }


def density_of_states(E: np.ndarray):
    levels, counts = np.unique(E, return_counts=True)
    return levels, counts


# ----------------------------------------------------------------------
# infinite-lattice 2D Ising closed forms
# ----------------------------------------------------------------------
def _ellipk_modulus(k: float) -> float:
    """Complete elliptic integral of the first kind K(k) (modulus k) via AGM."""
    a, b = 1.0, math.sqrt(1.0 - k * k)
    for _ in range(64):
        a, b = 0.5 * (a + b), math.sqrt(a * b)
        if abs(a - b) < 1e-17 * a:
            break
    return math.pi / (2.0 * a)


def onsager_energy(beta: float) -> float:
    """Energy per spin u = E/N of the infinite square-lattice Ising model (J = 1)."""
    t = 2.0 * beta
    kappa = 2.0 * math.sinh(t) / math.cosh(t) ** 2
    if abs(kappa - 1.0) < 1e-15:
        return -math.sqrt(2.0)
    K = _ellipk_modulus(kappa)
    return -(1.0 / math.tanh(t)) * (1.0 + (2.0 / math.pi) * (2.0 * math.tanh(t) ** 2 - 1.0) * K)


def yang_magnetisation(beta: float) -> float:
    """Spontaneous magnetisation per spin (0 for beta <= beta_c)."""
    if beta <= BETA_C_2D:
        return 0.0
    return (1.0 - math.sinh(2.0 * beta) ** -4) ** 0.125


# ----------------------------------------------------------------------
# exact finite-size torus (Kaufman; Ferdinand & Fisher)
# ----------------------------------------------------------------------
def kaufman_lnZ(K, L: int, mp):
    """ln Z of the L x L periodic Ising model at coupling K (mpmath number)."""
    n = m = L
    c2 = mp.cosh(2 * K) / mp.tanh(2 * K)  # cosh 2K coth 2K

    def gamma(l):
        if l == 0:
            return 2 * K + mp.log(mp.tanh(K))
        return mp.acosh(c2 - mp.cos(mp.pi * l / n))

    g_odd = [gamma(2 * r + 1) for r in range(n)]
    g_even = [gamma(2 * r) for r in range(n)]

    def logprod(vals, fn):
        sign = 1
        acc = mp.mpf(0)
        for v in vals:
            x = 2 * fn(m * v / 2)
            if x < 0:
                sign = -sign
                x = -x
            acc += mp.log(x)
        return sign, acc

    terms = [logprod(g_odd, mp.cosh), logprod(g_odd, mp.sinh),
             logprod(g_even, mp.cosh), logprod(g_even, mp.sinh)]
    big = max(t[1] for t in terms)
    s = mp.fsum(sign * mp.exp(lg - big) for sign, lg in terms)
    return mp.log(mp.mpf(1) / 2) + (mp.mpf(n * m) / 2) * mp.log(2 * mp.sinh(2 * K)) + big + mp.log(s)


def kaufman_thermo(beta: float, L: int, dps: int = 40):
    """Exact e = -E/N (the sign printed in Table 1), C_V per spin and ln Z / N."""
    import mpmath as mp

    with mp.workdps(dps):
        K = mp.mpf(beta)
        f = lambda k: kaufman_lnZ(k, L, mp)
        N = L * L
        d1 = mp.diff(f, K, 1)
        d2 = mp.diff(f, K, 2)
        return {"e": float(d1 / N), "C": float(K * K * d2 / N), "lnZ_per_site": float(f(K) / N)}


# ----------------------------------------------------------------------
# high-temperature behaviour
# ----------------------------------------------------------------------
def ising_highT_energy(beta: float, dim: int) -> float:
    """E/N of the d-dim simple-cubic Ising model to order t^3, t = tanh(beta).

    ln Z/N = ln 2 + d ln cosh(beta) + (d(d-1)/2) t^4 + O(t^6): the only closed
    graphs of 4 bonds are the elementary plaquettes, d(d-1)/2 per site.
    """
    t = math.tanh(beta)
    return -dim * t - 2.0 * dim * (dim - 1) * t ** 3 * (1.0 - t * t)


def langevin(beta: float) -> float:
    """<s_i . s_j> of two O(3) unit vectors coupled only to each other."""
    return 1.0 / math.tanh(beta) - 1.0 / beta


def heis_tree_energy(beta: float, dim: int) -> float:
    """E/N of the O(3) model neglecting closed loops: -d L(beta).

    The first loop correction (elementary plaquettes) is O(L(beta)^4) per bond.
    """
    return -dim * langevin(beta)


def heis_acceptance_probability(a: np.ndarray, H: np.ndarray, beta: float) -> np.ndarray:
    """Mean Metropolis acceptance of a uniform-on-sphere proposal s'.

    For a spin with a = s.h and H = |h|, the projection b = s'.h of a uniform
    direction is uniform on [-H, H], and Delta E = a - b, so
      P = (1/2H) [ (H - a) + (1 - exp(-beta (a + H))) / beta ].
    """
    a = np.asarray(a, np.float64)
    H = np.asarray(H, np.float64)
    if beta == 0.0:
        return np.ones_like(a)
    return ((H - a) + (1.0 - np.exp(-beta * (a + H))) / beta) / (2.0 * H)
