"""Exact balance properties of the oracle's updates on the 4x4 lattice.

Sec. 3.4 of the paper points out that the checkerboard sweep (all sites of
one colour, then all of the other) satisfies global balance but not
detailed balance, and that a palindromic sequence of the same single-colour
updates restores detailed balance.  On the 4x4 lattice (2^16 states) the
transfer matrices can be written down exactly:

* A single-colour update U_A (the sites of a set A of mutually
  non-adjacent sites, each attempted once, Eq. 2) moves state x to
  x xor m (m a subset of A) with probability prod_i p_i^{m_i} (1-p_i)^{1-m_i},
  where p_i = 1 if Delta E_i <= 0 and thr[Delta E_i / 4] / 2^32 otherwise:
  the oracle flips site i iff its 32-bit uniform u < thr, and u takes each of
  its 2^32 values with probability 2^-32.  That the oracle takes exactly these
  decisions, site by site, with the tabulated uniforms is pinned in
  test_oracle_streams.py; here the matrices are built from the oracle's
  thresholds and checked against the Boltzmann weights pi(x) ~ exp(-beta E(x)).
* The oracle's plain sweep is U_{colour 0} U_{colour 1}; its double
  checkerboard sweep with 2x2 tiles and k hits is
  (U_{00} U_{01})^k (U_{10} U_{11})^k with U_{tc} the sites of tile colour t
  and site colour c (its palindromic partner runs the same factors in reverse).

The integer thresholds bias an acceptance probability by less than 2^-32,
so the balance equations hold to a relative 1e-6 here (the printed bound
is checked), while the violations the paper predicts are of order one.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from tests import philox_ref as P
from tests.conftest import read_golden
import workloads as W

L = 4
N = 16
NS = 1 << N
IDX = np.arange(NS, dtype=np.int64)
BITS = ((IDX[:, None] >> np.arange(N)) & 1).astype(np.int8)
SPINS = (1 - 2 * BITS).astype(np.int64)          # bit i set <=> spin i = -1
X = np.arange(N) % L
Y = np.arange(N) // L
RIGHT = (X + 1) % L + L * Y
LEFT = (X - 1) % L + L * Y
UP = X + L * ((Y + 1) % L)
DOWN = X + L * ((Y - 1) % L)
SEED = W.seed_for(61)
TOL = 1e-6


def _couplings(ea):
    if not ea:
        return np.ones(N, np.int64), np.ones(N, np.int64)
    J = O.init_couplings(2, L, SEED, 2).astype(np.int64)
    return J[:N], J[N:]


def _energy(J0, J1):
    return -(SPINS * (J0 * SPINS[:, RIGHT] + J1 * SPINS[:, UP])).sum(axis=1)


def _delta_e(J0, J1):
    h = J0 * SPINS[:, RIGHT] + J0[LEFT] * SPINS[:, LEFT] + J1 * SPINS[:, UP] + J1[DOWN] * SPINS[:, DOWN]
    return 2 * SPINS * h                          # [NS, N]


def _pi(E, beta):
    w = np.exp(-beta * (E - E.min()))
    return w / w.sum()


class Update:
    """U_A as a dense [NS, 2^|A|] table of transition probabilities."""

    def __init__(self, sites, dE, beta, exact=False, downhill=1.0):
        self.sites = list(sites)
        thr = O.thresholds(beta, 2)
        p = np.ones((NS, len(self.sites)))
        for j, i in enumerate(self.sites):
            d = dE[:, i]
            p[d < 0, j] = downhill
            for m in (1, 2):
                sel = d == 4 * m
                p[sel, j] = math.exp(-beta * 4 * m) if exact else float(thr[m]) / 2.0 ** 32
        # column a of prob: the sites j with bit j of a set flip, the others stay
        masks = np.zeros(1, np.int64)
        prob = np.ones((NS, 1))
        for j, i in enumerate(self.sites):
            masks = np.concatenate([masks, masks | (1 << i)])
            prob = np.concatenate([prob * (1.0 - p[:, j:j + 1]), prob * p[:, j:j + 1]], axis=1)
        self.masks = masks
        self.prob = prob
        self.p = p

    # The sites of A are not neighbours, so p_i does not depend on the other
    # sites of A and U_A is the product of the single-site updates U_i
    # (x -> x with 1 - p_i(x), x -> x ^ bit_i with p_i(x)) in any order;
    # vectors are moved through those factors.

    def row(self, v):
        """v U (v a distribution over states)."""
        for j, i in enumerate(self.sites):
            moved = v * self.p[:, j]
            v = v - moved + moved[IDX ^ (1 << i)]
        return v

    def col(self, f):
        """U f (f a function of states)."""
        for j, i in reversed(list(enumerate(self.sites))):
            f = f + self.p[:, j] * (f[IDX ^ (1 << i)] - f)
        return f


def _row(updates, v):
    for u in updates:
        v = u.row(v)
    return v


def _col(updates, f):
    for u in reversed(updates):
        f = u.col(f)
    return f


def _db_violation(updates, pi, states):
    """max over the given x and all y of |pi(x) K(x,y) - pi(y) K(y,x)|,
    relative to max pi(x) K(x,y), for K the product of the updates."""
    worst = 0.0
    for x in states:
        e = np.zeros(NS)
        e[x] = 1.0
        fwd = pi[x] * _row(updates, e)            # pi(x) K(x, .)
        bwd = pi * _col(updates, e)               # pi(.) K(., x)
        worst = max(worst, np.abs(fwd - bwd).max() / fwd.max())
    return worst


def _sites(colour, tile_colour=None):
    c = (X + Y) & 1
    sel = c == colour
    if tile_colour is not None:
        sel &= ((X // 2 + Y // 2) & 1) == tile_colour
    return np.nonzero(sel)[0]


CASES = [(False, 0.3), (False, W.BETA_C_2D), (False, 0.6), (True, 0.7)]
TEST_STATES = [0, 0b1010010110100101, 0x1234, 0xBEEF]


@pytest.fixture(scope="module", params=CASES, ids=["ising-0.3", "ising-bc", "ising-0.6", "ea-0.7"])
def system(request):
    ea, beta = request.param
    J0, J1 = _couplings(ea)
    E = _energy(J0, J1)
    dE = _delta_e(J0, J1)
    pi = _pi(E, beta)
    U = [Update(_sites(c), dE, beta) for c in (0, 1)]
    return dict(ea=ea, beta=beta, J0=J0, J1=J1, E=E, dE=dE, pi=pi, U=U)


def test_threshold_bias_below_two_to_minus_32(system):
    beta = system["beta"]
    thr = O.thresholds(beta, 2)
    for m in (1, 2):
        assert 0 <= math.exp(-beta * 4 * m) - float(thr[m]) / 2.0 ** 32 < 2.0 ** -32


def test_single_colour_updates_are_stochastic_and_detailed_balanced(system):
    pi = system["pi"]
    for U in system["U"]:
        np.testing.assert_allclose(U.prob.sum(axis=1), 1.0, rtol=0, atol=1e-12)
        # pi(x) U(x, x^m) = pi(x^m) U(x^m, x) for every x and every subset m
        for a, m in enumerate(U.masks):
            lhs = pi * U.prob[:, a]
            rhs = pi[IDX ^ m] * U.prob[IDX ^ m, a]
            assert np.all(np.abs(lhs - rhs) <= TOL * np.maximum(lhs, rhs) + 1e-300)
        # hence pi is stationary
        np.testing.assert_allclose(U.row(pi), pi, rtol=TOL, atol=0)


def test_sweep_is_globally_but_not_detailed_balanced(system):
    """P = U_0 U_1: pi P = pi, but pi(x) P(x,y) != pi(y) P(y,x) (Sec. 3.4)."""
    pi, U = system["pi"], system["U"]
    np.testing.assert_allclose(_row(U, pi), pi, rtol=TOL, atol=0)
    assert _db_violation(U, pi, TEST_STATES) > 1e-2


def test_palindrome_is_detailed_balanced(system):
    """U_0 U_1 U_1 U_0 (a sweep followed by its mirror image) is reversible."""
    pi, (U0, U1) = system["pi"], system["U"]
    assert _db_violation([U0, U1, U1, U0], pi, TEST_STATES) < TOL
    assert _db_violation([U1, U0, U0, U1], pi, TEST_STATES) < TOL


def test_the_exact_boltzmann_rule_balances_to_rounding(system):
    """The same construction with p = exp(-beta Delta E) in float64 balances to
    1e-12: the 1e-6 tolerance above only covers the integer table's bias."""
    pi = system["pi"]
    U = [Update(_sites(c), system["dE"], system["beta"], exact=True) for c in (0, 1)]
    np.testing.assert_allclose(_row(U, pi), pi, rtol=1e-12, atol=0)
    assert _db_violation(U + U[::-1], pi, TEST_STATES[:2]) < 1e-12


def test_a_wrong_rule_is_caught():
    """The checks have power: accepting downhill moves with probability 1/2
    breaks stationarity by far more than the tolerance."""
    J0, J1 = _couplings(False)
    E, dE = _energy(J0, J1), _delta_e(J0, J1)
    pi = _pi(E, 0.4)
    U = Update(_sites(0), dE, 0.4, downhill=0.5)
    np.testing.assert_allclose(U.prob.sum(axis=1), 1.0, rtol=0, atol=1e-12)
    assert np.abs(U.row(pi) - pi).max() / pi.max() > 1e-2


# ---------------------------------------------------------------------------
# Double checkerboard with 2x2 tiles (Sec. 3.2 order, Sec. 3.4 hits).

@pytest.mark.parametrize("k", [1, 2])
def test_tiled_compound_move_balance(system, k):
    pi, dE, beta = system["pi"], system["dE"], system["beta"]
    U = {(t, c): Update(_sites(c, t), dE, beta) for t in (0, 1) for c in (0, 1)}
    fwd = [U[0, 0], U[0, 1]] * k + [U[1, 0], U[1, 1]] * k
    rev = fwd[::-1]
    np.testing.assert_allclose(_row(fwd, pi), pi, rtol=TOL, atol=0)
    assert _db_violation(fwd, pi, TEST_STATES) > 1e-2
    assert _db_violation(fwd + rev, pi, TEST_STATES) < TOL


def _table():
    return {int(r[1]): r[1:] for r in read_golden("stream_layout_4x4.txt") if r[0] == "M2"}


def _u32(row, seed, t, r):
    _, _, _, _, _, _, hc0, htag, hw, half, tc0, ttag = row
    w = P.seeded(seed, [int(hc0), t, r, int(htag)])[int(hw)]
    head = (w >> 16) if half == "hi" else (w & 0xFFFF)
    return (head << 16) | (P.seeded(seed, [int(tc0), t, r, int(ttag)])[0] & 0xFFFF)


def _apply(s, J0, J1, sites, thr, seed, t, r, table):
    """One single-colour update of the listed sites with the tabulated uniforms."""
    s = s.astype(np.int64).copy()
    for i in sites:
        h = J0[i] * s[RIGHT[i]] + J0[LEFT[i]] * s[LEFT[i]] + J1[i] * s[UP[i]] + J1[DOWN[i]] * s[DOWN[i]]
        d = 2 * s[i] * h
        if d <= 0 or _u32(table[i], seed, t, r) < int(thr[d // 4]):
            s[i] = -s[i]
    return s


@pytest.mark.parametrize("ea", [False, True])
@pytest.mark.parametrize("k,palindromic", [(1, False), (2, False), (1, True), (3, True)])
def test_oracle_tiled_run_is_the_product_of_updates(ea, k, palindromic):
    """orc_dcb_run with 2x2 tiles applies exactly the factors above, in that
    order, hit j of sweep t with the uniforms of plain sweep t k + j."""
    J0, J1 = _couplings(ea)
    J = None if not ea else np.concatenate([J0, J1]).astype(np.int8)
    table = _table()
    beta, r = 0.35, 3
    thr = O.thresholds(beta, 2)
    s = O.init_spins(2, L, SEED, r)
    want = s.astype(np.int64)
    for t in range(4):
        got = s.copy()
        O.dcb_run(L, 2, k, J, got, beta, SEED, r, t, 1, palindromic)
        rev = palindromic and (t & 1)
        for tc in ((1, 0) if rev else (0, 1)):
            for j in range(k):
                for c in ((1, 0) if rev else (0, 1)):
                    want = _apply(want, J0, J1, _sites(c, tc), thr, SEED, t * k + j, r, table)
        assert np.array_equal(got.astype(np.int64), want), (t, k, palindromic)
        s = got


@pytest.mark.parametrize("colour", [0, 1])
def test_oracle_half_sweep_samples_the_matrix_row(colour):
    """From fixed states, the successors of 20 000 half-sweeps (sweeps 0 ..
    19 999) follow the row U_c(x, .) of the exact matrix (chi^2 over the 256
    successor patterns): the eight sites' uniforms act as independent."""
    J0, J1 = _couplings(True)
    J = np.concatenate([J0, J1]).astype(np.int8)
    dE = _delta_e(J0, J1)
    beta = 0.25
    U = Update(_sites(colour), dE, beta)
    for x in (0x1234, 0xF0F0):
        s0 = SPINS[x].astype(np.int8)
        counts = np.zeros(len(U.masks))
        lookup = {int(m): a for a, m in enumerate(U.masks)}
        n = 20000
        for t in range(n):
            s = s0.copy()
            O.half_sweep(2, L, J, s, beta, SEED, 1, t, colour)
            flipped = int(((s != s0).astype(np.int64) << np.arange(N)).sum())
            counts[lookup[flipped]] += 1
        expect = n * U.prob[x]
        keep = expect > 5
        chi2 = ((counts[keep] - expect[keep]) ** 2 / expect[keep]).sum()
        dof = int(keep.sum()) - 1
        assert counts[~keep].sum() <= max(10.0, 3 * expect[~keep].sum())
        assert chi2 < dof + 6 * math.sqrt(2 * dof), (x, chi2, dof)
