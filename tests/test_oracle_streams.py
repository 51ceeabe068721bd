"""Pins of the oracle's random-number stream layout (which Philox counter,
word and 16-bit half feed each site, bond, move and exchange).

The layout is a definition, so it is pinned against a table written out by
hand for a 4x4 lattice (and sites of a 4x4x4 one) in
tests/golden/stream_layout_4x4.txt, evaluated with a second Philox written
in Python from the generator's published round definition
(tests/philox_ref.py).  A misreading of the layout in the oracle (a counter
word swapped, the wrong half, a colour or in-colour index off by one) makes
one of these tests fail even though the GPU path would copy it.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

from oracle import oracle as O
from tests import npref
from tests import philox_ref as P
from tests.conftest import read_golden
import workloads as W

SEEDS = [W.seed_for(3), 0xFFFFFFFF00000001, 0x0123456789ABCDEF]


def _rows(kind):
    return [r[1:] for r in read_golden("stream_layout_4x4.txt") if r[0] == kind]


def test_python_philox_known_answers():
    for row in read_golden("philox4x32_10_kat.txt"):
        v = [int(x, 16) for x in row]
        assert P.block(v[0:4], v[4:6]) == v[6:10]


def test_python_philox_equals_oracle_block():
    rng = np.random.default_rng(7)
    for _ in range(50):
        ctr = [int(x) for x in rng.integers(0, 1 << 32, 4, dtype=np.uint64)]
        key = [int(x) for x in rng.integers(0, 1 << 32, 2, dtype=np.uint64)]
        assert P.block(ctr, key) == [int(x) for x in O.philox(ctr, key)]


def test_uniform_maps_worked_examples():
    """unit23 / unit53 against values worked out by hand (exact decimals)."""
    getcontext().prec = 80
    for w0, w1, val in _rows("U23") + _rows("U53"):
        got = P.unit23(int(w0, 16)) if w1 == "-" else P.unit53(int(w0, 16), int(w1, 16))
        assert Decimal(got) == Decimal(val), (w0, w1)


def _head_tail_u32(seed, t, r, row):
    _, _, _, _, _, _, hc0, htag, hw, half, tc0, ttag = row
    head_block = P.seeded(seed, [int(hc0), t, r, int(htag)])
    word = head_block[int(hw)]
    head = (word >> 16) if half == "hi" else (word & 0xFFFF)
    tail = P.seeded(seed, [int(tc0), t, r, int(ttag)])[0] & 0xFFFF
    return (head << 16) | tail


@pytest.mark.parametrize("kind,dim", [("M2", 2), ("M3", 3)])
def test_metropolis_uniform_layout(kind, dim):
    """orc_metropolis_u32(colour, h) equals the head/tail composition of the
    tabulated counters, and the tabulated colour and h follow from (x, y, z)."""
    for seed in SEEDS:
        for t, r in [(0, 0), (5, 2), (0xFFFFFFFF, 77)]:
            for row in _rows(kind):
                i, x, y, z, c, h = (int(v) for v in row[:6])
                assert i == (x + 4 * y + 16 * z) and c == (x + y + z) % 2 and h == i // 2
                want = _head_tail_u32(seed, t, r, row)
                assert O.metropolis_u32(seed, t, r, c, h) == want, (seed, t, r, row)


def _threshold(beta, m):
    """floor(2^32 exp(-4 m beta)) in 50-digit arithmetic (Sec. 3.5 table)."""
    getcontext().prec = 50
    return int(Decimal(2) ** 32 * (Decimal(-4 * m) * Decimal(beta)).exp())


def _predict_half_sweep(dim, J, s, beta, seed, t, r, c, table):
    """The flips of a colour-c half-sweep predicted from the table alone:
    Delta E from numpy shifts, u from the tabulated counters, flip iff
    Delta E <= 0 or u < thr (Eq. 2 with the integer table).  Sites missing
    from the table are reported as unknown (-1 in the mask)."""
    h = npref.local_field(dim, 4, J, s)
    dE = 2 * s.astype(np.int64) * h
    flip = np.full(s.size, -1, np.int64)
    for row in table:
        i, cc = int(row[0]), int(row[4])
        if cc != c:
            continue
        if dE[i] <= 0:
            flip[i] = 1
        else:
            flip[i] = int(_head_tail_u32(seed, t, r, row) < _threshold(beta, int(dE[i]) // 4))
    return flip


@pytest.mark.parametrize("model", [W.MODEL_ISING, W.MODEL_EA])
@pytest.mark.parametrize("kind,dim", [("M2", 2), ("M3", 3)])
def test_half_sweep_decisions_follow_the_table(model, kind, dim):
    """Each half-sweep of the oracle flips exactly the tabulated sites whose
    tabulated uniform is below the threshold; beta is chosen so that about half
    of the uphill moves are accepted, which makes every decision informative."""
    table = _rows(kind)
    n_checked = 0
    for seed in SEEDS[:2]:
        J = O.init_couplings(dim, 4, seed, 3) if model == W.MODEL_EA else None
        for r in (0, 9):
            s = O.init_spins(dim, 4, seed, r)
            for t in range(6):
                beta = math.log(2.0) / 8.0 if t % 2 == 0 else 0.09
                for c in (0, 1):
                    want = _predict_half_sweep(dim, J, s, beta, seed, t, r, c, table)
                    before = s.copy()
                    O.half_sweep(dim, 4, J, s, beta, seed, r, t, c)
                    changed = (s != before).astype(np.int64)
                    known = want >= 0
                    assert np.array_equal(changed[known], want[known]), (seed, r, t, c)
                    n_checked += int(known.sum())
                    # sites of the other colour never change
                    col = npref.colours(dim, 4)
                    assert not np.any(changed[col != c])
    assert n_checked > 100


def test_random_start_layout():
    for seed in SEEDS:
        for r in (0, 1, 1000):
            s = O.init_spins(2, 4, seed, r)
            for i, c0, w in (tuple(int(v) for v in row) for row in _rows("I")):
                word = P.seeded(seed, [c0, 0, r, 2])[w]
                assert s[i] == (-1 if word >> 31 else 1), (seed, r, i)


@pytest.mark.parametrize("kind,dim", [("J2", 2), ("J3", 3)])
def test_coupling_layout(kind, dim):
    N = 4 ** dim
    for seed in SEEDS:
        for q in (0, 5):
            J = O.init_couplings(dim, 4, seed, q)
            for i, mu, c0, w in (tuple(int(v) for v in row) for row in _rows(kind)):
                assert c0 == (dim * i + mu) // 4 and w == (dim * i + mu) % 4
                word = P.seeded(seed, [c0, 0, q, 4])[w]
                assert J[mu * N + i] == (-1 if word >> 31 else 1), (seed, q, i, mu)


def _sphere(u0, u1):
    z = 2.0 * u0 - 1.0
    rho = math.sqrt(1.0 - z * z)
    return np.array([rho * math.cos(2 * math.pi * u1), rho * math.sin(2 * math.pi * u1), z])


def test_heisenberg_start_layout():
    for seed in SEEDS:
        s = O.init_heis(2, 4, seed, 6)
        for i, c0 in (tuple(int(v) for v in row) for row in _rows("H0")):
            w = P.seeded(seed, [c0, 0, 6, 2])
            u0, u1 = P.unit23(w[0]), P.unit23(w[1])
            assert s[i, 2] == 2.0 * u0 - 1.0            # exact: z is a dyadic rational
            np.testing.assert_allclose(s[i], _sphere(u0, u1), rtol=0, atol=1e-15)


def test_heisenberg_move_layout():
    """At beta = 0 every proposal is accepted, so after a half-sweep each site
    of the colour holds the point of words 0, 1 of its tabulated draw; at a
    finite beta the tabulated word 2 decides (sites near a tie skipped)."""
    seed, r = SEEDS[0], 4
    for t in (0, 3):
        s = O.init_heis(2, 4, seed, r)
        for c in (0, 1):
            O.heis_half_sweep(2, 4, s, 0.0, seed, r, t, c)
        for i, col, c0, c3 in (tuple(int(v) for v in row) for row in _rows("HM")):
            w = P.seeded(seed, [c0, t, r, c3])
            np.testing.assert_allclose(s[i], _sphere(P.unit23(w[0]), P.unit23(w[1])), rtol=0, atol=1e-15)
    decided = 0
    for t in range(40):
        s = O.init_heis(2, 4, seed, r)
        before = s.copy()
        for c in (0, 1):
            field = npref.heis_field(2, 4, s)
            O.heis_half_sweep(2, 4, s, 1.3, seed, r, t, c)
            for i, col, c0, c3 in (tuple(int(v) for v in row) for row in _rows("HM")):
                if col != c:
                    continue
                w = P.seeded(seed, [c0, t, r, c3])
                sp = _sphere(P.unit23(w[0]), P.unit23(w[1]))
                dE = -float(np.dot(sp - before[i], field[i]))
                p = 1.0 if dE <= 0 else math.exp(-1.3 * dE)
                u = P.unit23(w[2])
                if abs(u - p) < 1e-9:
                    continue
                moved = not np.array_equal(s[i], before[i])
                assert moved == (u < p), (t, i)
                decided += 1
            before = s.copy()
    assert decided > 100


def test_exchange_uniform_layout():
    for seed in SEEDS:
        for t, q in [(0, 0), (17, 3), (0xFFFFFFFE, 1023)]:
            for k, c0, c3 in (tuple(int(v) for v in row) for row in _rows("S")):
                w = P.seeded(seed, [c0, t, q, c3])
                assert O.swap_u53(seed, k, t, q) == P.unit53(w[0], w[1])


def test_acceptance_is_strict_at_an_exact_tie():
    """u < thr is strict: with beta chosen so that the threshold of an uphill
    move equals that site's uniform exactly the move is refused, and with the
    threshold one above it the move is taken (Eq. 2 with the integer table)."""
    seed, r, t = SEEDS[0], 2, 11
    row = _rows("M2")[0]                      # site 0: colour 0, h = 0
    u = _head_tail_u32(seed, t, r, row)
    for target, flips in ((u, False), (u + 1, True)):
        beta = -math.log((target + 0.5) / 2.0 ** 32) / 8.0
        assert _threshold(beta, 2) == target
        s = np.ones(16, np.int8)              # all up: Delta E = 8 at every site
        O.half_sweep(2, 4, None, s, beta, seed, r, t, 0)
        assert (s[0] == -1) == flips
