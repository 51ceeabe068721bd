"""The window sweep of the oracle (used for sampled-site parity of large
lattices) against the full-lattice oracle: inside the light cone every site
equals the full run, at the ring it does not."""
import numpy as np
import pytest

from oracle import oracle as O


def _window(full, L, x0, y0, W):
    return np.ascontiguousarray(full[np.ix_([(y0 + v) % L for v in range(W)], [(x0 + u) % L for u in range(W)])])


@pytest.mark.parametrize("L,x0,y0,W,beta,t0,n", [
    (64, 50, 40, 40, 0.44, 3, 5),      # window wrapping both axes
    (64, 0, 0, 30, 0.30, 0, 4),
    (48, 7, 33, 48, 0.60, 11, 6),      # window as large as the lattice
    (32, 31, 31, 24, 0.2, 2, 3),
])
def test_window_interior_equals_full_lattice(L, x0, y0, W, beta, t0, n):
    seed = 0x1101142700000077
    s0 = O.init_spins(2, L, seed, 3).reshape(L, L)
    full = s0.copy()
    O.run(2, L, None, full.reshape(-1), beta, seed, 3, t0, n)
    win = _window(s0, L, x0, y0, W)
    O.window_run(L, x0, y0, win, beta, seed, 3, t0, n)
    m = 2 * n + 1
    assert np.array_equal(win[m:W - m, m:W - m], _window(full, L, x0, y0, W)[m:W - m, m:W - m])


def test_window_edge_is_not_the_full_lattice():
    """The held ring makes the window differ from the full run near its edge
    (the comparison region above is a real restriction)."""
    L, W, n, seed = 64, 40, 6, 0x1101142700000078
    s0 = O.init_spins(2, L, seed, 0).reshape(L, L)
    full = s0.copy()
    O.run(2, L, None, full.reshape(-1), 0.3, seed, 0, 0, n)
    win = _window(s0, L, 5, 9, W)
    O.window_run(L, 5, 9, win, 0.3, seed, 0, 0, n)
    ref = _window(full, L, 5, 9, W)
    assert not np.array_equal(win[1:4, 1:W - 1], ref[1:4, 1:W - 1])
