"""The 2D Ising workload at its full size (16384^2, the benchmark's launch
configuration): sampled sites bit-exact against the oracle's window sweep,
tracked energies against measurement, and the equilibrium values against
Onsager's energy and Yang's spontaneous magnetisation."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1101_1427_amd as S
import workloads as W
from oracle import exact as X
from oracle import oracle as O

pytestmark = pytest.mark.gpu

DEV = "cuda"
CFG = W.ising_large()
L = CFG.L
N = L * L


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module")
def start():
    """The oracle's random start of replica 0 (independent of the GPU)."""
    return O.init_spins(2, L, CFG.seed, 0).reshape(L, L)


def _window(a, x0, y0, Wd):
    return np.ascontiguousarray(a[np.ix_([(y0 + v) % L for v in range(Wd)], [(x0 + u) % L for u in range(Wd)])])


@pytest.mark.parametrize("beta", CFG.betas)
def test_sampled_windows_bit_exact(start, beta):
    """8 sweeps of the whole lattice on the GPU; the centres of eight 96 x 96
    windows (corners, band edges, random places) equal the oracle's."""
    b = S.Batch(S.ISING, 2, L, 1, CFG.seed)
    assert S.sweep_plan(b) == (1, "k_ising2d_split")
    spins = torch.empty(N, dtype=torch.int8, device=DEV)
    S.spin_init(b, spins)
    dE = torch.zeros(1, dtype=torch.int64, device=DEV)
    n, Wd = 8, 96
    S.metropolis_sweep(b, spins, [beta], 5, n, dE_accum=dE)
    got = _host(spins).reshape(L, L)
    rng = np.random.default_rng(int(beta * 1000))
    places = [(0, 0), (L - 40, L - 40), (100, 32 - 48), (8000, 8192 - 48), (L - 48, 1000)]
    places += [tuple(int(v) for v in rng.integers(0, L, 2)) for _ in range(3)]
    m = 2 * n + 1
    for x0, y0 in places:
        x0 %= L
        y0 %= L
        win = _window(start, x0, y0, Wd)
        O.window_run(L, x0, y0, win, beta, CFG.seed, 0, 5, n)
        assert np.array_equal(_window(got, x0, y0, Wd)[m:Wd - m, m:Wd - m], win[m:Wd - m, m:Wd - m]), (x0, y0)
    # tracked energy change against a measurement of the final lattice
    E = torch.zeros(1, dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E)
    E0 = O.energy(2, L, None, start.reshape(-1))
    assert float(_host(E)[0]) == float(E0 + int(_host(dE)[0]))


def test_onsager_energy_at_beta_030():
    """Random start, 300 sweeps at beta = 0.30: energy per spin within 1e-3 of
    Onsager's infinite-lattice value."""
    b = S.Batch(S.ISING, 2, L, 1, CFG.seed)
    spins = torch.empty(N, dtype=torch.int8, device=DEV)
    S.spin_init(b, spins)
    S.metropolis_sweep(b, spins, [0.30], 0, 300)
    E = torch.zeros(1, dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E)
    assert abs(float(_host(E)[0]) / N - X.onsager_energy(0.30)) < 1e-3


def test_yang_magnetisation_at_beta_050_cold_start():
    """All spins up, 300 sweeps at beta = 0.50: magnetisation per spin within
    1e-3 of Yang's spontaneous magnetisation, energy within 1e-3 of Onsager's."""
    b = S.Batch(S.ISING, 2, L, 1, CFG.seed)
    spins = torch.ones(N, dtype=torch.int8, device=DEV)
    S.metropolis_sweep(b, spins, [0.50], 0, 300)
    E = torch.zeros(1, dtype=torch.float64, device=DEV)
    M = torch.zeros(1, dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E, M)
    assert abs(abs(float(_host(M)[0])) / N - X.yang_magnetisation(0.50)) < 1e-3
    assert abs(float(_host(E)[0]) / N - X.onsager_energy(0.50)) < 1e-3
