"""Table 1 with the Philox streams at reduced statistics: the internal
energy and specific heat of the 1024^2 Ising model at beta = 0.4 from the
plain checkerboard sweep and the double checkerboard agree with the exact
finite-size values (Kaufman) within 4.5 standard errors."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import bench
import paper_1101_1427_amd as S
import workloads as W
from oracle import exact as X

pytestmark = pytest.mark.gpu

DEV = "cuda"
L, BETA, N_REP = 1024, 0.4, 16


@pytest.fixture(scope="module")
def exact():
    return X.kaufman_thermo(BETA, L)


def _start(seed):
    b = S.Batch(S.ISING, 2, L, N_REP, seed)
    spins = torch.empty(N_REP * L * L, dtype=torch.int8, device=DEV)
    S.spin_init(b, spins)
    S.metropolis_sweep(b, spins, [BETA] * N_REP, 0, 300)
    E0 = torch.empty(N_REP, dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E0)
    return b, spins, E0


def _check(E, exact):
    e, de, c, dc = bench._e_and_c(E, L * L, BETA)
    assert abs(e - exact["e"]) < 4.5 * de, (e, de, exact["e"])
    assert abs(c - exact["C"]) < 4.5 * dc, (c, dc, exact["C"])
    assert de < 6e-5 and dc < 6e-2  # the statistics the check claims


def test_checkerboard_sweep(exact):
    b, spins, E0 = _start(W.seed_for(98))
    dE = torch.zeros(N_REP, dtype=torch.int64, device=DEV)
    calls, every = 600, 4
    trace = torch.empty(calls, N_REP, dtype=torch.int64, device=DEV)
    for i in range(calls):
        S.metropolis_sweep(b, spins, [BETA] * N_REP, 300 + i * every, every, dE_accum=dE)
        trace[i].copy_(dE)
    _check((E0.cpu().numpy()[None, :] + trace.cpu().numpy()).T, exact)


def test_double_checkerboard(exact):
    b, spins, E0 = _start(W.seed_for(99))
    n = 2400
    trace = torch.empty(n, N_REP, dtype=torch.int64, device=DEV)
    S.dcb_sweep(b, spins, [BETA] * N_REP, 300, n, 64, 1, dE_trace=trace)
    _check((E0.cpu().numpy()[None, :] + trace.cpu().numpy()).T, exact)
