"""The GPU sweeps against exact results directly (not through the oracle):
4096 replicas of the 4 x 4 periodic Ising model and of one 4 x 4 +-J sample,
time averages of E, E^2, |M| and M^2 against the exact Boltzmann averages of
all 2^16 states (Eq. 1 with the Metropolis rule of Eq. 2 as its stationary
law), and the exchange acceptance of 4096 tempering chains against its exact
double sum over the density of states.  With 4096 independent replicas the
standard errors are about six times smaller than in the oracle's own tests."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1101_1427_amd as S
import workloads as W
from oracle import exact as X
from oracle import oracle as O

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _series(model, beta, n_rep, seed, sweeps=2000, burn=100, every=10):
    """Per replica, the time series of E and M (every `every` sweeps after
    `burn`); float64 [n_rep, samples]."""
    L = 4
    b = S.Batch(model, 2, L, n_rep, seed, rep_per_sample=n_rep)
    spins = torch.zeros(n_rep * L * L, dtype=torch.int8, device=DEV)
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV) if model == S.EA else None
    S.spin_init(b, spins, coup)
    betas = [beta] * n_rep
    S.metropolis_sweep(b, spins, betas, 0, burn, couplings=coup)
    n = (sweeps - burn) // every
    E = torch.zeros((n, n_rep), dtype=torch.float64, device=DEV)
    M = torch.zeros((n, n_rep), dtype=torch.float64, device=DEV)
    t = burn
    for k in range(n):
        S.metropolis_sweep(b, spins, betas, t, every, couplings=coup)
        t += every
        S.measure_energy_magnetisation(b, spins, E[k], M[k], couplings=coup)
    torch.cuda.synchronize()
    return E.cpu().numpy().T, M.cpu().numpy().T, (coup.cpu().numpy() if coup is not None else None)


def _check(Es, Ms, ex, keys, tag):
    for key in keys:
        vals = {"E": Es, "E2": Es ** 2, "absM": np.abs(Ms), "M2": Ms ** 2}[key]
        per_rep = vals.mean(axis=1)
        mean, err = per_rep.mean(), per_rep.std(ddof=1) / math.sqrt(len(per_rep))
        assert abs(mean - ex[key]) < 4.5 * err, (tag, key, mean, ex[key], err)


@pytest.mark.parametrize("beta", [0.3, W.BETA_C_2D, 0.6])
def test_4x4_ising_many_replicas_match_enumeration(beta):
    Es, Ms, _ = _series(S.ISING, beta, 4096, W.seed_for(61))
    E_all, M_all = X.enumerate_states(2, 4)
    _check(Es, Ms, X.boltzmann_averages(E_all, M_all, beta), ("E", "E2", "absM", "M2"), beta)


def test_4x4_spin_glass_sample_many_replicas_match_enumeration():
    seed = W.seed_for(62)
    J = O.init_couplings(2, 4, seed, 0)  # the sample the GPU batch shares (checked bit for bit elsewhere)
    E_all, M_all = X.enumerate_states(2, 4, J)
    for beta in (0.4, 1.0):
        Es, Ms, coup = _series(S.EA, beta, 4096, seed)
        assert np.array_equal(coup.reshape(-1)[:J.size], J.reshape(-1))
        _check(Es, Ms, X.boltzmann_averages(E_all, M_all, beta), ("E", "E2", "M2"), beta)


def test_4x4_swap_rate_many_chains_matches_exact_double_sum():
    """Parallel tempering of 4096 chains of the 4 x 4 Ising model at two
    temperatures: the mean acceptance of the exchange (Eq. 12) equals the
    exact sum over the density of states of P_b1(E1) P_b2(E2)
    min(1, exp((b2 - b1)(E2 - E1)))."""
    b1, b2 = 0.30, 0.45
    E_all, M_all = X.enumerate_states(2, 4)
    lev, cnt = X.density_of_states(E_all)

    def p(b):
        w = cnt * np.exp(-b * (lev - lev.min()))
        return w / w.sum()

    x = (b2 - b1) * (lev[None, :] - lev[:, None])
    exact = float((p(b1)[:, None] * p(b2)[None, :] * np.minimum(1.0, np.exp(x))).sum())
    nc, nt, L = 4096, 2, 4
    b = S.Batch(S.ISING, 2, L, nc * nt, W.seed_for(63))
    spins = torch.zeros(nc * nt * L * L, dtype=torch.int8, device=DEV)
    S.spin_init(b, spins)
    E = torch.zeros(nc * nt, dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E)
    sot = torch.arange(nt, dtype=torch.int32, device=DEV).repeat(nc)
    betas = np.array([b1, b2])
    S.pt_sweep_swap(b, nc, nt, betas, spins, sot, E, 0, 100)  # equilibrate
    acc = torch.zeros(nc * (nt - 1), dtype=torch.int64, device=DEV)
    S.pt_sweep_swap(b, nc, nt, betas, spins, sot, E, 100, 2000, swap_accepts=acc)
    torch.cuda.synchronize()
    rates = acc.cpu().numpy().astype(np.float64) / 1000.0  # the pair is attempted on even steps
    mean, err = rates.mean(), rates.std(ddof=1) / math.sqrt(len(rates))
    assert abs(mean - exact) < 4.5 * err, (mean, exact, err)
    # the tracked energies are still the configurations' energies
    E2 = torch.zeros_like(E)
    S.measure_energy_magnetisation(b, spins, E2)
    assert torch.equal(E, E2)
