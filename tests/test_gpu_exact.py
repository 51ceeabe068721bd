"""The GPU sweeps against exact results directly (not through the oracle):
4096 replicas of the 4 x 4 periodic Ising model and of one 4 x 4 +-J sample,
time averages of E, E^2, |M| and M^2 against the exact Boltzmann averages of
all 2^16 states (Eq. 1 with the Metropolis rule of Eq. 2 as its stationary
law).  With 4096 independent replicas the standard errors are about six
times smaller than in the oracle's own enumeration test."""
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
