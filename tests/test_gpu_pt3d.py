"""GPU parity of the chain-resident tempering kernel (3D, edge 16) against the oracle.

Every chain of a batch runs all steps of a call in one workgroup with its
replicas in LDS; spins, temperature permutations, energies and exchange
counts must equal the oracle's step for step (bit-exact).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1101_1427_amd as S
import workloads as W
from oracle import oracle as O

pytestmark = pytest.mark.gpu

DEV = "cuda"
L = 16
N = L ** 3


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _perms(n_chains, n_temps, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.permutation(n_temps) for _ in range(n_chains)]).astype(np.int32)


def _run_gpu(model, n_chains, n_temps, rps, seed, beta, calls, perms, beta_per_chain=False, m=1):
    b = S.Batch(model, 3, L, n_chains * n_temps, seed, rep_per_sample=rps)
    assert S.pt_plan(b, n_chains, n_temps, beta, 10, beta_per_chain)[1] == "k_pt3d_chain"
    spins = torch.zeros(b.spins_shape()[0], dtype=torch.int8, device=DEV)
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV) if model == S.EA else None
    S.spin_init(b, spins, coup)
    E = torch.zeros(b.n_rep, dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E, couplings=coup)
    sot = torch.from_numpy(perms.copy()).to(DEV)
    acc = torch.zeros(n_chains * (n_temps - 1), dtype=torch.int64, device=DEV)
    for step0, n in calls:
        S.pt_sweep_swap(b, n_chains, n_temps, beta, spins, sot, E, step0, n, couplings=coup, swap_accepts=acc,
                        beta_per_chain=beta_per_chain, sweeps_per_step=m)
    return _host(spins).reshape(-1, N), _host(sot), _host(E), _host(acc)


def _oracle_chain(model, q, n_temps, rps, seed, beta_q, perm_q, t0, steps, m=1):
    r0 = q * n_temps
    chain = np.stack([O.init_spins(3, L, seed, r0 + k) for k in range(n_temps)])
    J = O.init_couplings(3, L, seed, r0 // rps) if model == S.EA else None
    E = np.array([O.energy(3, L, J, chain[k]) for k in range(n_temps)], np.int64)
    sq = perm_q.astype(np.int32).copy()
    aq = np.zeros(n_temps, np.uint64)
    O.pt_run(3, L, J, chain, np.asarray(beta_q, np.float64), sq, E, seed, q, r0, t0, steps, aq, sweeps_per_step=m)
    return chain, sq, E, aq[:n_temps - 1]


def _check(model, n_chains, n_temps, rps, seed, beta, calls, chains=None, beta_per_chain=False, m=1):
    perms = _perms(n_chains, n_temps, seed & 0xFFFF)
    got_s, got_p, got_E, got_a = _run_gpu(model, n_chains, n_temps, rps, seed, beta, calls, perms, beta_per_chain, m)
    t0 = calls[0][0]
    steps = sum(n for _, n in calls)
    beta = np.asarray(beta, np.float64).reshape(-1, n_temps)
    for q in (range(n_chains) if chains is None else chains):
        bq = beta[q] if beta_per_chain else beta[0]
        chain, sq, E, aq = _oracle_chain(model, q, n_temps, rps, seed, bq, perms[q * n_temps:(q + 1) * n_temps], t0,
                                         steps, m)
        sl = slice(q * n_temps, (q + 1) * n_temps)
        assert np.array_equal(got_s[sl], chain), f"spins of chain {q}"
        assert np.array_equal(got_p[sl], sq), f"permutation of chain {q}"
        assert np.array_equal(got_E[sl], E.astype(np.float64)), f"energies of chain {q}"
        assert np.array_equal(got_a[q * (n_temps - 1):(q + 1) * (n_temps - 1)], aq.astype(np.int64)), f"counts {q}"
    return got_s, got_E


def test_pt3d_sweeps_per_step():
    """Three sweeps between exchange rounds (sweep indices t*3 .. t*3 + 2)."""
    _check(S.EA, 3, 6, 6, W.seed_for(45), W.geometric_ladder(0.8, 2.0, 6), [(2, 5), (7, 4)], m=3)


def test_pt3d_ea_bit_exact_two_calls():
    """EA, 4 chains over 2 samples, 8 temperatures, 24 steps split over two calls."""
    _check(S.EA, 4, 8, 16, W.seed_for(40), W.geometric_ladder(0.8, 2.0, 8), [(3, 11), (14, 13)])


def test_pt3d_ea_full_chain_width():
    """32 temperatures (two replicas per wave), the width of the tempering workload."""
    _check(S.EA, 2, 32, 64, W.seed_for(41), W.geometric_ladder(0.8, 2.0, 32), [(0, 12)])


def test_pt3d_ising_odd_temperature_count():
    """Ising, 5 temperatures (waves with one replica), an odd step count."""
    _check(S.ISING, 3, 5, 1, W.seed_for(42), W.geometric_ladder(3.0, 6.0, 5), [(7, 9)])


def test_pt3d_beta_per_chain():
    n_chains, n_temps = 3, 6
    beta = np.stack([W.geometric_ladder(0.8 + 0.1 * q, 2.0, n_temps) for q in range(n_chains)])
    _check(S.EA, n_chains, n_temps, 6, W.seed_for(43), beta, [(0, 10)], beta_per_chain=True)


def test_pt3d_energies_match_measurement():
    """Tracked energies equal a fresh measurement of the final configurations."""
    n_chains, n_temps, rps = 2, 16, 32
    seed = W.seed_for(44)
    beta = W.geometric_ladder(0.8, 2.0, n_temps)
    b = S.Batch(S.EA, 3, L, n_chains * n_temps, seed, rep_per_sample=rps)
    spins = torch.zeros(b.spins_shape()[0], dtype=torch.int8, device=DEV)
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV)
    S.spin_init(b, spins, coup)
    E = torch.zeros(b.n_rep, dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E, couplings=coup)
    sot = torch.arange(n_temps, dtype=torch.int32, device=DEV).repeat(n_chains)
    S.pt_sweep_swap(b, n_chains, n_temps, beta, spins, sot, E, 0, 200, couplings=coup)
    E2 = torch.zeros_like(E)
    S.measure_energy_magnetisation(b, spins, E2, couplings=coup)
    assert np.array_equal(_host(E), _host(E2))
    assert sorted(_host(sot)[:n_temps].tolist()) == list(range(n_temps))


@pytest.mark.parametrize("L_edge", [16, 6])
def test_invalid_permutation_leaves_chain_unchanged(L_edge):
    """A chain whose slot_of_temp row is not a permutation is left as it is
    (edge 16: chain-resident kernel; edge 6: generic path)."""
    n_chains, n_temps = 2, 4
    seed = W.seed_for(45)
    beta = W.geometric_ladder(0.8, 2.0, n_temps)
    b = S.Batch(S.EA, 3, L_edge, n_chains * n_temps, seed, rep_per_sample=n_temps)
    want = "k_pt3d_chain" if L_edge == 16 else "k_half_sweep_generic"
    assert S.pt_plan(b, n_chains, n_temps, beta, 5)[1] == want
    spins = torch.zeros(b.spins_shape()[0], dtype=torch.int8, device=DEV)
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV)
    S.spin_init(b, spins, coup)
    E = torch.zeros(b.n_rep, dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E, couplings=coup)
    s0, E0 = _host(spins).copy(), _host(E).copy()
    perm = np.array([0, 1, 2, 3, 1, 1, 0, 3], np.int32)  # chain 1 repeats slot 1
    sot = torch.from_numpy(perm.copy()).to(DEV)
    acc = torch.zeros(n_chains * (n_temps - 1), dtype=torch.int64, device=DEV)
    S.pt_sweep_swap(b, n_chains, n_temps, beta, spins, sot, E, 0, 5, couplings=coup, swap_accepts=acc)
    Nl = L_edge ** 3
    got = _host(spins)
    assert np.array_equal(got[n_temps * Nl:], s0[n_temps * Nl:])
    assert np.array_equal(_host(E)[n_temps:], E0[n_temps:])
    assert np.array_equal(_host(sot)[n_temps:], perm[n_temps:])
    assert not _host(acc)[n_temps - 1:].any()
    assert not np.array_equal(got[:n_temps * Nl], s0[:n_temps * Nl])  # the valid chain moved


def test_pt3d_full_workload_sampled_chains():
    """The full tempering workload (512 samples x 2 replicas x 32 temperatures)
    in the launch shape of the benchmark, a few steps, chains sampled across
    the batch checked against the oracle."""
    cfg = W.ea3d_tempering(steps=6)
    _check(S.EA, cfg.n_chains, cfg.n_temps, 2 * cfg.n_temps, cfg.seed, cfg.betas, [(0, cfg.steps)],
           chains=[0, 1, 511, 1023])
