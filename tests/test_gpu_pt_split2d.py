"""GPU parity of tempering on the one-pass colour-split 2D Ising sweep
(uniform batches, L a power of two >= 1024): spins, temperature
permutations, energies and exchange counts equal the oracle's, with one or
several sweeps per exchange round; chains whose permutation row is invalid
are left unchanged."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1101_1427_amd as S
import workloads as W
from oracle import oracle as O

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _gpu(L, n_chains, n_temps, beta, seed, calls, perms, m, beta_per_chain=False):
    b = S.Batch(S.ISING, 2, L, n_chains * n_temps, seed)
    assert S.pt_plan(b, n_chains, n_temps, beta, 4, beta_per_chain, sweeps_per_step=m)[1] == "k_ising2d_split"
    spins = torch.zeros(b.n_rep * L * L, dtype=torch.int8, device=DEV)
    S.spin_init(b, spins)
    E = torch.zeros(b.n_rep, dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E)
    sot = torch.from_numpy(perms.copy()).to(DEV)
    acc = torch.zeros(n_chains * (n_temps - 1), dtype=torch.int64, device=DEV)
    for step0, n in calls:
        S.pt_sweep_swap(b, n_chains, n_temps, beta, spins, sot, E, step0, n, swap_accepts=acc,
                        beta_per_chain=beta_per_chain, sweeps_per_step=m)
    return _host(spins).reshape(b.n_rep, L * L), _host(sot), _host(E), _host(acc)


def _oracle(L, q, n_temps, beta_q, seed, perm_q, t0, steps, m):
    chain = np.stack([O.init_spins(2, L, seed, q * n_temps + k) for k in range(n_temps)])
    E = np.array([O.energy(2, L, None, chain[k]) for k in range(n_temps)], np.int64)
    sq = perm_q.astype(np.int32).copy()
    aq = np.zeros(n_temps, np.uint64)
    O.pt_run(2, L, None, chain, np.asarray(beta_q, np.float64), sq, E, seed, q, q * n_temps, t0, steps, aq,
             sweeps_per_step=m)
    return chain, sq, E, aq[:n_temps - 1]


def _check(L, n_chains, n_temps, beta, seed, calls, m, perms, beta_per_chain=False, chains=None):
    got_s, got_p, got_E, got_a = _gpu(L, n_chains, n_temps, beta, seed, calls, perms, m, beta_per_chain)
    t0, steps = calls[0][0], sum(n for _, n in calls)
    bt = np.asarray(beta, np.float64).reshape(-1, n_temps)
    for q in (range(n_chains) if chains is None else chains):
        sl = slice(q * n_temps, (q + 1) * n_temps)
        chain, sq, E, aq = _oracle(L, q, n_temps, bt[q] if beta_per_chain else bt[0], seed, perms[sl], t0, steps, m)
        assert np.array_equal(got_s[sl], chain), f"spins of chain {q}"
        assert np.array_equal(got_p[sl], sq), f"permutation of chain {q}"
        assert np.array_equal(got_E[sl], E.astype(np.float64)), f"energies of chain {q}"
        assert np.array_equal(got_a[q * (n_temps - 1):(q + 1) * (n_temps - 1)], aq.astype(np.int64)), f"counts {q}"
    return got_s, got_p, got_E, got_a


def test_split_tempering_two_sweeps_per_step():
    """1024^2, one chain of 4 temperatures, 2 sweeps per exchange, two calls."""
    perms = np.array([2, 0, 3, 1], np.int32)
    _check(1024, 1, 4, [0.30, 0.40, W.BETA_C_2D, 0.50], W.seed_for(92), [(3, 2), (5, 1)], 2, perms)


def test_split_tempering_one_sweep_per_step_two_chains():
    """Two chains with their own ladders (beta_per_chain), one sweep per step."""
    perms = np.array([0, 1, 2, 2, 0, 1], np.int32)
    beta = [[0.10, 0.125, 0.15], [0.35, 0.42, 0.48]]
    _check(1024, 2, 3, beta, W.seed_for(93), [(0, 4)], 1, perms, beta_per_chain=True)


def test_split_and_generic_paths_agree(monkeypatch):
    """The same call on the generic kernels (SPINMC_PT_SPLIT2D=0): identical
    spins, permutations, energies and counts."""
    perms = np.array([1, 0, 2, 3, 3, 2, 0, 1], np.int32)
    beta = W.geometric_ladder(0.3, 0.5, 4)
    split = _gpu(1024, 2, 4, beta, W.seed_for(94), [(7, 3)], perms, 2)
    monkeypatch.setenv("SPINMC_PT_SPLIT2D", "0")
    b = S.Batch(S.ISING, 2, 1024, 8, W.seed_for(94))
    assert S.pt_plan(b, 2, 4, beta, 3, sweeps_per_step=2)[1] == "k_half_sweep_generic"
    spins = torch.zeros(8 * 1024 * 1024, dtype=torch.int8, device=DEV)
    S.spin_init(b, spins)
    E = torch.zeros(8, dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E)
    sot = torch.from_numpy(perms.copy()).to(DEV)
    acc = torch.zeros(2 * 3, dtype=torch.int64, device=DEV)
    S.pt_sweep_swap(b, 2, 4, beta, spins, sot, E, 7, 3, swap_accepts=acc, sweeps_per_step=2)
    generic = (_host(spins).reshape(8, -1), _host(sot), _host(E), _host(acc))
    for a, g in zip(split, generic):
        assert np.array_equal(a, g)


def test_invalid_chain_is_left_unchanged():
    """Chain 1's row is not a permutation: its spins, energies, slots and
    counts stay as they were; chain 0 follows the oracle."""
    L, n_temps, seed = 1024, 3, W.seed_for(95)
    perms = np.array([2, 0, 1, 0, 0, 1], np.int32)
    beta = [0.35, 0.42, 0.48]
    b = S.Batch(S.ISING, 2, L, 2 * n_temps, seed)
    spins0 = torch.zeros(b.n_rep * L * L, dtype=torch.int8, device=DEV)
    S.spin_init(b, spins0)
    E0 = torch.zeros(b.n_rep, dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins0, E0)
    got_s, got_p, got_E, got_a = _check(L, 2, n_temps, beta, seed, [(0, 3)], 2, perms, chains=[0])
    sl = slice(n_temps, 2 * n_temps)
    assert np.array_equal(got_s[sl], _host(spins0).reshape(b.n_rep, L * L)[sl])
    assert np.array_equal(got_E[sl], _host(E0)[sl])
    assert np.array_equal(got_p[sl], perms[sl])
    assert not got_a[n_temps - 1:].any()
