"""GPU parity of the per-replica LDS tempering path for 2D batches (uneven or
uniform edges in {16, 32, ..., 256}) against the oracle: spins, permutations,
energies and exchange counts bit-exact, through the step graph and the plain
launch path."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1101_1427_amd as S
import workloads as W
from oracle import oracle as O
from tests import refrun

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _run(model, sizes, n_temps, beta, seed, calls, perms=None, m=1):
    inst = refrun.uneven_table(2, sizes, n_temps, model)
    n_chains = len(sizes)
    b = S.Batch(model, 2, 0, len(inst), seed, inst=inst)
    n_steps = sum(n for _, n in calls)
    assert S.pt_plan(b, n_chains, n_temps, beta, n_steps, sweeps_per_step=m)[1] == "k_uneven2d_sweep"
    spins = torch.zeros(b.spins_shape()[0], dtype=torch.int8, device=DEV)
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV) if model == S.EA else None
    S.spin_init(b, spins, coup)
    E = torch.zeros(len(inst), dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E, couplings=coup)
    if perms is None:
        perms = np.tile(np.arange(n_temps, dtype=np.int32), n_chains)
    sot = torch.from_numpy(perms.copy()).to(DEV)
    acc = torch.zeros(n_chains * (n_temps - 1), dtype=torch.int64, device=DEV)
    for step0, n in calls:
        S.pt_sweep_swap(b, n_chains, n_temps, beta, spins, sot, E, step0, n, couplings=coup, swap_accepts=acc,
                        sweeps_per_step=m)
    return inst, _host(spins), _host(sot), _host(E), _host(acc), perms


def _check_chain(model, inst, q, n_temps, beta, seed, t0, steps, got, perms, m=1):
    got_s, got_p, got_E, got_a = got
    rows = inst[q * n_temps:(q + 1) * n_temps]
    L = int(rows[0][0])
    N = L * L
    chain = np.stack([O.init_spins(2, L, seed, q * n_temps + k) for k in range(n_temps)])
    J = O.init_couplings(2, L, seed, int(rows[0][1])) if model == S.EA else None
    Eq = np.array([O.energy(2, L, J, chain[k]) for k in range(n_temps)], np.int64)
    sq = perms[q * n_temps:(q + 1) * n_temps].astype(np.int32).copy()
    aq = np.zeros(n_temps, np.uint64)
    O.pt_run(2, L, J, chain, np.asarray(beta, np.float64), sq, Eq, seed, q, q * n_temps, t0, steps, aq,
             sweeps_per_step=m)
    so = int(rows[0][2])
    assert np.array_equal(got_s[so:so + n_temps * N].reshape(n_temps, N), chain), f"spins of chain {q} (L={L})"
    assert np.array_equal(got_p[q * n_temps:(q + 1) * n_temps], sq), f"permutation of chain {q}"
    assert np.array_equal(got_E[q * n_temps:(q + 1) * n_temps], Eq.astype(np.float64)), f"energies of chain {q}"
    assert np.array_equal(got_a[q * (n_temps - 1):(q + 1) * (n_temps - 1)], aq[:n_temps - 1].astype(np.int64))


@pytest.mark.parametrize("model", [S.EA, S.ISING])
def test_uneven2d_every_edge_graph_and_remainder(model):
    """One chain per edge, 37 steps in two calls: a 32-step graph, a 5-step
    graph and a plain 2-step call."""
    sizes = [16, 32, 48, 256, 64, 96, 128, 192]
    n_temps, seed = 4, W.seed_for(50 + model)
    beta = W.geometric_ladder(0.5, 2.0, n_temps) if model == S.EA else W.geometric_ladder(1.8, 3.2, n_temps)
    perms = np.concatenate([np.random.default_rng(7).permutation(n_temps) for _ in sizes]).astype(np.int32)
    inst, *got = _run(model, sizes, n_temps, beta, seed, [(5, 37), (42, 2)], perms)
    got, perms = got[:4], got[4]
    for q in range(len(sizes)):
        _check_chain(model, inst, q, n_temps, beta, seed, 5, 39, got, perms)


@pytest.mark.parametrize("m", [3, 40])
def test_uneven2d_sweeps_per_step(m):
    """m sweeps between exchange rounds, all m in one launch per edge class
    with the replicas in LDS: a 13-step graph and a plain call of 2 steps."""
    sizes = [16, 32, 64, 256] if m < 10 else [16, 32, 64]
    n_temps, seed = 4, W.seed_for(58)
    beta = W.geometric_ladder(0.5, 2.0, n_temps)
    perms = np.concatenate([np.random.default_rng(9).permutation(n_temps) for _ in sizes]).astype(np.int32)
    inst, *got = _run(S.EA, sizes, n_temps, beta, seed, [(1, 13), (14, 2)], perms, m=m)
    got, perms = got[:4], got[4]
    for q in range(len(sizes)):
        _check_chain(S.EA, inst, q, n_temps, beta, seed, 1, 15, got, perms, m=m)


def test_uneven2d_repeated_calls_reuse_the_graph():
    """Three calls with identical arguments (the cached graph) continue the chain."""
    sizes = [32, 64, 32]
    n_temps, seed = 6, W.seed_for(53)
    beta = W.geometric_ladder(0.5, 2.0, n_temps)
    inst, *got = _run(S.EA, sizes, n_temps, beta, seed, [(0, 8), (8, 8), (16, 8)])
    got, perms = got[:4], got[4]
    for q in range(len(sizes)):
        _check_chain(S.EA, inst, q, n_temps, beta, seed, 0, 24, got, perms)


def test_uniform_2d_tempering_takes_the_lds_path():
    """A uniform 2D EA batch (L = 48) runs on the same path and matches the oracle."""
    L, n_chains, n_temps, seed = 48, 3, 5, W.seed_for(54)
    beta = W.geometric_ladder(0.5, 2.0, n_temps)
    b = S.Batch(S.EA, 2, L, n_chains * n_temps, seed, rep_per_sample=n_temps)
    assert S.pt_plan(b, n_chains, n_temps, beta, 12)[1] == "k_uneven2d_sweep"
    spins = torch.zeros(b.spins_shape()[0], dtype=torch.int8, device=DEV)
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV)
    S.spin_init(b, spins, coup)
    E = torch.zeros(b.n_rep, dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E, couplings=coup)
    sot = torch.arange(n_temps, dtype=torch.int32, device=DEV).repeat(n_chains)
    S.pt_sweep_swap(b, n_chains, n_temps, beta, spins, sot, E, 0, 12, couplings=coup)
    got_s, got_p, got_E = _host(spins).reshape(-1, L * L), _host(sot), _host(E)
    for q in range(n_chains):
        chain = np.stack([O.init_spins(2, L, seed, q * n_temps + k) for k in range(n_temps)])
        J = O.init_couplings(2, L, seed, q)
        Eq = np.array([O.energy(2, L, J, chain[k]) for k in range(n_temps)], np.int64)
        sq = np.arange(n_temps, dtype=np.int32)
        O.pt_run(2, L, J, chain, beta, sq, Eq, seed, q, q * n_temps, 0, 12)
        assert np.array_equal(got_s[q * n_temps:(q + 1) * n_temps], chain)
        assert np.array_equal(got_p[q * n_temps:(q + 1) * n_temps], sq)
        assert np.array_equal(got_E[q * n_temps:(q + 1) * n_temps], Eq.astype(np.float64))


def test_uneven2d_energies_match_measurement():
    sizes = [64, 128, 32, 96]
    n_temps, seed = 8, W.seed_for(55)
    beta = W.geometric_ladder(0.5, 2.0, n_temps)
    inst = refrun.uneven_table(2, sizes, n_temps, S.EA)
    b = S.Batch(S.EA, 2, 0, len(inst), seed, inst=inst)
    spins = torch.zeros(b.spins_shape()[0], dtype=torch.int8, device=DEV)
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV)
    S.spin_init(b, spins, coup)
    E = torch.zeros(len(inst), dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E, couplings=coup)
    sot = torch.arange(n_temps, dtype=torch.int32, device=DEV).repeat(len(sizes))
    S.pt_sweep_swap(b, len(sizes), n_temps, beta, spins, sot, E, 0, 300, couplings=coup)
    E2 = torch.zeros_like(E)
    S.measure_energy_magnetisation(b, spins, E2, couplings=coup)
    assert np.array_equal(_host(E), _host(E2))


def test_uneven2d_full_workload_sampled_chains():
    """The full uneven workload (4096 instances x 16 temperatures, edges drawn
    from {32, ..., 256}) for 6 steps in the benchmark's launch shape; chains of
    every edge sampled across the batch checked against the oracle."""
    cfg = W.ea2d_uneven(steps=6)
    n_temps = cfg.n_temps
    inst, *got = _run(S.EA, cfg.sizes, n_temps, cfg.betas, cfg.seed, [(0, cfg.steps)])
    got, perms = got[:4], got[4]
    picked = []
    for L in sorted(set(int(v) for v in cfg.sizes)):
        idx = np.nonzero(cfg.sizes == L)[0]
        picked += [int(idx[0]), int(idx[-1])]
    for q in picked:
        _check_chain(S.EA, inst, q, n_temps, cfg.betas, cfg.seed, 0, cfg.steps, got, perms)


def test_invalid_chain_next_to_a_valid_one():
    """Edge 32, two chains in one launch: the one whose slot_of_temp row
    repeats a slot is left unchanged, the other matches the oracle."""
    sizes, n_temps, seed = [32, 32], 4, W.seed_for(56)
    beta = W.geometric_ladder(0.5, 2.0, n_temps)
    perms = np.array([0, 1, 2, 3, 2, 2, 0, 1], np.int32)
    inst = refrun.uneven_table(2, sizes, n_temps, S.EA)
    b = S.Batch(S.EA, 2, 0, len(inst), seed, inst=inst)
    spins = torch.zeros(b.spins_shape()[0], dtype=torch.int8, device=DEV)
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV)
    S.spin_init(b, spins, coup)
    E = torch.zeros(len(inst), dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E, couplings=coup)
    s0, E0 = _host(spins).copy(), _host(E).copy()
    sot = torch.from_numpy(perms.copy()).to(DEV)
    acc = torch.zeros(2 * (n_temps - 1), dtype=torch.int64, device=DEV)
    S.pt_sweep_swap(b, 2, n_temps, beta, spins, sot, E, 0, 9, couplings=coup, swap_accepts=acc)
    got = (_host(spins), _host(sot), _host(E), _host(acc))
    N = 32 * 32
    assert np.array_equal(got[0][n_temps * N:], s0[n_temps * N:])
    assert np.array_equal(got[1][n_temps:], perms[n_temps:])
    assert np.array_equal(got[2][n_temps:], E0[n_temps:])
    assert not got[3][n_temps - 1:].any()
    _check_chain(S.EA, inst, 0, n_temps, beta, seed, 0, 9, got, perms)


def test_workgroup_size_never_changes_results(monkeypatch):
    """Forced workgroup sizes 64 and 512, and the autotuner's choice: identical
    spins, energies and permutations."""
    sizes, n_temps, seed = [48, 128, 32], 4, W.seed_for(57)
    beta = W.geometric_ladder(0.5, 2.0, n_temps)
    outs = []
    for env in ("64", "512", None):
        if env is None:
            monkeypatch.delenv("SPINMC_U2D_THREADS", raising=False)
        else:
            monkeypatch.setenv("SPINMC_U2D_THREADS", env)
        inst, *got = _run(S.EA, sizes, n_temps, beta, seed, [(0, 6)])
        outs.append(got[:4])
    for o in outs[1:]:
        for x, y in zip(o, outs[0]):
            assert np.array_equal(x, y)
