"""GPU parity of the asynchronous multi-spin-coded sweep (32 replicas per
word sharing their random numbers) against the oracle run replica by
replica with the group index in the counters: spins and energy changes
bit-exact, packed kernel and generic kernels alike."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1101_1427_amd as S
import workloads as W
from tests import refrun

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _run(model, dim, L, n_rep, betas, seed, t0, n, calls=None, w=32):
    b = S.Batch(model, dim, L, n_rep, seed)
    spins = torch.zeros(b.spins_shape()[0], dtype=torch.int8, device=DEV)
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV) if model == S.EA else None
    S.spin_init(b, spins, coup)
    dE = torch.zeros(n_rep, dtype=torch.int64, device=DEV)
    for s0, k in calls or [(t0, n)]:
        S.msc_sweep(b, spins, betas, s0, k, couplings=coup, dE_accum=dE, word_bits=w)
    return b, _host(spins).reshape(n_rep, -1), _host(dE)


def _reference(model, dim, L, n_rep, betas, seed, t0, n, w=32):
    ref_s, ref_c = refrun.init_uniform(model, dim, L, n_rep, seed)
    ref_dE = refrun.sweep_msc(model, dim, L, ref_s, ref_c, betas, seed, t0, n, w=w)
    return ref_s, ref_dE


@pytest.mark.parametrize("L,pairs,n", [(16, 3, 7), (32, 1, 5), (64, 1, 4)])
def test_msc2d_64_replicas_per_draw(L, pairs, n):
    """64 replicas per draw group (two words updated with one draw per site)."""
    seed, n_rep = W.seed_for(69 + L), 64 * pairs
    betas = np.repeat(np.linspace(0.6, 1.4, pairs), 64)
    b, got_s, got_dE = _run(S.EA, 2, L, n_rep, betas, seed, 3, n, w=64)
    assert S.msc_plan(b, n, word_bits=64) == (1, "k_msc2d")
    ref_s, ref_dE = _reference(S.EA, 2, L, n_rep, betas, seed, 3, n, w=64)
    assert np.array_equal(got_s, ref_s)
    assert np.array_equal(got_dE, ref_dE)


def test_msc_64_generic_path_and_ties(monkeypatch):
    """64 per draw: the generic kernels give the packed kernel's result, and
    32 groups x 50 sweeps at beta = 1 (head ties) match the oracle."""
    L, n_rep, seed, n = 16, 128, W.seed_for(70), 6
    betas = np.full(n_rep, 0.9)
    _, fast_s, fast_dE = _run(S.ISING, 2, L, n_rep, betas, seed, 2, n, w=64)
    monkeypatch.setenv("SPINMC_MSC2D", "0")
    b, gen_s, gen_dE = _run(S.ISING, 2, L, n_rep, betas, seed, 2, n, w=64)
    assert S.msc_plan(b, n, word_bits=64)[1] == "k_half_sweep_generic"
    assert np.array_equal(fast_s, gen_s) and np.array_equal(fast_dE, gen_dE)
    monkeypatch.delenv("SPINMC_MSC2D")
    n_rep, n = 64 * 32, 50
    betas = np.full(n_rep, 1.0)
    _, got_s, got_dE = _run(S.EA, 2, L, n_rep, betas, seed, 0, n, w=64)
    ref_s, ref_dE = _reference(S.EA, 2, L, n_rep, betas, seed, 0, n, w=64)
    assert np.array_equal(got_s, ref_s)
    assert np.array_equal(got_dE, ref_dE)


@pytest.mark.parametrize("L,groups,n", [(16, 3, 7), (32, 2, 5), (64, 1, 4)])
def test_msc2d_ea_bit_exact(L, groups, n):
    seed, n_rep = W.seed_for(60 + L), 32 * groups
    betas = np.repeat(np.linspace(0.6, 1.4, groups), 32)
    b, got_s, got_dE = _run(S.EA, 2, L, n_rep, betas, seed, 3, n)
    assert S.msc_plan(b, n) == (1, "k_msc2d")
    ref_s, ref_dE = _reference(S.EA, 2, L, n_rep, betas, seed, 3, n)
    assert np.array_equal(got_s, ref_s)
    assert np.array_equal(got_dE, ref_dE)


def test_msc2d_ising_and_split_calls():
    """Ising (no couplings), the sweeps split over three calls."""
    L, n_rep, seed = 16, 64, W.seed_for(64)
    betas = np.full(n_rep, 0.44)
    _, got_s, got_dE = _run(S.ISING, 2, L, n_rep, betas, seed, 0, 11, calls=[(0, 4), (4, 1), (5, 6)])
    ref_s, ref_dE = _reference(S.ISING, 2, L, n_rep, betas, seed, 0, 11)
    assert np.array_equal(got_s, ref_s)
    assert np.array_equal(got_dE, ref_dE)


def test_msc2d_many_groups_every_replica():
    """64 groups x 50 sweeps at beta = 1 (about 25 draws whose head ties a
    threshold and need the tail): every replica bit-exact."""
    L, groups, n, seed = 16, 64, 50, W.seed_for(65)
    n_rep = 32 * groups
    betas = np.full(n_rep, 1.0)
    _, got_s, got_dE = _run(S.EA, 2, L, n_rep, betas, seed, 0, n)
    ref_s, ref_dE = _reference(S.EA, 2, L, n_rep, betas, seed, 0, n)
    assert np.array_equal(got_s, ref_s)
    assert np.array_equal(got_dE, ref_dE)


def test_msc_generic_path_matches(monkeypatch):
    """SPINMC_MSC2D=0 (generic kernels, group-keyed draws) gives the packed
    kernel's result; an edge the packed kernel does not take (L = 20) and a
    3D batch go to the generic kernels and match the oracle."""
    L, n_rep, seed, n = 32, 64, W.seed_for(66), 6
    betas = np.full(n_rep, 0.9)
    _, fast_s, fast_dE = _run(S.EA, 2, L, n_rep, betas, seed, 2, n)
    monkeypatch.setenv("SPINMC_MSC2D", "0")
    b, gen_s, gen_dE = _run(S.EA, 2, L, n_rep, betas, seed, 2, n)
    assert S.msc_plan(b, n)[1] == "k_half_sweep_generic"
    assert np.array_equal(fast_s, gen_s) and np.array_equal(fast_dE, gen_dE)
    monkeypatch.delenv("SPINMC_MSC2D")
    for model, dim, L2 in ((S.EA, 2, 20), (S.ISING, 3, 8)):
        betas2 = np.full(32, 0.5)
        b, got_s, got_dE = _run(model, dim, L2, 32, betas2, seed, 1, 4)
        assert S.msc_plan(b, 4)[1] == "k_half_sweep_generic"
        ref_s, ref_dE = _reference(model, dim, L2, 32, betas2, seed, 1, 4)
        assert np.array_equal(got_s, ref_s)
        assert np.array_equal(got_dE, ref_dE)


def test_msc2d_benchmark_shape_sampled():
    """The benchmark's shape (16 x 16, 2^15 replicas) for 20 sweeps: replicas
    of groups spread over the batch against the oracle."""
    L, n_rep, n, seed = 16, 1 << 15, 20, W.seed_for(67)
    betas = np.full(n_rep, 1.0)
    b, got_s, got_dE = _run(S.EA, 2, L, n_rep, betas, seed, 0, n)
    from oracle import oracle as O

    for g in (0, 1, 517, n_rep // 32 - 1):
        for k in (0, 13, 31):
            r = 32 * g + k
            s = O.init_spins(2, L, seed, r)
            J = O.init_couplings(2, L, seed, r)
            d = O.run(2, L, J, s, 1.0, seed, g, 0, n)
            assert np.array_equal(got_s[r], s), r
            assert int(got_dE[r]) == int(d), r


def test_msc_unaligned_buffers_take_the_generic_kernels():
    """Spins one byte past an aligned address: same results as aligned."""
    L, n_rep, seed, n = 16, 32, W.seed_for(68), 5
    betas = np.full(n_rep, 0.8)
    _, ref_s, ref_dE = _run(S.EA, 2, L, n_rep, betas, seed, 0, n)
    b = S.Batch(S.EA, 2, L, n_rep, seed)
    buf = torch.zeros(b.spins_shape()[0] + 1, dtype=torch.int8, device=DEV)
    spins = buf[1:]
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV)
    S.spin_init(b, spins, coup)
    dE = torch.zeros(n_rep, dtype=torch.int64, device=DEV)
    S.msc_sweep(b, spins, betas, 0, n, couplings=coup, dE_accum=dE)
    assert np.array_equal(_host(spins).reshape(n_rep, -1), ref_s)
    assert np.array_equal(_host(dE), ref_dE)
