"""GPU parity of the double-checkerboard sweep with multi-hit updates
(smc_dcb_sweep) against the oracle's orc_dcb_run: spins and energy changes
bit-exact over tilings, hit counts, the palindromic order and both models."""
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


def _gpu(model, L, n_rep, betas, seed, calls, T, k, pal, rps=1):
    b = S.Batch(model, 2, L, n_rep, seed, rep_per_sample=rps)
    spins = torch.zeros(n_rep * L * L, dtype=torch.int8, device=DEV)
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV) if model == S.EA else None
    S.spin_init(b, spins, coup)
    dE = torch.zeros(n_rep, dtype=torch.int64, device=DEV)
    for s0, n in calls:
        S.dcb_sweep(b, spins, betas, s0, n, T, k, palindromic=pal, couplings=coup, dE_accum=dE)
    return _host(spins).reshape(n_rep, L * L), _host(dE)


def _oracle(model, L, n_rep, betas, seed, t0, n, T, k, pal, rps=1):
    out, dEs = [], []
    for r in range(n_rep):
        s = O.init_spins(2, L, seed, r)
        J = O.init_couplings(2, L, seed, r // rps) if model == S.EA else None
        dEs.append(O.dcb_run(L, T, k, J, s, float(betas[r]), seed, r, t0, n, palindromic=pal))
        out.append(s)
    return np.stack(out), np.array(dEs, np.int64)


@pytest.fixture(params=["packed", "per_site"])
def kernel(request, monkeypatch):
    """Both kernels: the packed one (four sites per word) and the per-site one."""
    monkeypatch.setenv("SPINMC_DCB_PACKED", "1" if request.param == "packed" else "0")
    return request.param


@pytest.mark.parametrize("model,L,T,k,pal", [
    (S.EA, 32, 16, 1, False), (S.EA, 64, 16, 3, True), (S.ISING, 64, 32, 5, False),
    (S.EA, 128, 64, 2, True), (S.ISING, 256, 128, 4, False), (S.EA, 16, 16, 2, False),
    (S.ISING, 128, 64, 3, True), (S.EA, 256, 128, 2, False), (S.ISING, 32, 32, 4, True),
    (S.EA, 96, 48, 2, False),
])
def test_dcb_matches_oracle(kernel, model, L, T, k, pal):
    seed, n_rep = W.seed_for(71), 3
    betas = [0.3, 0.44, 0.9]
    got_s, got_dE = _gpu(model, L, n_rep, betas, seed, [(5, 3), (8, 2)], T, k, pal)
    ref_s, ref_dE = _oracle(model, L, n_rep, betas, seed, 5, 5, T, k, pal)
    assert np.array_equal(got_s, ref_s)
    assert np.array_equal(got_dE, ref_dE)


def test_dcb_shared_samples(kernel):
    """Two replicas per coupling sample."""
    seed, L, T, k = W.seed_for(72), 64, 32, 3
    betas = [0.5, 1.1, 0.5, 1.1]
    got_s, got_dE = _gpu(S.EA, L, 4, betas, seed, [(0, 4)], T, k, False, rps=2)
    ref_s, ref_dE = _oracle(S.EA, L, 4, betas, seed, 0, 4, T, k, False, rps=2)
    assert np.array_equal(got_s, ref_s) and np.array_equal(got_dE, ref_dE)


def test_dcb_beta_zero_in_the_batch(kernel):
    """A replica at beta = 0 (threshold 2^32) sends the batch to the per-site
    kernel; results stay those of the oracle."""
    seed, L, T, k = W.seed_for(75), 64, 16, 2
    betas = [0.0, 0.44, 0.8]
    got_s, got_dE = _gpu(S.EA, L, 3, betas, seed, [(2, 3)], T, k, True)
    ref_s, ref_dE = _oracle(S.EA, L, 3, betas, seed, 2, 3, T, k, True)
    assert np.array_equal(got_s, ref_s) and np.array_equal(got_dE, ref_dE)


def test_dcb_many_small_tiles_per_workgroup(kernel):
    """16 x 16 tiles (four per workgroup in the packed kernel) over a batch
    whose tile count is not a multiple of four."""
    seed, L, T, k = W.seed_for(76), 32, 16, 3
    betas = [0.2, 0.35, 0.44, 0.5, 0.7]
    got_s, got_dE = _gpu(S.ISING, L, 5, betas, seed, [(0, 2), (2, 3)], T, k, False)
    ref_s, ref_dE = _oracle(S.ISING, L, 5, betas, seed, 0, 5, T, k, False)
    assert np.array_equal(got_s, ref_s) and np.array_equal(got_dE, ref_dE)


def test_single_tile_single_hit_equals_plain_sweep(kernel):
    """tile = L and hits = 1: the same chain as smc_metropolis_sweep."""
    seed, L, n_rep = W.seed_for(73), 64, 2
    b = S.Batch(S.EA, 2, L, n_rep, seed)
    outs = []
    for use_dcb in (True, False):
        spins = torch.zeros(n_rep * L * L, dtype=torch.int8, device=DEV)
        coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV)
        S.spin_init(b, spins, coup)
        dE = torch.zeros(n_rep, dtype=torch.int64, device=DEV)
        if use_dcb:
            S.dcb_sweep(b, spins, [0.7, 1.3], 3, 6, L, 1, couplings=coup, dE_accum=dE)
        else:
            S.metropolis_sweep(b, spins, [0.7, 1.3], 3, 6, couplings=coup, dE_accum=dE)
        outs.append((_host(spins).copy(), _host(dE).copy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_dcb_large_lattice(kernel):
    """1024 x 1024, 64 x 64 tiles, 8 hits, 2 sweeps, every site."""
    seed, L = W.seed_for(74), 1024
    got_s, got_dE = _gpu(S.ISING, L, 1, [0.44], seed, [(0, 2)], 64, 8, False)
    ref_s, ref_dE = _oracle(S.ISING, L, 1, [0.44], seed, 0, 2, 64, 8, False)
    assert np.array_equal(got_s, ref_s) and np.array_equal(got_dE, ref_dE)


def test_dcb_energy_trace(kernel):
    """dE_trace row m = the oracle's energy change over sweeps 0 .. m of the call."""
    seed, L, T, k, n, n_rep = W.seed_for(77), 64, 16, 3, 6, 3
    betas = [0.3, 0.44, 0.7]
    b = S.Batch(S.EA, 2, L, n_rep, seed)
    spins = torch.zeros(n_rep * L * L, dtype=torch.int8, device=DEV)
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV)
    S.spin_init(b, spins, coup)
    trace = torch.full((n, n_rep), -7, dtype=torch.int64, device=DEV)
    S.dcb_sweep(b, spins, betas, 4, n, T, k, palindromic=True, couplings=coup, dE_trace=trace)
    got = _host(trace)
    ref = np.zeros((n, n_rep), np.int64)
    for r in range(n_rep):
        s = O.init_spins(2, L, seed, r)
        J = O.init_couplings(2, L, seed, r)
        acc = 0
        for m in range(n):
            acc += O.dcb_run(L, T, k, J, s, betas[r], seed, r, 4 + m, 1, palindromic=True)
            ref[m, r] = acc
    assert np.array_equal(got, ref)


# ---------------------------------------------------------------- 3D --
def _gpu3(model, L, n_rep, betas, seed, calls, k, pal, rps=1):
    b = S.Batch(model, 3, L, n_rep, seed, rep_per_sample=rps)
    assert S.dcb_plan(b, betas, 16) == "k_dcb3d"
    spins = torch.zeros(n_rep * L ** 3, dtype=torch.int8, device=DEV)
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV) if model == S.EA else None
    S.spin_init(b, spins, coup)
    dE = torch.zeros(n_rep, dtype=torch.int64, device=DEV)
    for s0, n in calls:
        S.dcb_sweep(b, spins, betas, s0, n, 16, k, palindromic=pal, couplings=coup, dE_accum=dE)
    return _host(spins).reshape(n_rep, L ** 3), _host(dE)


def _oracle3(model, L, n_rep, betas, seed, t0, n, k, pal, rps=1):
    out, dEs = [], []
    for r in range(n_rep):
        s = O.init_spins(3, L, seed, r)
        J = O.init_couplings(3, L, seed, r // rps) if model == S.EA else None
        dEs.append(O.dcb_run(L, 16, k, J, s, float(betas[r]), seed, r, t0, n, palindromic=pal, dim=3))
        out.append(s)
    return np.stack(out), np.array(dEs, np.int64)


@pytest.mark.parametrize("model,L,k,pal,rps", [(S.ISING, 32, 2, True, 1), (S.EA, 32, 3, False, 1),
                                               (S.EA, 16, 2, True, 1), (S.EA, 32, 1, False, 3),
                                               (S.EA, 64, 2, True, 2)])
def test_dcb3d_matches_oracle(model, L, k, pal, rps):
    seed, n_rep = W.seed_for(78), 3
    betas = [0.15, 0.22, 0.4]
    got_s, got_dE = _gpu3(model, L, n_rep, betas, seed, [(2, 2), (4, 1)], k, pal, rps)
    ref_s, ref_dE = _oracle3(model, L, n_rep, betas, seed, 2, 3, k, pal, rps)
    assert np.array_equal(got_s, ref_s)
    assert np.array_equal(got_dE, ref_dE)


def test_dcb3d_single_tile_single_hit_equals_plain_sweep():
    seed, L = W.seed_for(79), 16
    b = S.Batch(S.EA, 3, L, 2, seed)
    outs = []
    for use_dcb in (True, False):
        spins = torch.zeros(2 * L ** 3, dtype=torch.int8, device=DEV)
        coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV)
        S.spin_init(b, spins, coup)
        dE = torch.zeros(2, dtype=torch.int64, device=DEV)
        if use_dcb:
            S.dcb_sweep(b, spins, [0.3, 0.8], 3, 5, L, 1, couplings=coup, dE_accum=dE)
        else:
            S.metropolis_sweep(b, spins, [0.3, 0.8], 3, 5, couplings=coup, dE_accum=dE)
        outs.append((_host(spins).copy(), _host(dE).copy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_dcb3d_64_every_site():
    """64^3, 16^3 tiles (B = 4), 4 hits, 2 sweeps, every site."""
    seed, L = W.seed_for(80), 64
    got_s, got_dE = _gpu3(S.ISING, L, 1, [0.22], seed, [(0, 2)], 4, False)
    ref_s, ref_dE = _oracle3(S.ISING, L, 1, [0.22], seed, 0, 2, 4, False)
    assert np.array_equal(got_s, ref_s) and np.array_equal(got_dE, ref_dE)


def test_dcb3d_beta_zero_in_the_batch():
    """A replica at beta = 0 (threshold 2^32: every attempt flips) beside one
    at beta = 0.5, both orders, on one tile and on 2^3 tiles."""
    seed = W.seed_for(81)
    for L, pal in ((16, True), (32, False)):
        got_s, got_dE = _gpu3(S.EA, L, 2, [0.0, 0.5], seed, [(1, 2)], 3, pal)
        ref_s, ref_dE = _oracle3(S.EA, L, 2, [0.0, 0.5], seed, 1, 2, 3, pal)
        assert np.array_equal(got_s, ref_s) and np.array_equal(got_dE, ref_dE)
