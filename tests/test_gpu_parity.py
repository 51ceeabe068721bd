"""GPU parity: the HIP library through its C ABI against the CPU oracle.

Ising / EA results must be bit-exact (spins, energies, permutations, swap
counts); Heisenberg results are compared within float32 tolerances.
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1101_1427_amd as S
import workloads as W
from oracle import oracle as O
from tests import refrun

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def gpu_init(batch: S.Batch):
    per = 3 if batch.model == S.HEISENBERG else 1
    dtype = torch.float32 if batch.model == S.HEISENBERG else torch.int8
    spins = torch.zeros(batch.spins_shape()[0], dtype=dtype, device=DEV)
    coup = None
    if batch.model == S.EA:
        coup = torch.zeros(batch.coup_len(), dtype=torch.int8, device=DEV)
    S.spin_init(batch, spins, coup)
    return spins, coup


# --------------------------------------------------------------- spin init --
@pytest.mark.parametrize("model,dim,L,n_rep,rps", [(S.ISING, 2, 64, 3, 1), (S.EA, 2, 48, 4, 2),
                                                    (S.EA, 3, 16, 3, 1), (S.ISING, 3, 6, 2, 1)])
def test_spin_init_bit_exact(model, dim, L, n_rep, rps):
    seed = W.seed_for(11)
    b = S.Batch(model, dim, L, n_rep, seed, rep_per_sample=rps)
    spins, coup = gpu_init(b)
    ref_s, ref_c = refrun.init_uniform(model, dim, L, n_rep, seed, rps)
    assert np.array_equal(_host(spins).reshape(ref_s.shape), ref_s)
    if model == S.EA:
        assert np.array_equal(_host(coup).reshape(ref_c.shape), ref_c)


def test_heisenberg_init_matches_within_float32():
    seed = W.seed_for(12)
    b = S.Batch(S.HEISENBERG, 3, 16, 2, seed)
    spins, _ = gpu_init(b)
    ref, _ = refrun.init_uniform(refrun.HEIS, 3, 16, 2, seed)
    got = _host(spins).reshape(ref.shape).astype(np.float64)
    assert np.abs(got - ref).max() < 1e-6


# ----------------------------------------------------------- small config --
def test_ising_64_critical_1000_sweeps_bit_exact():
    """64 x 64, beta = ln(1+sqrt 2)/2, 1000 sweeps: spins equal after every 100."""
    cfg = W.ising_small()
    b = S.Batch(S.ISING, 2, cfg.L, 1, cfg.seed)
    spins, _ = gpu_init(b)
    ref = O.init_spins(2, cfg.L, cfg.seed, 0)
    E0 = O.energy(2, cfg.L, None, ref)
    dE = torch.zeros(1, dtype=torch.int64, device=DEV)
    for k in range(0, cfg.sweeps, 100):
        S.metropolis_sweep(b, spins, [cfg.betas[0]], k, 100, dE_accum=dE)
        O.run(2, cfg.L, None, ref, cfg.betas[0], cfg.seed, 0, k, 100)
        assert np.array_equal(_host(spins), ref), f"diverged before sweep {k + 100}"
    assert int(_host(dE)[0]) == O.energy(2, cfg.L, None, ref) - E0


@pytest.mark.parametrize("model,dim,L", [
    (S.ISING, 2, 4), (S.ISING, 2, 6), (S.EA, 2, 18), (S.ISING, 2, 36), (S.EA, 2, 48), (S.ISING, 2, 130),
    (S.EA, 2, 64), (S.ISING, 3, 4), (S.EA, 3, 6), (S.ISING, 3, 10), (S.EA, 3, 16)])
def test_sweeps_bit_exact_many_shapes(model, dim, L):
    seed = W.seed_for(13)
    n_rep, rps = 3, 2
    betas = [0.25, 0.6, 1.1]
    b = S.Batch(model, dim, L, n_rep, seed, rep_per_sample=rps)
    spins, coup = gpu_init(b)
    ref_s, ref_c = refrun.init_uniform(model, dim, L, n_rep, seed, rps)
    dE = torch.zeros(n_rep, dtype=torch.int64, device=DEV)
    S.metropolis_sweep(b, spins, betas, 7, 12, couplings=coup, dE_accum=dE)
    ref_dE = refrun.sweep_uniform(model, dim, L, ref_s, ref_c, betas, seed, 7, 12, rps)
    assert np.array_equal(_host(spins).reshape(ref_s.shape), ref_s)
    assert np.array_equal(_host(dE), ref_dE)


def test_uneven_batch_bit_exact():
    seed = W.seed_for(14)
    inst = refrun.uneven_table(2, [8, 32, 6, 48, 16], 2)
    b = S.Batch(S.EA, 2, 0, len(inst), seed, inst=inst)
    spins, coup = gpu_init(b)
    ref_s, ref_c = refrun.init_uneven(S.EA, 2, inst, seed)
    assert np.array_equal(_host(spins), ref_s)
    assert np.array_equal(_host(coup), ref_c)
    betas = np.linspace(0.3, 1.2, len(inst))
    S.metropolis_sweep(b, spins, betas, 0, 9, couplings=coup)
    for rep, (L, q, so, co) in enumerate(inst):
        N = L * L
        s = ref_s[so:so + N]
        O.run(2, int(L), ref_c[co:co + 2 * N], s, float(betas[rep]), seed, rep, 0, 9)
    assert np.array_equal(_host(spins), ref_s)


def test_closed_form_temperatures_on_gpu():
    seed = W.seed_for(15)
    b = S.Batch(S.EA, 3, 8, 2, seed)
    spins, coup = gpu_init(b)
    s0 = _host(spins).copy()
    S.metropolis_sweep(b, spins, [0.0, 0.0], 0, 3, couplings=coup)
    assert np.array_equal(_host(spins), -s0)      # beta = 0: every spin flips each sweep
    up = torch.ones(2 * 512, dtype=torch.int8, device=DEV)
    S.metropolis_sweep(S.Batch(S.ISING, 3, 8, 2, seed), up, [1e3, 1e3], 0, 2)
    assert bool((up == 1).all())                  # beta = inf: the ground state stays


@pytest.mark.parametrize("beta", [0.30, W.BETA_C_2D, 0.50])
def test_ising_1024_crop_bit_exact(beta):
    """Independent 1024^2 periodic lattice with the large configuration's seed."""
    cfg = W.ising_large()
    L, n = 1024, 12
    b = S.Batch(S.ISING, 2, L, 1, cfg.seed)
    spins, _ = gpu_init(b)
    ref = O.init_spins(2, L, cfg.seed, 0)
    S.metropolis_sweep(b, spins, [beta], 100, n)
    O.run(2, L, None, ref, beta, cfg.seed, 0, 100, n)
    assert np.array_equal(_host(spins), ref)


# ------------------------------------------------------------- measurement --
@pytest.mark.parametrize("model,dim,L", [(S.ISING, 2, 64), (S.EA, 2, 48), (S.EA, 3, 16), (S.ISING, 3, 6)])
def test_measure_exact(model, dim, L):
    seed = W.seed_for(16)
    n_rep = 3
    b = S.Batch(model, dim, L, n_rep, seed)
    spins, coup = gpu_init(b)
    E = torch.zeros(n_rep, dtype=torch.float64, device=DEV)
    M = torch.zeros(n_rep, dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E, M, couplings=coup)
    ref_s, ref_c = refrun.init_uniform(model, dim, L, n_rep, seed)
    for r in range(n_rep):
        J = None if ref_c is None else ref_c[r]
        assert _host(E)[r] == O.energy(dim, L, J, ref_s[r])
        assert _host(M)[r] == O.magnetisation(dim, L, ref_s[r])


def test_measure_heisenberg_fp64():
    """float64 reductions of float32 spins: the oracle's own start rounded to
    float32 is measured by both sides."""
    seed = W.seed_for(17)
    L, n_rep = 16, 2
    ref, _ = refrun.init_uniform(refrun.HEIS, 3, L, n_rep, seed)
    ref32 = ref.astype(np.float32)
    b = S.Batch(S.HEISENBERG, 3, L, n_rep, seed)
    spins = _dev(ref32.reshape(-1))
    E = torch.zeros(n_rep, dtype=torch.float64, device=DEV)
    M = torch.zeros(n_rep, 3, dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E, M)
    N = L ** 3
    for r in range(n_rep):
        exact = np.ascontiguousarray(ref32[r].astype(np.float64))
        assert abs(_host(E)[r] - O.heis_energy(3, L, exact)) <= 2 ** -20 * N
        assert np.allclose(_host(M)[r], O.heis_magnetisation(3, L, exact), atol=1e-9)


# ------------------------------------------------------------- Heisenberg --
def test_heisenberg_first_sweep_within_tolerance():
    """One sweep at beta = 0.693 from each side's own start: components agree to
    1e-5 wherever the accept decisions agree; decisions may differ only where
    u is within float32 rounding of exp(-beta dE)."""
    seed = W.seed_for(18)
    L, beta = 16, 0.693
    b = S.Batch(S.HEISENBERG, 3, L, 1, seed, renorm_every=16)
    spins, _ = gpu_init(b)
    ref = O.init_heis(3, L, seed, 0)
    S.metropolis_sweep(b, spins, [beta], 0, 1)
    O.heis_sweep(3, L, ref, beta, seed, 0, 0, 16)
    got = _host(spins).astype(np.float64).reshape(-1, 3)
    dev = np.abs(got - ref).max(axis=1)
    mismatches = int((dev > 1e-5).sum())
    assert mismatches <= max(4, int(16 * L ** 3 * 2.0 ** -24))
    assert np.abs(np.linalg.norm(got, axis=1) - 1).max() < 1e-6


# --------------------------------------------------------- parallel tempering --
def _pt_case(model, dim, sizes, n_temps, steps, seed, beta, m=1):
    inst = refrun.uneven_table(dim, sizes, n_temps, model)
    n_chains = len(sizes)
    b = S.Batch(model, dim, 0, len(inst), seed, inst=inst)
    spins, coup = gpu_init(b)
    E = torch.zeros(len(inst), dtype=torch.float64, device=DEV)
    S.measure_energy_magnetisation(b, spins, E, couplings=coup)
    sot = torch.arange(n_temps, dtype=torch.int32, device=DEV).repeat(n_chains)
    acc = torch.zeros(n_chains * (n_temps - 1), dtype=torch.int64, device=DEV)
    S.pt_sweep_swap(b, n_chains, n_temps, beta, spins, sot, E, 0, steps // 2, couplings=coup, swap_accepts=acc,
                    sweeps_per_step=m)
    S.pt_sweep_swap(b, n_chains, n_temps, beta, spins, sot, E, steps // 2, steps - steps // 2, couplings=coup,
                    swap_accepts=acc, sweeps_per_step=m)
    # oracle
    ref_s, ref_c = refrun.init_uneven(model, dim, inst, seed)
    for q, L in enumerate(sizes):
        N = int(L) ** dim
        rows = inst[q * n_temps:(q + 1) * n_temps]
        so0, co = int(rows[0][2]), int(rows[0][3])
        chain = ref_s[so0:so0 + n_temps * N].reshape(n_temps, N).copy()
        J = ref_c[co:co + dim * N] if ref_c is not None else None
        Eq = np.array([O.energy(dim, int(L), J, chain[k]) for k in range(n_temps)], np.int64)
        sq = np.arange(n_temps, dtype=np.int32)
        aq = np.zeros(n_temps, np.uint64)
        O.pt_run(dim, int(L), J, chain, beta, sq, Eq, seed, q, q * n_temps, 0, steps, aq, sweeps_per_step=m)
        assert np.array_equal(_host(spins)[so0:so0 + n_temps * N].reshape(n_temps, N), chain), q
        assert np.array_equal(_host(sot)[q * n_temps:(q + 1) * n_temps], sq), q
        assert np.array_equal(_host(E)[q * n_temps:(q + 1) * n_temps], Eq.astype(np.float64)), q
        assert np.array_equal(_host(acc)[q * (n_temps - 1):(q + 1) * (n_temps - 1)], aq[:n_temps - 1].astype(np.int64))


def test_pt_uneven_2d_bit_exact():
    _pt_case(S.EA, 2, [8, 12, 32, 6], 5, 40, W.seed_for(19), W.geometric_ladder(0.5, 2.0, 5))


def test_pt_generic_sweeps_per_step():
    """Four sweeps between exchange rounds on the generic kernels."""
    _pt_case(S.EA, 2, [8, 12, 6], 4, 11, W.seed_for(23), W.geometric_ladder(0.5, 2.0, 4), m=4)


def test_pt_3d_bit_exact():
    _pt_case(S.EA, 3, [4, 6, 4], 8, 30, W.seed_for(20), W.geometric_ladder(0.8, 2.0, 8))


def test_pt_ising_equal_betas_walk():
    _pt_case(S.ISING, 2, [8, 8], 4, 9, W.seed_for(21), np.full(4, 0.4))


# ------------------------------------------- one-pass split-layout 2D kernel --
@pytest.mark.parametrize("L,n_rep,n,sweep0", [(1024, 2, 5, 0), (2048, 1, 4, 33), (1024, 3, 1, 7), (1024, 1, 2, 3),
                                               (4096, 2, 3, 0), (2048, 3, 2, 11)])
def test_split_kernel_bit_exact(L, n_rep, n, sweep0):
    """Uniform 2D Ising batches served by the one-pass kernel: odd and even
    sweep counts, nonzero first sweep index, per-replica beta, dE tracking."""
    seed = W.seed_for(22)
    b = S.Batch(S.ISING, 2, L, n_rep, seed)
    assert S.sweep_plan(b) == (1, "k_ising2d_split")
    spins, _ = gpu_init(b)
    betas = [0.30, W.BETA_C_2D, 0.55][:n_rep]
    dE = torch.zeros(n_rep, dtype=torch.int64, device=DEV)
    S.metropolis_sweep(b, spins, betas, sweep0, n, dE_accum=dE)
    ref_s, _ = refrun.init_uniform(S.ISING, 2, L, n_rep, seed)
    ref_dE = refrun.sweep_uniform(S.ISING, 2, L, ref_s, None, betas, seed, sweep0, n)
    assert np.array_equal(_host(spins).reshape(ref_s.shape), ref_s)
    assert np.array_equal(_host(dE), ref_dE)


def test_split_kernel_launch_shape_invariance(monkeypatch):
    """Band heights (equal or split between the two halves of the grid) and
    lane width change the schedule, never the result."""
    seed = W.seed_for(23)
    L = 8192
    b = S.Batch(S.ISING, 2, L, 1, seed)
    outs = []
    for chunks, H, h1, h2 in [(1, 64, 0, 0), (2, 16, 0, 0), (1, 4, 0, 0), (2, 128, 0, 0), (2, 32, 0, 0),
                              (2, 32, 36, 28), (1, 16, 20, 12), (2, 32, 8, 56)]:
        monkeypatch.setenv("SPINMC_L2D_CHUNKS", str(chunks))
        monkeypatch.setenv("SPINMC_L2D_H", str(H))
        monkeypatch.setenv("SPINMC_L2D_H1", str(h1))
        monkeypatch.setenv("SPINMC_L2D_H2", str(h2))
        spins, _ = gpu_init(b)
        dE = torch.zeros(1, dtype=torch.int64, device=DEV)
        S.metropolis_sweep(b, spins, [0.42], 0, 6, dE_accum=dE)
        outs.append((_host(spins).copy(), int(_host(dE)[0])))
    for s, d in outs[1:]:
        assert np.array_equal(s, outs[0][0]) and d == outs[0][1]


@pytest.mark.parametrize("L,n_rep", [(1024, 3), (2048, 1), (8192, 1)])
def test_split_kernel_fused_layout_equals_separate_conversions(monkeypatch, L, n_rep):
    """The first sweep reading the caller's rows and the last writing them
    back give the same spins and energy changes as converting to the split
    layout before the sweeps and back after them, for 1 to 4 sweeps."""
    seed = W.seed_for(24)
    b = S.Batch(S.ISING, 2, L, n_rep, seed)
    betas = [0.30, W.BETA_C_2D, 0.55][:n_rep]
    for n in (1, 2, 3, 4):
        outs = []
        for fuse in ("1", "0"):
            monkeypatch.setenv("SPINMC_L2D_FUSE", fuse)
            spins, _ = gpu_init(b)
            dE = torch.zeros(n_rep, dtype=torch.int64, device=DEV)
            S.metropolis_sweep(b, spins, betas, 5, n, dE_accum=dE)
            outs.append((_host(spins).copy(), _host(dE).copy()))
        assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1]), n


# ------------------------------------------------- LDS-resident small lattices --
@pytest.mark.parametrize("model,L,n_rep,rps", [(S.ISING, 16, 5, 1), (S.EA, 64, 4, 2), (S.EA, 256, 8, 1)])
def test_small_lattice_sweeps_in_lds(model, L, n_rep, rps):
    """Uniform 2D batches of edge 16 .. 128 (and edge 256 with at least 2^19
    sites in the batch) keep each replica in LDS for up to 256 sweeps per
    launch: 300 sweeps (two launches) bit-exact against the oracle."""
    seed = W.seed_for(24)
    betas = np.linspace(0.3, 1.0, n_rep)
    b = S.Batch(model, 2, L, n_rep, seed, rep_per_sample=rps)
    assert S.sweep_plan(b)[1] == "k_uneven2d_sweep"
    spins, coup = gpu_init(b)
    dE = torch.zeros(n_rep, dtype=torch.int64, device=DEV)
    n = 300 if L <= 64 else 40
    S.metropolis_sweep(b, spins, betas, 11, n, couplings=coup, dE_accum=dE)
    ref_s, ref_c = refrun.init_uniform(model, 2, L, n_rep, seed, rps)
    ref_dE = refrun.sweep_uniform(model, 2, L, ref_s, ref_c, betas, seed, 11, n, rps)
    assert np.array_equal(_host(spins).reshape(ref_s.shape), ref_s)
    assert np.array_equal(_host(dE), ref_dE)


def test_small_lattice_lds_path_equals_generic(monkeypatch):
    """The LDS path and the generic kernels agree on a call that crosses the
    256-sweep chunk boundary at an odd sweep index; one replica of edge 256
    takes the generic kernels."""
    assert S.sweep_plan(S.Batch(S.ISING, 2, 256, 1, 1))[1] == "k_half_sweep_generic"
    seed, L, n_rep = W.seed_for(25), 32, 3
    betas = [0.4, 0.44, 0.6]
    outs = []
    for lds in ("1", "0"):
        monkeypatch.setenv("SPINMC_SWEEP_LDS2D", lds)
        b = S.Batch(S.EA, 2, L, n_rep, seed)
        spins, coup = gpu_init(b)
        dE = torch.zeros(n_rep, dtype=torch.int64, device=DEV)
        S.metropolis_sweep(b, spins, betas, 255, 520, couplings=coup, dE_accum=dE)
        outs.append((_host(spins).copy(), _host(dE).copy()))
    assert S.sweep_plan(S.Batch(S.EA, 2, L, n_rep, seed))[1] == "k_half_sweep_generic"
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
