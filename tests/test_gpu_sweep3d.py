"""GPU parity of the 3D Ising / EA sweeps on 16-site row segments against the
oracle's plain checkerboard sweeps (Eq. 2 on the simple cubic lattice):
spins and energy changes bit-exact, for the one-pass kernel
(k_ising3d_pass: strips of rows streamed along z; taken from edge 512 up,
and with SPINMC_SWEEP3D_PASS=1 from 32) and the two half-sweep launches
(k_ising3d_half: smaller edges, SPINMC_SWEEP3D_PASS=0, and every edge of
16)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1101_1427_amd as S
import workloads as W
from tests import refrun

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _run(model, L, n_rep, rps, betas, t0, n, seed):
    b = S.Batch(model, 3, L, n_rep, seed, rep_per_sample=rps)
    spins = torch.zeros(b.spins_shape()[0], dtype=torch.int8, device=DEV)
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV) if model == S.EA else None
    S.spin_init(b, spins, coup)
    dE = torch.zeros(n_rep, dtype=torch.int64, device=DEV)
    S.metropolis_sweep(b, spins, betas, t0, n, couplings=coup, dE_accum=dE)
    torch.cuda.synchronize()
    ref_s, ref_c = refrun.init_uniform(model, 3, L, n_rep, seed, rps)
    ref_dE = refrun.sweep_uniform(model, 3, L, ref_s, ref_c, betas, seed, t0, n, rps)
    return b, spins.cpu().numpy().reshape(ref_s.shape), dE.cpu().numpy(), ref_s, ref_dE


@pytest.mark.parametrize("pass3d", ["1", "0"])
@pytest.mark.parametrize("model,L,n_rep,rps,t0,n", [
    (S.ISING, 16, 3, 1, 0, 9), (S.EA, 16, 4, 2, 5, 7), (S.EA, 32, 3, 1, 1, 6), (S.ISING, 48, 2, 1, 3, 4),
    (S.EA, 80, 2, 2, 2, 3), (S.ISING, 64, 2, 1, 4, 1)])
def test_sweeps_bit_exact(monkeypatch, pass3d, model, L, n_rep, rps, t0, n):
    """Several temperatures per batch (from the disordered phase to deep in
    the ordered one), shared coupling samples, odd first sweep indices, odd
    and even sweep counts, edges with 1 to 5 segments per row (48 and 80: rows
    cross wavefront bounds)."""
    monkeypatch.setenv("SPINMC_SWEEP3D_PASS", pass3d)
    betas = np.linspace(0.12, 1.3, n_rep)
    b, got, dE, ref, ref_dE = _run(model, L, n_rep, rps, betas, t0, n, W.seed_for(40))
    assert S.sweep_plan(b)[1] == ("k_ising3d_pass" if pass3d == "1" and L >= 32 else "k_ising3d_half")
    assert np.array_equal(got, ref)
    assert np.array_equal(dE, ref_dE)


@pytest.mark.parametrize("ty,segs", [("8", "1"), ("8", "2"), ("16", "1"), ("16", "2")])
def test_pass_launch_shapes_bit_exact(monkeypatch, ty, segs):
    """Rows per strip and segments per thread of the one-pass kernel change
    the schedule only (two segments per thread need an even number of
    segments per row; 48 and 80 fall back to one)."""
    monkeypatch.setenv("SPINMC_SWEEP3D_PASS", "1")
    monkeypatch.setenv("SPINMC_PASS3D_TY", ty)
    monkeypatch.setenv("SPINMC_PASS3D_SEGS", segs)
    for model, L, n_rep, rps in ((S.EA, 48, 3, 3), (S.ISING, 32, 2, 1), (S.EA, 64, 2, 1), (S.ISING, 80, 1, 1)):
        betas = np.linspace(0.15, 0.9, n_rep)
        b, got, dE, ref, ref_dE = _run(model, L, n_rep, rps, betas, 3, 5, W.seed_for(46))
        assert S.sweep_plan(b)[1] == "k_ising3d_pass"
        assert np.array_equal(got, ref) and np.array_equal(dE, ref_dE)


@pytest.mark.parametrize("model,L", [(S.ISING, 512), (S.EA, 512), (S.ISING, 1024), (S.EA, 1024)])
def test_pass_equals_half_sweeps_at_bench_sizes(monkeypatch, model, L):
    """At the bench's large edges the one-pass kernel (its default launch
    shape) and the two half-sweep launches give the same spins and energy
    changes after three sweeps (the half-sweep kernel is bit-exact against
    the oracle above)."""
    outs = []
    for flag in ("1", "0"):
        monkeypatch.setenv("SPINMC_SWEEP3D_PASS", flag)
        b = S.Batch(model, 3, L, 1, W.seed_for(47))
        spins = torch.zeros(L ** 3, dtype=torch.int8, device=DEV)
        coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV) if model == S.EA else None
        S.spin_init(b, spins, coup)
        dE = torch.zeros(1, dtype=torch.int64, device=DEV)
        S.metropolis_sweep(b, spins, [0.2216], 7, 3, couplings=coup, dE_accum=dE)
        torch.cuda.synchronize()
        outs.append((spins.cpu().numpy(), int(dE.cpu()[0])))
        del spins, coup
        torch.cuda.empty_cache()
    assert outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][0], outs[1][0])


@pytest.mark.parametrize("model,L,D", [(S.ISING, 256, 256), (S.EA, 512, 256), (S.ISING, 512, 512),
                                         (S.EA, 1024, 512)])
def test_pass_long_z_segments_equal_half_sweeps(monkeypatch, model, L, D):
    """z segments of 256 and 512 planes (one segment per strip when D = L,
    whose halo planes wrap onto the strip itself) give the same spins and
    energy changes as the two half-sweep launches, over three sweeps from an
    odd start."""
    outs = []
    for flag in ("1", "0"):
        monkeypatch.setenv("SPINMC_SWEEP3D_PASS", flag)
        if flag == "1":
            monkeypatch.setenv("SPINMC_PASS3D_D", str(D))
        else:
            monkeypatch.delenv("SPINMC_PASS3D_D", raising=False)
        b = S.Batch(model, 3, L, 1, W.seed_for(49))
        spins = torch.zeros(L ** 3, dtype=torch.int8, device=DEV)
        coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV) if model == S.EA else None
        S.spin_init(b, spins, coup)
        dE = torch.zeros(1, dtype=torch.int64, device=DEV)
        assert S.sweep_plan(b)[1] == ("k_ising3d_pass" if flag == "1" else "k_ising3d_half")
        S.metropolis_sweep(b, spins, [0.2216], 7, 3, couplings=coup, dE_accum=dE)
        torch.cuda.synchronize()
        outs.append((spins.cpu().numpy(), int(dE.cpu()[0])))
        del spins, coup
        torch.cuda.empty_cache()
    assert outs[0][1] == outs[1][1]
    assert np.array_equal(outs[0][0], outs[1][0])


@pytest.mark.parametrize("model,n,t0", [(S.ISING, 2, 5), (S.EA, 1, 2)])
def test_pass_bit_exact_at_512(model, n, t0):
    """The one-pass kernel in its default launch shape at the bench's 512^3
    edge against the oracle, every site (about 11 s of oracle time per sweep):
    an even sweep count ends in the caller's buffer, an odd one is copied
    back."""
    b, got, dE, ref, ref_dE = _run(model, 512, 1, 1, [0.2216], t0, n, W.seed_for(48))
    assert S.sweep_plan(b)[1] == "k_ising3d_pass"
    assert np.array_equal(dE, ref_dE)
    assert np.array_equal(got, ref)


def test_beta_zero_replica_takes_the_generic_kernels():
    """A replica at beta = 0 (threshold 2^32, whose high half does not fit 16
    bits) sends the call to the per-site kernels; results stay exact."""
    b, got, dE, ref, ref_dE = _run(S.ISING, 32, 2, 1, [0.0, 0.3], 0, 3, W.seed_for(41))
    assert np.array_equal(got, ref) and np.array_equal(dE, ref_dE)


@pytest.mark.parametrize("model,L,n", [(S.ISING, 256, 2), (S.EA, 128, 3), (S.ISING, 128, 4)])
def test_large_lattice_bit_exact(model, L, n):
    """The bench workload's edge (256) and a 128^3 EA sample, every site: at
    these sizes heads equal to a threshold's high half occur in every sweep,
    so the exact (tail) decisions are exercised too."""
    b, got, dE, ref, ref_dE = _run(model, L, 1, 1, [0.2216], 11, n, W.seed_for(42))
    assert np.array_equal(got, ref)
    assert np.array_equal(dE, ref_dE)


def test_equals_generic_kernels(monkeypatch):
    """The segment kernel and the per-site kernels give the same chain."""
    outs = []
    monkeypatch.setenv("SPINMC_SWEEP3D_PASS", "1")
    for flag in ("1", "0"):
        monkeypatch.setenv("SPINMC_SWEEP3D", flag)
        b = S.Batch(S.EA, 3, 64, 2, W.seed_for(43))
        assert S.sweep_plan(b)[1] == ("k_ising3d_pass" if flag == "1" else "k_half_sweep_generic")
        spins = torch.zeros(b.spins_shape()[0], dtype=torch.int8, device=DEV)
        coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV)
        S.spin_init(b, spins, coup)
        dE = torch.zeros(2, dtype=torch.int64, device=DEV)
        S.metropolis_sweep(b, spins, [0.25, 0.9], 100, 20, couplings=coup, dE_accum=dE)
        torch.cuda.synchronize()
        outs.append((spins.cpu().numpy(), dE.cpu().numpy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("z,nt", [("1", "0"), ("2", "1"), ("4", "0"), ("4", "1"), ("8", "1"), ("16", "1")])
def test_launch_shapes_bit_exact(monkeypatch, z, nt):
    """Rows per thread along z (1 to 16; reduced to a divisor of (L / 16)^3,
    so 1 at L = 16 and 48, at most 8 at L = 32) and non-temporal stores do
    not change the chain."""
    monkeypatch.setenv("SPINMC_SWEEP3D_Z", z)
    monkeypatch.setenv("SPINMC_SWEEP3D_NT", nt)
    monkeypatch.setenv("SPINMC_SWEEP3D_PASS", "0")
    for model, L, n_rep, rps in ((S.EA, 48, 3, 2), (S.ISING, 16, 2, 1), (S.EA, 32, 2, 1), (S.ISING, 64, 2, 1)):
        betas = np.linspace(0.15, 0.9, n_rep)
        b, got, dE, ref, ref_dE = _run(model, L, n_rep, rps, betas, 3, 5, W.seed_for(44))
        assert np.array_equal(got, ref) and np.array_equal(dE, ref_dE)


@pytest.mark.parametrize("pack", ["1", "0"])
def test_ea_bond_forms_bit_exact(monkeypatch, pack):
    """EA calls of four or more sweeps read bit-packed bonds (SPINMC_SWEEP3D_PACK=0:
    the int8 bonds); both match the oracle, with samples shared by two replicas."""
    monkeypatch.setenv("SPINMC_SWEEP3D_PACK", pack)
    monkeypatch.setenv("SPINMC_SWEEP3D_PASS", "0")
    betas = np.linspace(0.2, 1.1, 4)
    b, got, dE, ref, ref_dE = _run(S.EA, 48, 4, 2, betas, 9, 6, W.seed_for(45))
    assert np.array_equal(got, ref) and np.array_equal(dE, ref_dE)
