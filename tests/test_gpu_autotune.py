"""smc_autotune: measures and records launch shapes (the workgroup size of
the LDS-resident 2D kernel, the band height of the one-pass 2D Ising sweep,
the strip shape of the one-pass 3D sweep, the rows per thread of the 3D
half-sweeps), reads them back from its cache file, and never changes
results."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1101_1427_amd as S
import workloads as W

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _sweep(b, seed_spins=True):
    spins = torch.zeros(b.spins_shape()[0], dtype=torch.int8, device=DEV)
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV)
    S.spin_init(b, spins, coup)
    dE = torch.zeros(b.n_rep, dtype=torch.int64, device=DEV)
    S.metropolis_sweep(b, spins, np.linspace(0.3, 1.0, b.n_rep), 3, 40, couplings=coup, dE_accum=dE)
    torch.cuda.synchronize()
    return spins.cpu().numpy(), dE.cpu().numpy()


def test_autotune_writes_reads_and_keeps_results(tmp_path, monkeypatch):
    path = tmp_path / "spinmc_tune.txt"
    b = S.Batch(S.EA, 2, 48, 6, W.seed_for(101))
    monkeypatch.setenv("SPINMC_U2D_THREADS", "64")
    ref = _sweep(b)
    monkeypatch.delenv("SPINMC_U2D_THREADS")
    S.autotune(b, str(path))
    lines = [l.split() for l in path.read_text().splitlines() if not l.startswith("#")]
    assert any(l[1] == "u2d" and int(l[2]) == 48 and int(l[3]) == 1 and int(l[5]) in (64, 128, 256, 512)
               for l in lines)
    # a second call reads the file (nothing new to measure) and keeps its lines
    before = path.read_text()
    S.autotune(b, str(path))
    assert path.read_text() == before
    got = _sweep(b)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])


def _run(b, n, t0=5):
    spins = torch.zeros(b.spins_shape()[0], dtype=torch.int8, device=DEV)
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device=DEV) if b.model == S.EA else None
    S.spin_init(b, spins, coup)
    dE = torch.zeros(b.n_rep, dtype=torch.int64, device=DEV)
    S.metropolis_sweep(b, spins, np.linspace(0.2, 0.5, b.n_rep), t0, n, couplings=coup, dE_accum=dE)
    torch.cuda.synchronize()
    return spins.cpu().numpy(), dE.cpu().numpy()


@pytest.mark.parametrize("model,dim,L,n_rep,kind", [
    (S.ISING, 2, 1024, 2, "band2d"), (S.ISING, 3, 512, 1, "pass3d"), (S.EA, 3, 512, 1, "pass3d"),
    (S.EA, 3, 64, 2, "half3d")])
def test_autotune_tile_shapes(tmp_path, model, dim, L, n_rep, kind):
    """The tuned shape is recorded for the batch's edge, model and replica
    count, read back by a second call, and the sweeps give the same spins and
    energy changes as with the default shapes."""
    path = tmp_path / "spinmc_tune.txt"
    b = S.Batch(model, dim, L, n_rep, W.seed_for(105), rep_per_sample=1)
    ref = _run(b, 3)
    S.autotune(b, str(path))
    lines = [l.split() for l in path.read_text().splitlines() if not l.startswith("#")]
    mine = [l for l in lines if l[1] == kind and int(l[2]) == L and int(l[3]) == (1 if model == S.EA else 0)
            and int(l[4]) == n_rep]
    assert len(mine) == 1, lines
    before = path.read_text()
    S.autotune(b, str(path))
    assert path.read_text() == before
    got = _run(b, 3)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
