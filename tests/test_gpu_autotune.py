"""smc_autotune: measures and records the workgroup sizes of the LDS-resident
2D kernel, reads them back, and never changes results."""
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
    assert any(int(l[1]) == 48 and int(l[2]) == 1 and int(l[3]) in (64, 128, 256, 512) for l in lines)
    # a second call reads the file (nothing new to measure) and keeps its lines
    before = path.read_text()
    S.autotune(b, str(path))
    assert path.read_text() == before
    got = _sweep(b)
    assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
