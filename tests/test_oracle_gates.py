"""The stored digests of the full-length gates (tests/golden/gate_hashes.txt)
are complete and still what the oracle computes: the fixture lists every
checkpoint of every chain, and the cheapest row (a 32^2 chain of the uneven
batch at its first checkpoint) is recomputed here from the oracle."""
import importlib.util
import os

import numpy as np

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "gate_hashes.txt")


def _gen():
    spec = importlib.util.spec_from_file_location("make_gate_hashes", os.path.join(HERE, "golden", "make_gate_hashes.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def _rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, key, step, hs, hst, e, a = line.split()
                rows.append((k, int(key), int(step), hs, hst, int(e), int(a)))
    return rows


def test_fixture_lists_every_chain_and_checkpoint():
    g = _gen()
    rows = _rows()
    keys = {(r[0], r[1], r[2]) for r in rows}
    assert len(keys) == len(rows)
    want = {("crop2d", k, s) for k in range(3) for s in g.CROP_CHECKPOINTS}
    want |= {("pt3d", q, s) for q in g.pt3d_chains() for s in g.PT3D_CHECKPOINTS}
    c5 = W.ea2d_uneven()
    want |= {("uneven2d", q, s) for q in g.uneven_chains(c5.sizes) for s in g.UNEVEN_CHECKPOINTS}
    assert keys == want
    assert len(g.pt3d_chains()) == 64 and len({q // 2 for q in g.pt3d_chains()}) == 32
    assert {int(c5.sizes[q]) for q in g.uneven_chains(c5.sizes)} == set(W.UNEVEN_SIZES)
    assert g.PT3D_CHECKPOINTS[-1] == W.ea3d_tempering().steps
    assert g.UNEVEN_CHECKPOINTS[-1] == c5.steps
    assert g.CROP_CHECKPOINTS[-1] == W.ising_large().sweeps


def test_smallest_uneven_chain_recomputed():
    g = _gen()
    c5 = W.ea2d_uneven()
    q = min(g.uneven_chains(c5.sizes), key=lambda q: (int(c5.sizes[q]), q))
    L = int(c5.sizes[q])
    assert L == 32
    step = g.UNEVEN_CHECKPOINTS[0]
    rows = g.chain_job(("uneven2d", 2, L, c5.seed, q, c5.n_temps, q, list(c5.betas), (step,)))
    want = [r for r in _rows() if r[0] == "uneven2d" and r[1] == q and r[2] == step]
    assert len(want) == 1 and rows[0][:7] == want[0]
    assert rows[0][7] == 0


def test_digests_see_every_part_of_the_state():
    g = _gen()
    a = np.ones((4, 16), np.int8)
    b = a.copy()
    b[3, 15] = -1
    assert g.spins_digest(a) != g.spins_digest(b)
    sq, E, acc = np.arange(4, dtype=np.int32), np.array([-8, 0, 4, 8], np.int64), np.zeros(3, np.int64)
    base = g.state_digest(sq, E, acc)
    assert g.state_digest(sq[[1, 0, 2, 3]], E, acc) != base
    assert g.state_digest(sq, E + np.array([0, 0, 0, 4]), acc) != base
    assert g.state_digest(sq, E, acc + np.array([0, 0, 1])) != base


def test_heisenberg_series_first_sweep_recomputed():
    """The stored float64 energy series of the 256^3 Heisenberg workload has
    one value per sweep and starts with what the oracle computes for sweep 0
    (about four seconds)."""
    from oracle import oracle as O

    rows = []
    with open(os.path.join(HERE, "golden", "heis3d_L256_energy.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                t, e = line.split()
                assert int(t) == len(rows)
                rows.append(float(e))
    cfg = W.heisenberg_3d()
    assert len(rows) == cfg.sweeps
    L = cfg.L
    s = O.init_heis(3, L, cfg.seed, 0)
    O.heis_run(3, L, s, cfg.betas[0], cfg.seed, 0, 0, 1, cfg.renorm_every)
    assert O.heis_energy(3, L, s) / L ** 3 == rows[0]
    # relaxing from a random start: the energy falls, and stays above the
    # ground state (-3 per site)
    assert rows[0] > rows[100] > -3.0 and min(rows) > -3.0
