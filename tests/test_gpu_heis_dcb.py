"""GPU parity of the 2D Heisenberg double checkerboard (smc_heis_dcb_sweep)
in its three arithmetic modes against the float64 oracle (orc_heis_dcb_run).

Both sides start from the oracle's random start (rounded to float32 for the
float modes).  double: every component within 1e-12 and the same accepted
moves.  float / fast: the same random numbers, float32 rounding; components
within 1e-5 except where an accept decision sits within float32 rounding of
exp(-beta dE) (a handful of sites at most).  fast with one tile and one hit
is the plain sweep of smc_metropolis_sweep, bit for bit.  Long runs: every
mode samples the same energy as the oracle within the combined errors."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1101_1427_amd as S
import workloads as W
from oracle import exact as X
from oracle import oracle as O

pytestmark = pytest.mark.gpu

DEV = "cuda"
MODES = {"float": S.HEIS_FLOAT, "fast": S.HEIS_FAST, "double": S.HEIS_DOUBLE}


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _starts(L, n_rep, seed, mode):
    """The oracle's start per replica, as the GPU mode stores it (float32
    rounding for the float modes), and the same values in float64."""
    ref = [O.init_heis(2, L, seed, r) for r in range(n_rep)]
    if mode != S.HEIS_DOUBLE:
        ref = [x.astype(np.float32).astype(np.float64) for x in ref]
    dt = torch.float64 if mode == S.HEIS_DOUBLE else torch.float32
    spins = torch.tensor(np.concatenate([x.reshape(-1) for x in ref]), dtype=dt, device=DEV)
    return spins, [np.ascontiguousarray(x) for x in ref]


def _run_both(mode, L, T, k, pal, betas, seed, t0, n, renorm=16, cap=0.0):
    n_rep = len(betas)
    b = S.Batch(S.HEISENBERG, 2, L, n_rep, seed, renorm_every=renorm)
    spins, ref = _starts(L, n_rep, seed, mode)
    acc = torch.zeros(n_rep, dtype=torch.int64, device=DEV)
    S.heis_dcb_sweep(b, spins, betas, t0, n, T, k, precision=mode, palindromic=pal, cap=cap, accepts=acc)
    ref_acc = [O.heis_dcb_run(L, T, k, ref[r], betas[r], seed, r, t0, n, palindromic=pal, renorm_every=renorm,
                              cap=cap) for r in range(n_rep)]
    got = _host(spins).astype(np.float64).reshape(n_rep, L * L, 3)
    return got, np.stack(ref), _host(acc), np.array(ref_acc)


@pytest.mark.parametrize("L,T,k,pal", [(64, 16, 3, True), (64, 32, 2, False), (32, 32, 2, True), (128, 32, 1, False)])
def test_double_matches_oracle(L, T, k, pal):
    got, ref, acc, ref_acc = _run_both(S.HEIS_DOUBLE, L, T, k, pal, [0.4, 1.5, 3.0], W.seed_for(82), 14, 3)
    assert np.abs(got - ref).max() < 1e-12
    assert np.array_equal(acc, ref_acc)


@pytest.mark.parametrize("cap", [0.25, 2.0])
def test_double_small_steps_match_oracle(cap):
    """Small-step proposals (cap around the current direction) in float64."""
    got, ref, acc, ref_acc = _run_both(S.HEIS_DOUBLE, 64, 16, 3, False, [0.4, 1.5, 3.0], W.seed_for(87), 14, 3,
                                       cap=cap)
    assert np.abs(got - ref).max() < 1e-12
    assert np.array_equal(acc, ref_acc)


@pytest.mark.parametrize("mode", ["float", "fast"])
@pytest.mark.parametrize("L,T,k,pal,cap", [(64, 16, 2, False, 0.0), (128, 64, 2, True, 0.0), (64, 32, 3, False, 0.0),
                                           (64, 16, 2, False, 0.3), (64, 32, 2, True, 1.5)])
def test_float_modes_match_oracle_sitewise(mode, L, T, k, pal, cap):
    betas = [0.5, 1.5, 3.0]
    got, ref, acc, ref_acc = _run_both(MODES[mode], L, T, k, pal, betas, W.seed_for(83), 7, 1, cap=cap)
    dev = np.abs(got - ref).max(axis=2)
    mismatches = int((dev > 1e-5).sum())
    # a decision differs only where u is within a few float32 ulps of exp(-beta dE)
    attempts = len(betas) * L * L * k
    assert mismatches <= max(8, int(64 * attempts * 2.0 ** -21)), mismatches
    assert np.abs(acc - ref_acc).max() <= max(2, mismatches)


def test_fast_single_tile_single_hit_is_the_plain_sweep():
    """tile = L, hits = 1, fast arithmetic: the chain of smc_metropolis_sweep,
    bit for bit, across a renormalisation sweep."""
    seed, L, n_rep = W.seed_for(84), 64, 2
    betas = [0.7, 2.0]
    b = S.Batch(S.HEISENBERG, 2, L, n_rep, seed, renorm_every=16)
    outs = []
    for dcb in (True, False):
        spins = torch.zeros(n_rep * L * L * 3, dtype=torch.float32, device=DEV)
        S.spin_init(b, spins)
        acc = torch.zeros(n_rep, dtype=torch.int64, device=DEV)
        if dcb:
            S.heis_dcb_sweep(b, spins, betas, 10, 9, L, 1, precision=S.HEIS_FAST, accepts=acc)
        else:
            S.metropolis_sweep(b, spins, betas, 10, 9, dE_accum=acc)
        outs.append((_host(spins).copy(), _host(acc).copy()))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def _energy_series(mode, L, T, k, beta, n_rep, seed, sweeps, every=2, cap=0.0):
    b = S.Batch(S.HEISENBERG, 2, L, n_rep, seed, renorm_every=16)
    work, _ = _starts(L, n_rep, seed, mode)
    E = torch.zeros(n_rep, dtype=torch.float64, device=DEV)
    out = []
    t = 0
    while t < sweeps:
        S.heis_dcb_sweep(b, work, [beta] * n_rep, t, every, T, k, precision=mode, cap=cap)
        t += every
        # the energy of float64 spins is measured on their float32 rounding
        S.measure_energy_magnetisation(b, work if mode != S.HEIS_DOUBLE else work.float(), E)
        out.append(_host(E).copy() / (L * L))
    return np.array(out)  # [time, replica]


@pytest.mark.parametrize("mode", ["float", "fast", "double"])
def test_high_temperature_tree_energy(mode):
    """beta = 0.05: e = -2 L(beta) up to O(L^4), for every mode."""
    e = _energy_series(MODES[mode], 64, 16, 3, 0.05, 32, W.seed_for(85), 40)[5:]
    per_rep = e.mean(axis=0)
    m, err = per_rep.mean(), per_rep.std(ddof=1) / np.sqrt(len(per_rep))
    assert abs(m - X.heis_tree_energy(0.05, 2)) < 4.5 * err + 1e-5


@pytest.mark.parametrize("cap", [0.0, 0.3])
def test_modes_agree_with_the_oracle_at_low_temperature(cap):
    """beta = 1.5 on 32^2 with 16 x 16 tiles and 4 hits, uniform and
    small-step proposals: the long-run energy of every GPU mode within the
    combined errors of the oracle's."""
    L, T, k, beta, seed = 32, 16, 4, 1.5, W.seed_for(86)
    burn, sweeps = 50, 450
    ref = []
    for r in range(4):
        s = O.init_heis(2, L, seed, 100 + r)
        series = []
        for t in range(sweeps):
            O.heis_dcb_run(L, T, k, s, beta, seed, 100 + r, t, 1, cap=cap)
            if t >= burn and t % 2 == 0:
                series.append(O.heis_energy(2, L, s) / (L * L))
        ref.append(np.mean(series))
    ref_m, ref_err = np.mean(ref), np.std(ref, ddof=1) / np.sqrt(len(ref))
    for mode in MODES.values():
        e = _energy_series(mode, L, T, k, beta, 64, seed, sweeps, cap=cap)[burn // 2:]
        per_rep = e.mean(axis=0)
        m, err = per_rep.mean(), per_rep.std(ddof=1) / np.sqrt(len(per_rep))
        assert abs(m - ref_m) < 4.5 * np.hypot(err, ref_err), (mode, m, ref_m, err, ref_err)
