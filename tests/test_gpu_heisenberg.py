"""Heisenberg model: float32 GPU sweeps against the float64 oracle.

The two sides use the same random numbers but round differently, so their
configurations part after a while; the checks are (i) the first sweep site by
site at the full 256^3 size, (ii) the long-run mean energy within three
combined standard errors.
"""
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


def _binned_mean_err(x, n_bins=20):
    """Mean and its standard error from n_bins consecutive bins (autocorrelation-safe)."""
    x = np.asarray(x, np.float64)
    m = len(x) // n_bins
    bins = x[:m * n_bins].reshape(n_bins, m).mean(axis=1)
    return bins.mean(), bins.std(ddof=1) / np.sqrt(n_bins)


# A float32 decision can differ from the float64 oracle's only where the
# uniform u lies within the float32 error of exp(-beta dE): spins and
# proposals carry ~2^-23 relative error, the field of six neighbours and the
# difference s' - s put at most ~2e-5 on dE, and beta = 0.693 scales that to
# below 2^-16 on the acceptance probability (the hardware exp2 adds ~1e-7).
NEAR_TIE = 2.0 ** -16


def _neighbours_of(mask, L):
    g = mask.reshape(L, L, L)
    out = np.zeros_like(g)
    for ax in range(3):
        out |= np.roll(g, 1, axis=ax) | np.roll(g, -1, axis=ax)
    return out.reshape(-1)


def test_heisenberg_256_first_sweep_sitewise():
    """256^3 at beta = 0.693 (the Heisenberg workload): one sweep from each
    side's own start; every component within 1e-5 except at sites whose
    decision differs, and each such site is either a near tie of the oracle's
    acceptance test (|u - exp(-beta dE)| < 2^-16) or a colour-1 neighbour of
    a colour-0 near tie (whose field the tie changed)."""
    cfg = W.heisenberg_3d()
    L, beta = cfg.L, cfg.betas[0]
    N = L ** 3
    b = S.Batch(S.HEISENBERG, 3, L, 1, cfg.seed, renorm_every=cfg.renorm_every)
    spins = torch.zeros(3 * N, dtype=torch.float32, device=DEV)
    S.spin_init(b, spins)
    n_acc = torch.zeros(1, dtype=torch.int64, device=DEV)
    S.metropolis_sweep(b, spins, [beta], 0, 1, dE_accum=n_acc)
    ref = O.init_heis(3, L, cfg.seed, 0)
    ref_acc, gap = O.heis_sweep_gaps(3, L, ref, beta, cfg.seed, 0, 0, cfg.renorm_every)
    got = _host(spins).astype(np.float64).reshape(-1, 3)
    dev = np.abs(got - ref).max(axis=1)
    mis = dev > 1e-5
    idx = np.arange(N)
    colour = ((idx % L) + (idx // L) % L + idx // (L * L)) & 1
    primary = mis & (np.abs(gap) < NEAR_TIE)
    secondary = mis & (colour == 1) & _neighbours_of(primary & (colour == 0), L)
    unexplained = int((mis & ~primary & ~secondary).sum())
    print(f"256^3 first sweep: {int(mis.sum())} differing sites ({int(primary.sum())} near ties, "
          f"{int((secondary & ~primary).sum())} neighbours of one); sites within 2^-16 of a tie: "
          f"{int((np.abs(gap) < NEAR_TIE).sum())}")
    assert unexplained == 0
    # at most max(4, 16 N 2^-24) = 16 differing sites at 256^3 (1 observed)
    assert mis.sum() <= max(4, int(16 * N * 2.0 ** -24)), int(mis.sum())
    assert abs(int(_host(n_acc)[0]) - ref_acc) <= int(mis.sum())
    assert np.abs(np.linalg.norm(got, axis=1) - 1).max() < 2e-6


def test_heisenberg_long_run_energy_within_three_sigma():
    """16^3 at beta = 0.693, 500 sweeps burn-in then 3000 sweeps measured every
    10: the float32 GPU chain and the float64 oracle chain agree on <e> within
    three combined standard errors."""
    L, beta, seed = 16, 0.693, W.seed_for(30)
    N = L ** 3
    b = S.Batch(S.HEISENBERG, 3, L, 1, seed, renorm_every=16)
    spins = torch.zeros(3 * N, dtype=torch.float32, device=DEV)
    S.spin_init(b, spins)
    ref = O.init_heis(3, L, seed, 0)
    E = torch.zeros(1, dtype=torch.float64, device=DEV)
    burn, total, every = 500, 3500, 10
    S.metropolis_sweep(b, spins, [beta], 0, burn)
    O.heis_run(3, L, ref, beta, seed, 0, 0, burn, 16)
    e_gpu, e_ref = [], []
    for t in range(burn, total, every):
        S.metropolis_sweep(b, spins, [beta], t, every)
        S.measure_energy_magnetisation(b, spins, E)
        e_gpu.append(float(_host(E)[0]) / N)
        O.heis_run(3, L, ref, beta, seed, 0, t, every, 16)
        e_ref.append(O.heis_energy(3, L, ref) / N)
    mg, sg = _binned_mean_err(e_gpu)
    mr, sr = _binned_mean_err(e_ref)
    assert abs(mg - mr) <= 3.0 * np.hypot(sg, sr), (mg, sg, mr, sr)
    # beta = 0.693 is close to the 3D critical point: about one third of the
    # maximal bond energy, e in (-1.5, -0.5)
    assert -1.5 < mg < -0.5 and -1.5 < mr < -0.5


@pytest.mark.parametrize("L,n_rep,n", [(16, 3, 20), (32, 2, 19), (64, 1, 20), (128, 1, 5)])
def test_gpu_heisenberg_kernels_agree(monkeypatch, L, n_rep, n):
    """The one-pass tiled kernel (edge >= 32), the two-launch indexed kernel
    and the generic kernel perform the same float32 arithmetic in the same
    order: identical spins and acceptance counts after n sweeps (one
    renormalisation included; an odd count ends in the scratch buffer and is
    copied back)."""
    seed = W.seed_for(31)
    b = S.Batch(S.HEISENBERG, 3, L, n_rep, seed, renorm_every=16)
    assert S.sweep_plan(b)[1] == ("k_heis3d_tiled" if L >= 32 else "k_heis3d_half")
    out = []
    for tiled, indexed, remap in (("1", "1", "1"), ("1", "1", "0"), ("0", "1", "1"), ("0", "0", "1")):
        monkeypatch.setenv("SPINMC_XCD_REMAP", remap)
        monkeypatch.setenv("SPINMC_HEIS_TILED", tiled)
        monkeypatch.setenv("SPINMC_HEIS3D", indexed)
        spins = torch.zeros(3 * n_rep * L ** 3, dtype=torch.float32, device=DEV)
        S.spin_init(b, spins)
        acc = torch.zeros(n_rep, dtype=torch.int64, device=DEV)
        S.metropolis_sweep(b, spins, [0.693, 0.5, 1.2][:n_rep], 3, n, dE_accum=acc)
        out.append((_host(spins).copy(), _host(acc).copy()))
    for o in out[1:]:
        assert np.array_equal(out[0][0], o[0])
        assert np.array_equal(out[0][1], o[1])


def test_gpu_heisenberg_kernels_agree_at_the_largest_edge(monkeypatch):
    """At the largest edge the one-pass kernel supports (1024^3, 2^30 sites,
    32-bit site indices up to 2^30 - 1) it gives the same spins and
    acceptance counts as the two-launch kernel after two sweeps (compared on
    the device: 12.9 GB per copy)."""
    L, n = 1024, 2
    b = S.Batch(S.HEISENBERG, 3, L, 1, W.seed_for(33), renorm_every=16)
    assert S.sweep_plan(b)[1] == "k_heis3d_tiled"
    out = []
    for tiled in ("1", "0"):
        monkeypatch.setenv("SPINMC_HEIS_TILED", tiled)
        spins = torch.zeros(3 * L ** 3, dtype=torch.float32, device=DEV)
        S.spin_init(b, spins)
        acc = torch.zeros(1, dtype=torch.int64, device=DEV)
        S.metropolis_sweep(b, spins, [0.693], 14, n, dE_accum=acc)  # sweep 15 renormalises
        torch.cuda.synchronize()
        out.append((spins, int(acc.cpu()[0])))
    assert out[0][1] == out[1][1] and out[0][1] > 0
    assert torch.equal(out[0][0], out[1][0])
    # unit vectors after the renormalisation of sweep 15
    norms = out[0][0].view(-1, 3).norm(dim=1)
    assert float((norms - 1.0).abs().max()) < 1e-6
    del out
    torch.cuda.empty_cache()
