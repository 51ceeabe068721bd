"""Seeded synthetic workloads (inputs only; no Monte Carlo arithmetic here).

Both the HIP library's tests/benchmark and the CPU oracle draw their inputs
from this module, so it holds parameters only: lattice sizes, inverse
temperatures, ladders, seeds and the size mix of the uneven batch.  The spins
and couplings themselves are produced by each side's own ``spin_init`` from
the seed (counter-based, keyed by site), never passed between them.

The workloads are the paper's own kind (no external data set exists): 2D/3D
Ising ferromagnet, 3D Heisenberg model, +-J Edwards-Anderson spin glass and
parallel-tempering ladders (Secs. 3-6).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MODEL_ISING, MODEL_EA, MODEL_HEIS = 0, 1, 2
BETA_C_2D = 0.5 * math.log(1.0 + math.sqrt(2.0))
SEED_BASE = 0x1101142700000000


def seed_for(index: int) -> int:
    return SEED_BASE + index


def geometric_ladder(t_min: float, t_max: float, n: int) -> np.ndarray:
    """Inverse temperatures of a geometric temperature ladder, coldest first."""
    k = np.arange(n, dtype=np.float64)
    T = t_min * (t_max / t_min) ** (k / (n - 1))
    return 1.0 / T


@dataclass
class Uniform:
    """A batch of n_rep replicas of one lattice size."""
    name: str
    model: int
    dim: int
    L: int
    n_rep: int
    betas: list
    sweeps: int
    seed: int
    rep_per_sample: int = 1
    renorm_every: int = 0


@dataclass
class Tempering:
    """Parallel tempering: n_chains chains of n_temps replicas each."""
    name: str
    model: int
    dim: int
    L: int  # 0 = uneven sizes in ``sizes``
    n_chains: int
    n_temps: int
    betas: np.ndarray
    steps: int
    seed: int
    chains_per_sample: int = 1
    sizes: np.ndarray = field(default=None)


def ising_small() -> Uniform:
    """64 x 64 square lattice at the exact critical coupling, 1000 sweeps."""
    return Uniform("ising2d_L64", MODEL_ISING, 2, 64, 1, [BETA_C_2D], 1000, seed_for(1))


def ising_large(L: int = 16384) -> Uniform:
    """16384^2 square lattice at beta in {0.30, beta_c, 0.50}, 2000 sweeps each."""
    return Uniform(f"ising2d_L{L}", MODEL_ISING, 2, L, 1, [0.30, BETA_C_2D, 0.50], 2000, seed_for(2))


def heisenberg_3d(L: int = 256) -> Uniform:
    """256^3 O(3) model at beta = 0.693, renormalised every 16 sweeps, 1000 sweeps."""
    return Uniform(f"heis3d_L{L}", MODEL_HEIS, 3, L, 1, [0.693], 1000, seed_for(3), renorm_every=16)


def ea3d_tempering(n_samples: int = 512, steps: int = 10_000) -> Tempering:
    """3D +-J spin glass L=16: samples x 2 real replicas x 32 temperatures in [0.8, 2.0]."""
    return Tempering("ea3d_L16_pt", MODEL_EA, 3, 16, n_chains=2 * n_samples, n_temps=32,
                     betas=geometric_ladder(0.8, 2.0, 32), steps=steps, seed=seed_for(4),
                     chains_per_sample=2)


UNEVEN_SIZES = (32, 48, 64, 96, 128, 192, 256)


def uneven_sizes(n_instances: int, seed: int) -> np.ndarray:
    """Edge lengths drawn uniformly from UNEVEN_SIZES with a seeded PCG64 stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.asarray(UNEVEN_SIZES, np.int32)[rng.integers(0, len(UNEVEN_SIZES), size=n_instances)]


def ea2d_uneven(n_instances: int = 4096, steps: int = 5000) -> Tempering:
    """Uneven batch of 2D +-J instances, 16 temperatures in [0.5, 2.0] each."""
    seed = seed_for(5)
    return Tempering("ea2d_uneven_pt", MODEL_EA, 2, 0, n_chains=n_instances, n_temps=16,
                     betas=geometric_ladder(0.5, 2.0, 16), steps=steps, seed=seed,
                     chains_per_sample=1, sizes=uneven_sizes(n_instances, seed))


def uneven_table(dim, sizes, reps_per_instance, model=MODEL_EA):
    """Rows (L, sample, spin_off, coup_off): instance k has reps_per_instance
    replicas sharing sample k; spins and couplings packed back to back."""
    rows = []
    so = co = 0
    for k, L in enumerate(sizes):
        N = int(L) ** dim
        for _ in range(reps_per_instance):
            rows.append((int(L), k, so, co))
            so += N
        co += dim * N if model == MODEL_EA else 0
    return np.array(rows, np.int64)
