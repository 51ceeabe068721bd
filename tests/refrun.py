"""Oracle runs of whole batches, in the layouts of the C ABI (tests only)."""
import numpy as np

from oracle import oracle as O
from workloads import uneven_table  # noqa: F401  (re-exported for the tests)

ISING, EA, HEIS = 0, 1, 2


def init_uniform(model, dim, L, n_rep, seed, rep_per_sample=1):
    """(spins [n_rep][N] int8 or [n_rep][N][3] f64, couplings [n_samples][d][N] or None)."""
    if model == HEIS:
        return np.stack([O.init_heis(dim, L, seed, r) for r in range(n_rep)]), None
    spins = np.stack([O.init_spins(dim, L, seed, r) for r in range(n_rep)])
    coup = None
    if model == EA:
        n_s = -(-n_rep // rep_per_sample)
        coup = np.stack([O.init_couplings(dim, L, seed, q) for q in range(n_s)])
    return spins, coup


def sweep_uniform(model, dim, L, spins, coup, betas, seed, t0, n, rep_per_sample=1):
    """n sweeps of every replica in place; returns the per-replica dE sums."""
    dE = np.zeros(len(spins), np.int64)
    for r in range(len(spins)):
        J = None if coup is None else coup[r // rep_per_sample]
        dE[r] = O.run(dim, L, J, spins[r], float(betas[r]), seed, r, t0, n)
    return dE


def init_uneven(model, dim, inst, seed):
    """Flat spin / coupling buffers for an uneven table (rows L, sample, spin_off, coup_off)."""
    n_sp = max(int(r[2]) + int(r[0]) ** dim for r in inst)
    spins = np.zeros(n_sp, np.int8)
    coup = None
    if model == EA:
        n_c = max(int(r[3]) + dim * int(r[0]) ** dim for r in inst)
        coup = np.zeros(n_c, np.int8)
    for rep, row in enumerate(inst):
        L, q, so, co = (int(v) for v in row)
        N = L ** dim
        spins[so:so + N] = O.init_spins(dim, L, seed, rep)
        if coup is not None:
            coup[co:co + dim * N] = O.init_couplings(dim, L, seed, q)
    return spins, coup


def sweep_msc(model, dim, L, spins, coup, betas, seed, t0, n, w=32):
    """Multi-spin-coded sweeps (groups of w replicas share their draws): each
    replica is the ordinary chain with the group index r // w in the counters."""
    dE = np.zeros(len(spins), np.int64)
    for r in range(len(spins)):
        J = None if coup is None else coup[r]
        dE[r] = O.run(dim, L, J, spins[r], float(betas[r]), seed, r // w, t0, n)
    return dE
