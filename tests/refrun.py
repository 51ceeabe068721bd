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


def pt_chain(job):
    """One tempering chain of a batch run by the oracle (module-level so that a
    process pool can call it).  job: dict with dim, L, model, seed, q (chain
    index), n_temps, sample, beta, perm, t0, steps and m.  Returns (spins
    [n_temps][N], slot_of_temp, E, swap counts [n_temps-1], near-tie audit)."""
    dim, L, n_temps, q = job["dim"], job["L"], job["n_temps"], job["q"]
    r0 = q * n_temps
    chain = np.stack([O.init_spins(dim, L, job["seed"], r0 + k) for k in range(n_temps)])
    J = O.init_couplings(dim, L, job["seed"], job["sample"]) if job["model"] == EA else None
    E = np.array([O.energy(dim, L, J, chain[k]) for k in range(n_temps)], np.int64)
    sq = np.asarray(job["perm"], np.int32).copy()
    aq = np.zeros(n_temps, np.uint64)
    O.pt_audit(reset=True)
    O.pt_run(dim, L, J, chain, np.asarray(job["beta"], np.float64), sq, E, job["seed"], q, r0, job["t0"],
             job["steps"], aq, sweeps_per_step=job.get("m", 1))
    return chain, sq, E, aq[:n_temps - 1], O.pt_audit(reset=True)


def run_parallel(fn, jobs):
    """fn over jobs in fresh worker processes (spawned, so that they never
    inherit a GPU context), at most 16 at a time; results in job order."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import os

    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    n = max(1, min(16, n, len(jobs)))
    with cf.ProcessPoolExecutor(max_workers=n, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(fn, jobs))


def sweeps_parallel(job):
    """n sweeps of one 2D/3D replica by the oracle (for a process pool): job has
    dim, L, seed, r, beta, t0, n and checkpoints (sweep counts after which the
    spins are recorded).  Returns the list of recorded spin arrays."""
    s = O.init_spins(job["dim"], job["L"], job["seed"], job["r"])
    out, done = [], 0
    for upto in job["checkpoints"]:
        O.run(job["dim"], job["L"], None, s, job["beta"], job["seed"], job["r"], job["t0"] + done, upto - done)
        done = upto
        out.append(s.copy())
    return out
