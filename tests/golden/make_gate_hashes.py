"""Writes gate_hashes.txt: digests of the oracle's states along the full-length
runs of three scope workloads, for the GPU bit-exactness gates of
tests/test_gpu_gates.py.  Calls the oracle only; nothing here touches the
HIP library.

  crop2d   independent 1024^2 Ising lattices with the 16384^2 workload's seed,
           one per beta in {0.30, beta_c, 0.50}, sweeps 0 .. 1999
  pt3d     64 chains (32 samples, both real replicas, all 32 temperatures) of
           the 3D +-J L=16 tempering batch, steps 0 .. 9999
  uneven2d 64 chains (one of every edge, 57 drawn at random) of the 4096-
           instance 2D +-J tempering batch, steps 0 .. 4999

Usage: python tests/golden/make_gate_hashes.py [--jobs N]   (about 40 minutes
on 8 cores; progress on stderr)."""
import argparse
import hashlib
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402

OUT = os.path.join(HERE, "gate_hashes.txt")

CROP_L = 1024
CROP_CHECKPOINTS = (500, 1000, 1500, 2000)
PT3D_CHECKPOINTS = (2500, 5000, 7500, 10000)
UNEVEN_CHECKPOINTS = (1000, 2000, 3000, 4000, 5000)


# digests: the first 128 bits of SHA-256, as 32 hex digits
def spins_digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, np.int8).tobytes()).hexdigest()[:32]


def state_digest(slot_of_temp, E, acc):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(slot_of_temp, "<i4").tobytes())
    h.update(np.ascontiguousarray(E, "<i8").tobytes())
    h.update(np.ascontiguousarray(acc, "<i8").tobytes())
    return h.hexdigest()[:32]


def pt3d_chains():
    """Chains 2s and 2s+1 of 32 samples spread over the 512 (both real replicas)."""
    samples = np.unique(np.linspace(0, 511, 32).round().astype(int))
    return [int(q) for s in samples for q in (2 * s, 2 * s + 1)]


def uneven_chains(sizes):
    """The first instance of every edge, then 57 more in a seeded random order."""
    picks = [int(np.nonzero(sizes == L)[0][0]) for L in sorted(set(int(v) for v in sizes))]
    rng = np.random.default_rng(5000)
    rest = [int(q) for q in rng.permutation(len(sizes)) if int(q) not in picks][:64 - len(picks)]
    return picks + rest


def crop_job(k):
    cfg = W.ising_large()
    beta = cfg.betas[k]
    s = O.init_spins(2, CROP_L, cfg.seed, 0)
    rows, done = [], 0
    for upto in CROP_CHECKPOINTS:
        O.run(2, CROP_L, None, s, beta, cfg.seed, 0, done, upto - done)
        done = upto
        rows.append(("crop2d", k, upto, spins_digest(s), "-", int(O.energy(2, CROP_L, None, s)), 0, 0))
    return rows


def chain_job(args):
    kind, dim, L, seed, q, n_temps, sample, betas, checkpoints = args
    r0 = q * n_temps
    chain = np.stack([O.init_spins(dim, L, seed, r0 + k) for k in range(n_temps)])
    J = O.init_couplings(dim, L, seed, sample)
    E = np.array([O.energy(dim, L, J, chain[k]) for k in range(n_temps)], np.int64)
    sq = np.arange(n_temps, dtype=np.int32)
    acc = np.zeros(n_temps, np.uint64)
    O.pt_audit(reset=True)
    rows, done = [], 0
    for upto in checkpoints:
        O.pt_run(dim, L, J, chain, np.asarray(betas, np.float64), sq, E, seed, q, r0, done, upto - done, acc)
        done = upto
        a = acc[:n_temps - 1].astype(np.int64)
        rows.append((kind, q, upto, spins_digest(chain), state_digest(sq, E, a), int(E.sum()), int(a.sum()),
                     O.pt_audit(reset=False)["near_ties"]))
    return rows


def run(job):
    return crop_job(job[1]) if job[0] == "crop2d" else chain_job(job[1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=len(os.sched_getaffinity(0)))
    a = ap.parse_args()
    c4 = W.ea3d_tempering()
    c5 = W.ea2d_uneven()
    rps = c4.chains_per_sample * c4.n_temps
    jobs = [("crop2d", k, CROP_L ** 2 * 2000) for k in range(3)]
    jobs += [("pt3d", ("pt3d", 3, c4.L, c4.seed, q, c4.n_temps, q * c4.n_temps // rps, list(c4.betas),
                       PT3D_CHECKPOINTS), c4.n_temps * c4.L ** 3 * c4.steps) for q in pt3d_chains()]
    jobs += [("uneven2d", ("uneven2d", 2, int(c5.sizes[q]), c5.seed, q, c5.n_temps, q, list(c5.betas),
                           UNEVEN_CHECKPOINTS), c5.n_temps * int(c5.sizes[q]) ** 2 * c5.steps)
             for q in uneven_chains(c5.sizes)]
    jobs.sort(key=lambda j: -j[2])          # longest first
    t0 = time.time()
    rows = []
    with mp.get_context("spawn").Pool(a.jobs) as pool:
        for i, r in enumerate(pool.imap_unordered(run, [(j[0], j[1]) for j in jobs])):
            rows += r
            print(f"[{time.time() - t0:7.0f} s] {i + 1}/{len(jobs)} {r[-1][0]} {r[-1][1]}", file=sys.stderr, flush=True)
    assert all(r[7] == 0 for r in rows), "an exchange decision within 2^-40 of exp(x): digests not comparable"
    order = {"crop2d": 0, "pt3d": 1, "uneven2d": 2}
    rows.sort(key=lambda r: (order[r[0]], r[1], r[2]))
    with open(OUT, "w") as f:
        f.write("# Oracle state digests along the full-length runs of three scope workloads (bit-exactness gates).\n")
        f.write("# Written by tests/golden/make_gate_hashes.py, which calls the oracle only.\n")
        f.write("# spins: SHA-256 of the int8 spins (the chain's replicas in storage order), first 128 bits;\n")
        f.write("# state: SHA-256 of slot_of_temp (int32 LE), energies (int64 LE), swap accepts (int64 LE), first 128 bits;\n")
        f.write("# E_total: sum of the energies; acc_total: sum of the swap accepts.\n")
        f.write("# kind key step spins state E_total acc_total\n")
        for r in rows:
            f.write(" ".join(str(v) for v in r[:7]) + "\n")
    print(f"wrote {OUT} ({len(rows)} rows, {time.time() - t0:.0f} s)", file=sys.stderr)


if __name__ == "__main__":
    main()
