"""Writes heis3d_L256_energy.txt: the float64 oracle's energy per site after
each of the 1000 sweeps of the 3D Heisenberg workload (256^3, beta = 0.693,
renormalisation every 16 sweeps, the workload's seed), for the long-run
comparison of tests/test_gpu_gates.py.  Calls the oracle only; one core,
about an hour.

Usage: python tests/golden/make_heis_series.py"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import oracle as O  # noqa: E402

OUT = os.path.join(HERE, "heis3d_L256_energy.txt")


def main():
    cfg = W.heisenberg_3d()
    L, beta = cfg.L, cfg.betas[0]
    N = L ** 3
    s = O.init_heis(3, L, cfg.seed, 0)
    rows = []
    t0 = time.time()
    for t in range(cfg.sweeps):
        O.heis_run(3, L, s, beta, cfg.seed, 0, t, 1, cfg.renorm_every)
        rows.append(O.heis_energy(3, L, s) / N)
        if (t + 1) % 50 == 0:
            print(f"[{time.time() - t0:7.0f} s] sweep {t + 1}: e = {rows[-1]:.9f}", file=sys.stderr, flush=True)
    with open(OUT, "w") as f:
        f.write("# Energy per site of the float64 oracle after each sweep of the 3D Heisenberg workload:\n")
        f.write(f"# L = {L}, beta = {beta}, renormalisation every {cfg.renorm_every} sweeps, seed {cfg.seed:#x},\n")
        f.write("# replica 0, sweeps 0 .. 999 from the workload's random start.\n")
        f.write("# Written by tests/golden/make_heis_series.py, which calls the oracle only.\n")
        f.write("# sweep e\n")
        for t, e in enumerate(rows):
            f.write(f"{t} {e!r}\n")
    print(f"wrote {OUT} ({time.time() - t0:.0f} s)", file=sys.stderr)


if __name__ == "__main__":
    main()
