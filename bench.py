"""Benchmark: checkerboard Metropolis on the 16384^2 2D Ising lattice.

A step is one full sweep (colour 0 then colour 1, with Delta E tracking) of
the 16384 x 16384 periodic Ising lattice; the K timed steps are split evenly
over the three inverse temperatures beta in {0.30, beta_c, 0.50}, each on its
own lattice from the seeded random start.  Spins are resident in HBM before
the timed region.  Prints one JSON line: ns per spin flip (lower is better),
the HBM roofline of the sweep kernel and the CPU oracle timed on a bounded
sample (1024^2 lattice) of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_FLIP = 2.0  # int8 spin read once and written once per sweep


def cpu_baseline(cfg, seconds: float = 12.0):
    """The oracle (serial C, 1 thread) on a 1024^2 lattice of the same workload."""
    from oracle import oracle as O

    L = 1024
    N = L * L
    flips, elapsed = 0, 0.0
    per_beta = []
    for beta in cfg.betas:
        s = O.init_spins(2, L, cfg.seed, 0)
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < seconds / len(cfg.betas):
            O.run(2, L, None, s, beta, cfg.seed, 0, n, 1)
            n += 1
        dt = time.perf_counter() - t0
        per_beta.append(n)
        flips += n * N
        elapsed += dt
    return {"value": elapsed / flips * 1e9, "unit": "ns/flip", "cores": 1, "kind": "oracle",
            "sample": f"1024^2 Ising lattice, {'/'.join(map(str, per_beta))} sweeps at beta="
                      f"{'/'.join(f'{b:.4f}' for b in cfg.betas)}, serial C oracle"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--L", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1101_1427_amd as S
    import workloads as W

    cfg = W.ising_large(args.L)
    L = cfg.L
    N = L * L
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    b = S.Batch(S.ISING, 2, L, 1, cfg.seed)
    lattices = []
    for beta in cfg.betas:
        s = torch.empty(N, dtype=torch.int8, device=dev)
        S.spin_init(b, s)
        lattices.append((beta, s, torch.zeros(1, dtype=torch.int64, device=dev)))
    nb = len(lattices)
    steps = max(nb, args.steps - args.steps % nb)
    per = steps // nb
    warm = max(1, args.warmup // nb)
    for beta, s, dE in lattices:
        S.metropolis_sweep(b, s, [beta], 0, warm, dE_accum=dE)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_wall = time.perf_counter()
    ev0.record(stream)
    for beta, s, dE in lattices:
        S.metropolis_sweep(b, s, [beta], warm, per, dE_accum=dE)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / steps
    ns_per_flip = gpu_ms * 1e6 / (steps * N)

    launches_per_sweep = int(os.environ.get("SPINMC_LAUNCHES_PER_SWEEP", S.launches_per_sweep(b)))
    launch_ms = ms_per_step / launches_per_sweep
    bytes_per_launch = BYTES_PER_FLIP * N / launches_per_sweep
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9

    out = {
        "metric": "ns per spin flip (+% HBM roofline); batched PT sweeps/s vs per-instance",
        "value": round(ns_per_flip, 6),
        "unit": "ns/flip",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm * nb,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": f"2D Ising {L}x{L} periodic, int8 spins, random start, beta in "
                               f"{{0.30, ln(1+sqrt2)/2, 0.50}}, {per} sweeps each, Delta E tracked",
                   "L": L, "betas": cfg.betas, "sweeps_per_beta": per, "seed": cfg.seed},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": S.sweep_kernel_name(b), "launches_per_sweep": launches_per_sweep,
                     "algorithmic_bytes_per_launch": bytes_per_launch},
        "wall_s": round(wall, 4),
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(cfg)
        out["cpu_baseline"] = cb
    print(json.dumps(out))


if __name__ == "__main__":
    main()
