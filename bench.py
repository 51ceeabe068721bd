"""Benchmark: checkerboard Metropolis on 16384^2 2D Ising lattices, plus the
tempering and Heisenberg workloads.

The headline workload is three 16384 x 16384 periodic Ising lattices, one at
each inverse temperature beta in {0.30, beta_c, 0.50}, from seeded random
starts, swept as one batch of three replicas: a step is one sweep (colour 0
then colour 1, with Delta E tracking) of all three, one kernel launch.
Spins are resident in HBM before the timed region.  Prints one JSON line:
ns per spin flip (lower is better), the HBM roofline of the sweep kernel
(and the same kernel on one lattice alone), the 3D Heisenberg workload,
the batched tempering workloads against per-instance launches and the
paper's 20-replica tempering workload, multi-spin coding, the double
checkerboard against k and L, the paper's 2D Heisenberg workload in three
arithmetic modes, and the CPU oracle timed on a bounded sample (1024^2
lattice) of the workload.  Separate modes (--tau-only, --table1-only, ...)
run the autocorrelation study and Table 1 with the Philox streams.
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


PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = {
    "k_ising2d_split": ("lattice2d.hip", "lattice2d.hpp", "intrin.hpp", "philox.hpp", "tables.hpp"),
    "k_heis3d_tiled": ("heis3d.hip", "heis_math.hpp", "philox.hpp"),
    "k_ising3d_half": ("sweep3d.hip", "segment3d.hpp", "intrin.hpp", "philox.hpp", "tables.hpp"),
    "k_ising3d_pass": ("pass3d.hip", "segment3d.hpp", "intrin.hpp", "philox.hpp", "tables.hpp"),
    "k_pt3d_chain": ("pt3d.hip", "intrin.hpp", "philox.hpp", "tables.hpp"),
    "k_uneven2d_sweep": ("batched2d.hip", "intrin.hpp", "philox.hpp", "tables.hpp"),
}


def kernel_source_hash(kernel: str = "k_ising2d_split") -> str:
    """sha256 over the sources a sweep kernel is compiled from."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_1101_1427_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def traffic_file(kernel: str, L: int) -> str:
    return os.path.join(PROFILES, f"{kernel}_L{L}_traffic.txt")


def traffic_per_launch(kernel: str, L: int):
    """HBM bytes per launch of the sweep kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size);
    None if there is none or the kernel sources changed since it was taken."""
    path = traffic_file(kernel, L)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash(kernel):
        return None
    return float(kv["traffic_bytes_per_launch"])


def copy_calibration(nbytes: int = 1 << 30, reps: int = 4):
    """A plain device-to-device copy of nbytes, reps times (for the counter scale)."""
    import torch

    src = torch.ones(nbytes, dtype=torch.int8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}))


KT_WORKLOADS = {
    "k_ising2d_split": "2D Ising {L}x{L}, the headline batch of three lattices",
    "k_heis3d_tiled": "3D Heisenberg {L}^3, one lattice",
    "k_ising3d_pass": "3D Ising and EA (one +-J sample), one L^3 lattice per model, L up to {L}",
    "k_ising3d_half": "3D Ising and EA (one +-J sample), one L^3 lattice per model, L up to {L}",
    "k_pt3d_chain": "3D +-J tempering, L = {L}: 512 samples x 2 replicas x 32 temperatures, chain-resident",
    "k_uneven2d_sweep": "uneven 2D +-J tempering batch: 4096 instances x 16 temperatures, edges 32 .. {L}",
}


def kt_summary(db: str, log: str, kernel: str, L: int, command: str):
    """Per-kernel totals of a rocprofv3 --kernel-trace --stats run, beside the
    bench line the same run printed; written next to the traffic summary."""
    import sqlite3

    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    bench_line = ""
    with open(log) as fh:
        for line in fh:
            if line.startswith("{") and '"metric"' in line:
                bench_line = line.strip()
    lines = [f"# rocprofv3 --kernel-trace --stats summary: {kernel}, {KT_WORKLOADS[kernel].format(L=L)}",
             f"# command: {command}",
             "# durations in microseconds (top_kernels view of the results database)",
             f"kernel_source_sha256: {kernel_source_hash(kernel)}",
             f"{'kernel':40s} {'calls':>7s} {'total_us':>12s} {'avg_us':>10s} {'pct':>7s}"]
    for name, calls, total, avg, pct in rows:
        lines.append(f"{short_name(name):40s} {calls:7d} {total:12.1f} {avg:10.3f} {pct:7.2f}")
    # the same run times the batched launch and then single-lattice launches:
    # the kernel's dispatches per grid size, from the kernels view
    lines.append(f"# {kernel} per grid size (work-items): dispatches, mean duration in microseconds")
    for grid, calls, avg in con.execute("select grid_x, count(*), avg(duration) / 1000.0 from kernels "
                                        "where name like ? group by grid_x order by grid_x desc",
                                        (f"%{kernel}%",)):
        lines.append(f"grid_{grid}: {calls} {avg:.3f}")
    lines.append(f"# {kernel} per instantiation and grid size: dispatches, mean duration in microseconds")
    for name, grid, calls, avg in con.execute("select name, grid_x, count(*), avg(duration) / 1000.0 from kernels "
                                              "where name like ? group by name, grid_x order by grid_x desc, name",
                                              (f"%{kernel}%",)):
        import re

        inst = re.search(r"<[^>]*>", name)
        lines.append(f"{kernel}{inst.group(0) if inst else ''} grid_{grid}: {calls} {avg:.3f}")
    if bench_line:
        import json

        d = json.loads(bench_line)
        if kernel in ("k_pt3d_chain", "k_uneven2d_sweep"):
            t = d.get("tempering", {}).get("ea3d_L16" if kernel == "k_pt3d_chain" else "ea2d_uneven", {})
            for key in ("steps", "ms", "replica_sweeps_per_s", "speedup_vs_per_instance"):
                if key in t:
                    lines.append(f"bench_line_{key}: {t[key]}")
        else:
            r = d["roofline"]
            lines.append(f"bench_line_kernel_us_per_launch: {r['kernel_us_per_launch']}")
            lines.append(f"bench_line_roofline_frac: {r['frac']}")
            lines.append(f"bench_line_ns_per_flip: {d['value']}")
    os.makedirs(PROFILES, exist_ok=True)
    path = os.path.join(PROFILES, f"{kernel}_L{L}_kernel_trace.txt")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def valu_summary(db: str, command: str):
    """VALU use of the hot kernels from a rocprofv3 --pmc run with
    SQ_INSTS_VALU, SQ_ACTIVE_INST_VALU, SQ_ACTIVE_INST_VALU2,
    SQ_BUSY_CU_CYCLES and GRBM_GUI_ACTIVE, per dispatch of each kernel's
    largest grid, against C = CU_NUM x GRBM_GUI_ACTIVE (CU-cycles of the
    dispatch; GRBM_GUI_ACTIVE is summed over the 8 XCDs in the database and
    taken as that sum / 8):
      issue = SQ_INSTS_VALU / C: wave64 VALU instructions per CU per cycle;
              1.0 when each of the four SIMDs issues one per quad-cycle;
              gfx950 can issue two per quad-cycle, so this can exceed 1;
      dual  = SQ_ACTIVE_INST_VALU2 / SQ_ACTIVE_INST_VALU: the share of VALU
              instructions issued in a quad-cycle that issued two;
      busy  = (SQ_ACTIVE_INST_VALU - SQ_ACTIVE_INST_VALU2) / C: the share of
              SIMD quad-cycles that issued at least one VALU instruction
              (SQ_ACTIVE_INST_VALU counts one quad-cycle per instruction, so
              dual-issued quad-cycles are counted twice; the profiler's
              VALUBusy is SQ_ACTIVE_INST_VALU / C);
      cu    = SQ_BUSY_CU_CYCLES / C: the share of CU-cycles with work."""
    import sqlite3

    cu_num = 256
    con = sqlite3.connect(db)
    rows = con.execute("select kernel_name, counter_name, value, grid_size from counters_collection").fetchall()
    # per kernel: its largest grid, and of that grid the instantiation with
    # the most dispatches (the 2D sweep: the split-to-split launches)
    count = {}
    for name, cname, _, grid in rows:
        if cname == "SQ_INSTS_VALU":
            count[(short_name(name), grid, name)] = count.get((short_name(name), grid, name), 0) + 1
    pick = {}
    for (k, grid, name), n in count.items():
        if k not in pick or (grid, n) > (pick[k][0], pick[k][1]):
            pick[k] = (grid, n, name)
    acc = {}
    for name, cname, val, grid in rows:
        k = short_name(name)
        if k in pick and (grid, name) == (pick[k][0], pick[k][2]):
            acc.setdefault(k, {}).setdefault(cname, []).append(val)
    lines = ["# VALU use per dispatch of each kernel's largest grid, most frequent instantiation (rocprofv3 --pmc)",
             f"# command: {command}",
             "# C = CU_NUM (256) x GRBM_GUI_ACTIVE (8-XCD sum / 8): CU-cycles of the dispatch",
             "# issue = SQ_INSTS_VALU / C: wave64 VALU instructions per CU per cycle (1.0 = one per SIMD per",
             "#         quad-cycle; gfx950 dual-issues, so up to 2)",
             "# dual  = SQ_ACTIVE_INST_VALU2 / SQ_ACTIVE_INST_VALU (share of instructions issued two at a time)",
             "# busy  = (SQ_ACTIVE_INST_VALU - SQ_ACTIVE_INST_VALU2) / C: SIMD quad-cycles issuing >= 1 VALU op",
             "# cu    = SQ_BUSY_CU_CYCLES / C",
             f"{'kernel':24s} {'disp':>5s} {'VALU_insts':>11s} {'gui_cycles':>11s} {'issue':>6s} {'dual':>6s} "
             f"{'busy':>6s} {'cu':>6s}"]
    names = ("k_ising2d_split", "k_pt3d_chain", "k_uneven2d_sweep", "k_heis3d_tiled", "k_heis3d_half",
             "k_ising3d_half", "k_ising3d_pass", "k_half_sweep_generic", "k_msc2d", "k_dcb2d_packed", "k_dcb2d",
             "k_dcb3d", "k_heis_dcb2d", "k_philox_bench", "k_dcb_rng")
    for k in names:
        a = acc.get(k, {})
        if "SQ_INSTS_VALU" not in a or "GRBM_GUI_ACTIVE" not in a:
            continue
        mean = lambda key: sum(a[key]) / len(a[key]) if key in a else float("nan")
        vi, gui = mean("SQ_INSTS_VALU"), mean("GRBM_GUI_ACTIVE") / 8.0
        act, act2, cub = mean("SQ_ACTIVE_INST_VALU"), mean("SQ_ACTIVE_INST_VALU2"), mean("SQ_BUSY_CU_CYCLES")
        C = cu_num * gui
        lines.append(f"{k:24s} {len(a['SQ_INSTS_VALU']):5d} {vi:11.4g} {gui:11.4g} {vi / C:6.3f} "
                     f"{(act2 / act if act > 0 else float('nan')):6.3f} {(act - act2) / C:6.3f} {cub / C:6.3f}")
    os.makedirs(PROFILES, exist_ok=True)
    with open(os.path.join(PROFILES, "valu_utilisation.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def short_name(name: str) -> str:
    import re

    m = re.search(r"(k_\w+|__amd_\w+|\w*[Cc]opy\w*)", name)
    return m.group(1) if m else name[:60]


def pmc_summary(fetch_db: str, write_db: str, cfetch_db: str, cwrite_db: str, kernel: str, L: int,
                commands: list[str], grid_rule: str = "most"):
    """kernel k_ising2d_split: one launch sweeps the bench's batch of three
    L x L lattices; k_heis3d_tiled: one launch sweeps one L^3 lattice."""
    """Mean FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the sweep kernel and
    of the copy kernel, from rocprofv3 result databases; writes the summary
    that traffic_per_launch reads."""
    import sqlite3

    def per_kernel(db, counter, main_grid=False):
        con = sqlite3.connect(db)
        rows = con.execute("select kernel_name, value, grid_size from counters_collection where counter_name=?",
                           (counter,)).fetchall()
        # per kernel instantiation, its grid with the most dispatches (the
        # timed batch's launches, not the single-lattice launches the same
        # run makes afterwards nor the launch shapes the autotuner tries), or
        # with grid_rule "largest" its largest grid (the largest lattice of a
        # run that sweeps several)
        count = {}
        for name, _, grid in rows:
            count[(name, grid)] = count.get((name, grid), 0) + 1
        main = {}
        for (name, grid), n in count.items():
            if grid_rule == "largest":
                if name not in main or grid > main[name]:
                    main[name] = grid
            elif name not in main or n > count[(name, main[name])]:
                main[name] = grid
        acc = {}
        for name, val, grid in rows:
            if not main_grid or grid == main[name]:
                acc.setdefault(name, []).append(val)
        per_kernel.grids = main
        return acc

    def mean_of(acc, key):
        # the variant of the kernel with the most dispatches: for the 2D sweep
        # the split-to-split launches, not the first and last sweeps of a call
        # (which read and write the caller's rows)
        name = max((n for n in acc if key in n), key=lambda n: (len(acc[n]), sum(acc[n]) / len(acc[n])))
        return name, sum(acc[name]) / len(acc[name])

    kf, kfv = mean_of(per_kernel(fetch_db, "FETCH_SIZE", True), kernel)
    fetch_grid = per_kernel.grids[kf]
    kw, kwv = mean_of(per_kernel(write_db, "WRITE_SIZE", True), kernel)
    write_grid = per_kernel.grids[kw]
    # the copy kernel: the one that fetched the most; its sums over the run
    # divided by the number of 1 GiB copies
    cf_all, cw_all = per_kernel(cfetch_db, "FETCH_SIZE"), per_kernel(cwrite_db, "WRITE_SIZE")
    copy_name = max(cf_all, key=lambda n: sum(cf_all[n]))
    reps = 4
    cfv, cwv = sum(cf_all[copy_name]) / reps, sum(cw_all[copy_name]) / reps
    copy_kib = (1 << 30) / 1024.0
    fetch_scale = copy_kib / cfv
    write_scale = copy_kib / cwv
    traffic = (kfv * fetch_scale + kwv * write_scale) * 1024.0
    if kernel == "k_heis3d_tiled":
        algorithmic = 24.0 * L ** 3
        what = f"one launch = one sweep of a 3D Heisenberg {L}^3 lattice (24 B per site)"
    elif kernel == "k_ising3d_pass":
        algorithmic = BYTES_PER_FLIP * L ** 3
        what = (f"one launch = one sweep of a 3D Ising {L}^3 lattice; algorithmic bytes = one read and one write "
                f"of every spin (2 B per site)")
    elif kernel == "k_ising3d_half":
        algorithmic = 1.0 * L ** 3
        what = (f"one launch = one half-sweep of a 3D Ising {L}^3 lattice; algorithmic bytes = half of the "
                f"sweep's one read and one write of every spin (1 B per site per launch)")
    else:
        algorithmic = BYTES_PER_FLIP * L * L * 3
        what = f"one launch = one sweep of a batch of three 2D Ising {L}x{L} lattices"
    lines = [f"# rocprofv3 --pmc summary: {kernel}, {what}",
             "# figures are means per dispatch of the counter over the dispatches of the kernel's instantiation and "
             + ("grid with the most dispatches in the run (the timed batch)" if grid_rule == "most" else
                "largest grid in the run (the largest lattice)")]
    lines += [f"# command: {c}" for c in commands]
    lines += [f"kernel_source_sha256: {kernel_source_hash(kernel)}",
              f"kernel_dispatches: {short_name(kf)} grid {fetch_grid} (FETCH_SIZE run), grid {write_grid} "
              f"(WRITE_SIZE run)",
              f"kernel_FETCH_SIZE_KiB_per_dispatch: {kfv:.1f}",
              f"kernel_WRITE_SIZE_KiB_per_dispatch: {kwv:.1f}",
              f"copy_kernel: {short_name(copy_name)}",
              "copy_bytes_read_and_written_per_copy: 1073741824",
              f"copy_FETCH_SIZE_KiB_per_copy: {cfv:.1f}",
              f"copy_WRITE_SIZE_KiB_per_copy: {cwv:.1f}",
              f"fetch_scale: {fetch_scale:.4f}",
              f"write_scale: {write_scale:.4f}",
              f"fetch_bytes_per_launch: {kfv * fetch_scale * 1024:.0f}",
              f"write_bytes_per_launch: {kwv * write_scale * 1024:.0f}",
              f"traffic_bytes_per_launch: {traffic:.0f}",
              f"algorithmic_bytes_per_launch: {algorithmic:.0f}",
              f"traffic_over_algorithmic: {traffic / algorithmic:.4f}"]
    os.makedirs(PROFILES, exist_ok=True)
    with open(traffic_file(kernel, L), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _host_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))  # the share of host cores that goes with one GPU


def oracle_job(kind: str, seconds: float, index: int = 0) -> dict:
    """One timed run of the serial oracle (1 thread) on a bounded sample of a
    workload: repeats its unit of work until `seconds` have passed.
      c2: the 1024^2 Ising crop of the 16384^2 workload, the three betas in turn;
      c3: the FP64 Heisenberg oracle on 32^3 at beta = 0.693 (renormalised every 16);
      c4: one chain of the 3D EA tempering workload (32 temperatures, 16^3);
      c5: one instance of the uneven 2D EA tempering workload (16 temperatures),
          instance `index` of the batch.
    Returns attempted flips, elapsed seconds and what the sample was."""
    import numpy as np

    from oracle import oracle as O
    import workloads as W

    flips = 0
    units = 0
    if kind == "c2":
        cfg = W.ising_large()
        L = 1024
        spins = [O.init_spins(2, L, cfg.seed, 0) for _ in cfg.betas]
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            k = units % len(cfg.betas)
            O.run(2, L, None, spins[k], cfg.betas[k], cfg.seed, 0, units // len(cfg.betas), 1)
            units += 1
            flips += L * L
        what = f"1024^2 Ising crop, {units} sweeps cycling beta over {cfg.betas}"
    elif kind == "c3":
        cfg = W.heisenberg_3d()
        L = 32
        s = O.init_heis(3, L, cfg.seed, 0)
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            O.heis_run(3, L, s, cfg.betas[0], cfg.seed, 0, units, 1, cfg.renorm_every)
            units += 1
            flips += L ** 3
        what = f"3D Heisenberg 32^3 at beta = {cfg.betas[0]}, FP64, {units} sweeps"
    elif kind == "c4":
        cfg = W.ea3d_tempering()
        L, nt = cfg.L, cfg.n_temps
        q = index % cfg.n_chains
        J = O.init_couplings(3, L, cfg.seed, q // cfg.chains_per_sample)
        spins = np.stack([O.init_spins(3, L, cfg.seed, q * nt + k) for k in range(nt)])
        E = np.array([O.energy(3, L, J, spins[k]) for k in range(nt)], np.int64)
        sot = np.arange(nt, dtype=np.int32)
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            O.pt_run(3, L, J, spins, cfg.betas, sot, E, cfg.seed, q, q * nt, units, 1)
            units += 1
            flips += nt * L ** 3
        what = f"3D EA tempering chain {q} (32 temperatures x 16^3), {units} steps"
    elif kind == "c5":
        cfg = W.ea2d_uneven()
        nt = cfg.n_temps
        q = index % cfg.n_chains
        L = int(cfg.sizes[q])
        J = O.init_couplings(2, L, cfg.seed, q)
        spins = np.stack([O.init_spins(2, L, cfg.seed, q * nt + k) for k in range(nt)])
        E = np.array([O.energy(2, L, J, spins[k]) for k in range(nt)], np.int64)
        sot = np.arange(nt, dtype=np.int32)
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds:
            O.pt_run(2, L, J, spins, cfg.betas, sot, E, cfg.seed, q, q * nt, units, 1)
            units += 1
            flips += nt * L * L
        what = f"uneven 2D EA instance {q} (L = {L}, 16 temperatures), {units} steps"
    else:
        raise ValueError(kind)
    return {"flips": flips, "seconds": time.perf_counter() - t0, "units": units, "sample": what}


def _oracle_children(kind: str, seconds: float, n: int) -> list:
    """n oracle jobs of one kind at once, one child process each (fresh
    interpreters that never touch the GPU)."""
    import subprocess

    procs = [subprocess.Popen([sys.executable, os.path.abspath(__file__), "--oracle-job", kind, str(seconds), str(i)],
                              stdout=subprocess.PIPE, text=True) for i in range(n)]
    out = []
    for p in procs:
        stdout, _ = p.communicate()
        if p.returncode != 0:
            raise RuntimeError(f"oracle job {kind} failed with status {p.returncode}")
        out.append(json.loads(stdout.strip().splitlines()[-1]))
    return out


def cpu_baseline(seconds: float = 4.0) -> dict:
    """The oracle (serial C, one thread per process) timed on the host's cores
    on bounded samples of the workloads: ns per attempted flip on one core for
    the 2D crop (the headline), the FP64 Heisenberg and one chain of each
    tempering batch, and for the tempering batches the aggregate of
    independent chains run one per core."""
    import workloads as W

    cores = _host_cores()
    rates = {}
    c2 = oracle_job("c2", 1.5 * seconds)
    value = c2["seconds"] / c2["flips"] * 1e9
    rates["ising2d_crop"] = {"ns_per_flip": round(value, 3), "cores": 1, "sample": c2["sample"]}
    c3 = oracle_job("c3", seconds)
    rates["heisenberg3d"] = {"ns_per_flip": round(c3["seconds"] / c3["flips"] * 1e9, 3), "cores": 1,
                             "sample": c3["sample"]}
    for kind, name, sites in (("c4", "ea3d_L16", 16 ** 3),
                              ("c5", "ea2d_uneven", None)):
        one = oracle_job(kind, seconds)
        many = _oracle_children(kind, seconds, cores)
        agg_flips_per_s = sum(r["flips"] / r["seconds"] for r in many)
        if sites is None:  # replica-sweeps/s at the uneven batch's mean lattice size
            cfg = W.ea2d_uneven()
            sites = float(sum(int(L) ** 2 for L in cfg.sizes)) / len(cfg.sizes)
        rates[name] = {"ns_per_flip_one_core": round(one["seconds"] / one["flips"] * 1e9, 3),
                       "replica_sweeps_per_s_one_core": round(one["flips"] / one["seconds"] / sites, 1),
                       "aggregate_replica_sweeps_per_s": round(agg_flips_per_s / sites, 1),
                       "aggregate_cores": cores,
                       "sample": f"{one['sample']}; aggregate: {cores} chains, one process each"}
    return {"value": round(value, 4), "unit": "ns/flip", "cores": 1, "kind": "oracle",
            "sample": c2["sample"] + f" ({c2['seconds']:.1f} s, serial C oracle, 1 thread)",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "host_cores_used": cores,
            "rates": rates}


def under_profiler() -> bool:
    """True when the process runs under rocprofv3 (its tool library is
    preloaded and its options are passed in ROCPROF_* variables)."""
    if "rocprof" in os.environ.get("LD_PRELOAD", ""):
        return True
    return any(k.startswith("ROCPROF") for k in os.environ)


# Profiled runs (rocprofv3 with hardware counters) have stopped with a
# malformed-packet queue error while thousands of small kernels were queued
# back to back without a host synchronisation (the autotuner's replica copies;
# dcb_scan's double-checkerboard launches at L = 64 with a budget of 2e8
# flips).  Under a profiler the sections that queue many small launches are
# held to the sizes with which profiled runs have completed.
PROFILED_LIMITS = {
    "dcb_scan": ("flips", 2e6),
    "dcb3d": ("flips", 2e6),
    "tempering.ising2d_paper": ("flips", 2e8),
    "tempering.ea2d_uneven": ("steps", 40),
}


def profiler_guard(section: str, value: float) -> None:
    if not under_profiler() or section not in PROFILED_LIMITS:
        return
    what, limit = PROFILED_LIMITS[section]
    if value > limit:
        raise RuntimeError(f"{section}: {what} = {value:g} under a profiler (limit {limit:g}, the largest size with "
                           f"which profiled runs have completed); reduce it for profiled runs")


def autotune_report(S, b, envs=({},)):
    """smc_autotune for batch b (once under each environment of envs) and the
    shapes it recorded for b's edge: kind, model, replicas, values."""
    import tempfile

    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "tune.txt")
        for env in envs:
            old = {k: os.environ.get(k) for k in env}
            os.environ.update(env)
            try:
                S.autotune(b, path)
            finally:
                for k, v in old.items():
                    if v is None:
                        os.environ.pop(k, None)
                    else:
                        os.environ[k] = v
        lines = []
        if os.path.exists(path):
            with open(path) as fh:
                lines = [l.split() for l in fh if not l.startswith("#")]
    return [{"kind": l[1], "model": "EA" if l[3] == "1" else "Ising", "replicas": int(l[4]),
             "values": [int(x) for x in l[5:8]]} for l in lines if len(l) == 8 and int(l[2]) == b.L]


def _events():
    import torch

    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _timed(fn):
    """GPU milliseconds of fn() between events on the current stream."""
    import torch

    e0, e1 = _events()
    e0.record()
    fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def _pt_batch(S, model, dim, L, n_chains, n_temps, seed, rps=1, inst=None):
    """Spins, couplings, energies and permutations of a tempering batch, on the device."""
    import torch

    n_rep = n_chains * n_temps
    b = S.Batch(model, dim, L, n_rep, seed, rep_per_sample=rps, inst=inst)
    spins = torch.zeros(b.spins_shape()[0], dtype=torch.int8, device="cuda")
    coup = torch.zeros(b.coup_len(), dtype=torch.int8, device="cuda") if model == S.EA else None
    S.spin_init(b, spins, coup)
    E = torch.zeros(n_rep, dtype=torch.float64, device="cuda")
    S.measure_energy_magnetisation(b, spins, E, couplings=coup)
    sot = torch.arange(n_temps, dtype=torch.int32, device="cuda").repeat(n_chains)
    return b, spins, coup, E, sot


def _section(name, fn):
    """Run one measurement section and report its wall time on stderr."""
    t0 = time.perf_counter()
    res = fn()
    print(f"[bench] {name}: {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    return res


def tempering_ising2d(S, W, sizes=(64, 128, 256, 1024, 2048), n_temps=20, every=(100, 10), flips=2e9):
    """The paper's tempering benchmark (Sec. 6): one chain of 20 replicas of
    the 2D Ising model at inverse temperatures equally spaced in
    [0.1, 0.15], one exchange round per 100 (or 10) sweeps: ps per attempted
    flip (exchange rounds included) against L.  Steps per size are chosen
    for about `flips` attempted flips."""
    import numpy as np

    beta = np.linspace(0.10, 0.15, n_temps)
    profiler_guard("tempering.ising2d_paper", flips)
    rows = []
    for L in sizes:
        for m in every:
            b, spins, coup, E, sot = _pt_batch(S, S.ISING, 2, L, 1, n_temps, W.seed_for(96))
            per_step = n_temps * L * L * m
            steps = max(2, int(flips // per_step))
            _, kernel = S.pt_plan(b, 1, n_temps, beta, steps, sweeps_per_step=m)
            S.pt_sweep_swap(b, 1, n_temps, beta, spins, sot, E, 0, 1, sweeps_per_step=m)  # warm-up
            ms = _timed(lambda: S.pt_sweep_swap(b, 1, n_temps, beta, spins, sot, E, 1, steps, sweeps_per_step=m))
            rows.append({"L": L, "sweeps_per_exchange": m, "steps": steps, "kernel": kernel, "ms": round(ms, 3),
                         "ps_per_flip": round(ms * 1e9 / (per_step * steps), 4)})
            del spins, E, sot
    return {"workload": f"2D Ising parallel tempering, one chain of {n_temps} replicas, beta equally spaced in "
                        f"[0.10, 0.15], one exchange round per m sweeps; ps per attempted flip",
            "by_size": rows}


def tempering_ea3d(S, W, steps, per_inst_chains=16, per_inst_steps=50, per_step_steps=3):
    """3D EA, L = 16, 512 samples x 2 replicas x 32 temperatures: the whole
    batch in one call (one launch), against one call per chain and against
    the generic path's per-step launches over the whole batch."""
    import torch

    cfg = W.ea3d_tempering(steps=steps)
    nc, nt = cfg.n_chains, cfg.n_temps
    rps = cfg.chains_per_sample * nt
    b, spins, coup, E, sot = _pt_batch(S, S.EA, 3, cfg.L, nc, nt, cfg.seed, rps)
    N = cfg.L ** 3
    _, kernel = S.pt_plan(b, nc, nt, cfg.betas, cfg.steps)
    S.pt_sweep_swap(b, nc, nt, cfg.betas, spins, sot, E, 0, 2, couplings=coup)  # warm-up
    ms = _timed(lambda: S.pt_sweep_swap(b, nc, nt, cfg.betas, spins, sot, E, 2, cfg.steps, couplings=coup))
    rate = cfg.steps * nc * nt / (ms * 1e-3)
    # one call per chain: views of the chain's replicas and its sample's couplings
    one = S.Batch(S.EA, 3, cfg.L, nt, cfg.seed, rep_per_sample=nt)

    def per_chain():
        for q in range(per_inst_chains):
            sp = spins[q * nt * N:(q + 1) * nt * N]
            cp = coup[(q * nt // rps) * 3 * N:(q * nt // rps + 1) * 3 * N]
            S.pt_sweep_swap(one, 1, nt, cfg.betas, sp, sot[q * nt:(q + 1) * nt], E[q * nt:(q + 1) * nt], 0,
                            per_inst_steps, couplings=cp)

    per_chain()
    ms_pi = _timed(per_chain)
    rate_pi = per_inst_chains * per_inst_steps * nt / (ms_pi * 1e-3)
    # the generic per-step launches (three per step) over the whole batch
    os.environ["SPINMC_PT3D"] = "0"
    try:
        ms_ps = _timed(lambda: S.pt_sweep_swap(b, nc, nt, cfg.betas, spins, sot, E, 0, per_step_steps,
                                               couplings=coup))
    finally:
        del os.environ["SPINMC_PT3D"]
    rate_ps = per_step_steps * nc * nt / (ms_ps * 1e-3)
    del spins, coup, E, sot
    torch.cuda.empty_cache()
    return {"workload": f"3D +-J EA L=16, {cfg.n_chains // cfg.chains_per_sample} samples x "
                        f"{cfg.chains_per_sample} replicas x {nt} temperatures (T geometric 0.8..2.0), "
                        f"{cfg.steps} steps of sweep + exchange",
            "kernel": kernel, "steps": cfg.steps, "ms": round(ms, 3),
            "replica_sweeps_per_s": round(rate, 1), "ns_per_flip": round(1e9 / (rate * N), 6),
            "per_instance": {"replica_sweeps_per_s": round(rate_pi, 1),
                             "sample": f"{per_inst_chains} chains, {per_inst_steps} steps, one call per chain"},
            "speedup_vs_per_instance": round(rate / rate_pi, 2),
            "per_step_launches": {"replica_sweeps_per_s": round(rate_ps, 1),
                                  "sample": f"whole batch, {per_step_steps} steps, generic kernels"},
            "speedup_vs_per_step_launches": round(rate / rate_ps, 2)}


def msc_ea2d(S, W, sweeps, L=16, sizes=(14, 16, 18, 20), single_spin_sweeps=20):
    """Asynchronous multi-spin coding of the 2D +-J spin glass (Sec. 5,
    Fig. 14 shape): 16 x 16 lattices, replicas in groups of 32 (and 64)
    sharing their draws, at T = 1; ps per attempted flip against the number
    of replicas, and the same batch swept by smc_metropolis_sweep (one
    replica per site update, per-replica draws) for comparison."""
    import torch

    seed = W.seed_for(90)
    rows = []
    for lg in sizes:
        n_rep = 1 << lg
        b = S.Batch(S.EA, 2, L, n_rep, seed)
        spins = torch.zeros(n_rep * L * L, dtype=torch.int8, device="cuda")
        coup = torch.zeros(b.coup_len(), dtype=torch.int8, device="cuda")
        S.spin_init(b, spins, coup)
        n = sweeps << max(0, sizes[-1] - lg)  # about the same number of flips at every size
        S.msc_sweep(b, spins, [1.0], 0, 5, couplings=coup)
        S.kernel_timing_read()
        S.kernel_timing_enable(True)
        ms = _timed(lambda: S.msc_sweep(b, spins, [1.0], 5, n, couplings=coup))
        kernel_ms, _ = S.kernel_timing_read()
        S.kernel_timing_enable(False)
        flips = n_rep * L * L * n
        row = {"replicas": n_rep, "sweeps": n, "ms": round(ms, 3), "ps_per_flip": round(ms * 1e9 / flips, 5),
               "kernel_ps_per_flip": round(kernel_ms * 1e9 / flips, 5)}
        # 64 replicas per draw (the paper's w = 64): two words per thread, one draw
        S.kernel_timing_read()
        S.kernel_timing_enable(True)
        ms64 = _timed(lambda: S.msc_sweep(b, spins, [1.0], 5 + n, n, couplings=coup, word_bits=64))
        kernel_ms64, _ = S.kernel_timing_read()
        S.kernel_timing_enable(False)
        row["w64_ps_per_flip"] = round(ms64 * 1e9 / flips, 5)
        row["w64_kernel_ps_per_flip"] = round(kernel_ms64 * 1e9 / flips, 5)
        if lg == sizes[-1]:
            t = _timed(lambda: S.metropolis_sweep(b, spins, [1.0], 5 + 2 * n, single_spin_sweeps, couplings=coup))
            row["single_spin_ps_per_flip"] = round(t * 1e9 / (n_rep * L * L * single_spin_sweeps), 4)
            row["single_spin_kernel"] = S.sweep_plan(b)[1]
            row["speedup_vs_single_spin"] = round(row["single_spin_ps_per_flip"] / row["ps_per_flip"], 1)
        rows.append(row)
        del spins, coup
        torch.cuda.empty_cache()
    _, kernel = S.msc_plan(S.Batch(S.EA, 2, L, 32, seed), 1)
    return {"workload": f"2D +-J EA {L}x{L}, T = 1, replicas packed 32 per word with shared draws, "
                        f"{sweeps} sweeps at 2^{sizes[-1]} replicas, proportionally more for fewer",
            "kernel": kernel, "by_replicas": rows}


def dcb2d(S, W, sweeps, L=16384, tiles=(64, 128), hits=(1, 2, 4, 8, 16, 64, 100)):
    """Double checkerboard with multi-hit updates (Sec. 3.2, Sec. 3.4) on the
    2D Ising 16384^2 lattice at beta_c: ps per attempted flip against the
    tile edge and the number of hits k per tile (k attempts per site and
    sweep), in place on the caller's int8 spins."""
    import torch

    cfg = W.ising_large(L)
    b = S.Batch(S.ISING, 2, L, 1, cfg.seed)
    spins = torch.empty(L * L, dtype=torch.int8, device="cuda")
    S.spin_init(b, spins)
    rows = []
    t0 = 0
    for tile in tiles:
        for k in hits:
            n = max(2, sweeps // k)
            S.dcb_sweep(b, spins, [cfg.betas[1]], t0, 1, tile, k)
            t0 += 1
            S.kernel_timing_read()
            S.kernel_timing_enable(True)
            ms = _timed(lambda: S.dcb_sweep(b, spins, [cfg.betas[1]], t0, n, tile, k))
            kernel_ms, launches = S.kernel_timing_read()
            S.kernel_timing_enable(False)
            t0 += n
            flips = L * L * k * n
            rows.append({"tile": tile, "hits": k, "sweeps": n, "ms": round(ms, 3),
                         "ps_per_flip": round(ms * 1e9 / flips, 4),
                         "hbm_frac_at_2B_per_site_sweep": round(
                             2.0 * L * L * n / (kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)})
    del spins
    torch.cuda.empty_cache()
    return {"workload": f"2D Ising {L}x{L}, beta_c, double checkerboard with T x T tiles, k hits per tile "
                        f"and sweep, in place on int8 spins",
            "kernel": S.dcb_plan(b, [cfg.betas[1]], tiles[0]), "by_tile_and_hits": rows}


def dcb_scan(S, W, sizes=(64, 256, 1024, 4096, 16384), hits=(1, 100), beta=0.4, flips=4e9):
    """Spin-flip time against L for one 2D Ising lattice at beta = 0.4 (the
    shape of the paper's Figs. 8 and 9): the plain checkerboard sweep and the
    double checkerboard with k = 1 and 100 hits (tiles of 16 up to L = 256,
    64 above)."""
    import torch

    profiler_guard("dcb_scan", flips)
    rows = []
    for L in sizes:
        b = S.Batch(S.ISING, 2, L, 1, W.seed_for(100))
        spins = torch.empty(L * L, dtype=torch.int8, device="cuda")
        S.spin_init(b, spins)
        tile = 16 if L <= 256 else 64
        n = max(2, min(20000, int(flips // (L * L))))  # small lattices: capped by launches
        S.metropolis_sweep(b, spins, [beta], 0, 2)
        ms = _timed(lambda: S.metropolis_sweep(b, spins, [beta], 2, n))
        row = {"L": L, "plain_ps_per_flip": round(ms * 1e9 / (n * L * L), 4), "tile": tile}
        for k in hits:
            nk = max(2, n // k)
            S.dcb_sweep(b, spins, [beta], 0, 1, tile, k)
            ms = _timed(lambda: S.dcb_sweep(b, spins, [beta], 1, nk, tile, k))
            row[f"dcb_k{k}_ps_per_flip"] = round(ms * 1e9 / (nk * k * L * L), 4)
        rows.append(row)
        del spins
    torch.cuda.empty_cache()
    return {"workload": f"2D Ising L x L, one lattice, beta = {beta}: plain checkerboard sweeps and double "
                        f"checkerboard with k hits, ps per attempted flip", "by_size": rows}


def dcb3d(S, W, L=256, hits=(1, 10, 100), beta=0.22, flips=4e9):
    """3D Ising double checkerboard (16^3 tiles; the paper's 3D timings use
    k = 100) on one 256^3 lattice near the critical coupling: ps per
    attempted flip against k, and the plain 3D checkerboard sweep."""
    import torch

    profiler_guard("dcb3d", flips)
    b = S.Batch(S.ISING, 3, L, 1, W.seed_for(102))
    spins = torch.empty(L ** 3, dtype=torch.int8, device="cuda")
    S.spin_init(b, spins)
    n = max(2, int(flips // L ** 3))
    S.metropolis_sweep(b, spins, [beta], 0, 2)
    ms = _timed(lambda: S.metropolis_sweep(b, spins, [beta], 2, n))
    rows = [{"update": "checkerboard", "kernel": S.sweep_plan(b)[1], "ps_per_flip": round(ms * 1e9 / (n * L ** 3), 4)}]
    for k in hits:
        nk = max(2, n // k)
        S.dcb_sweep(b, spins, [beta], 0, 1, 16, k)
        ms = _timed(lambda: S.dcb_sweep(b, spins, [beta], 1, nk, 16, k))
        rows.append({"update": f"double checkerboard k = {k}", "kernel": S.dcb_plan(b, [beta], 16),
                     "ps_per_flip": round(ms * 1e9 / (nk * k * L ** 3), 4)})
    del spins
    torch.cuda.empty_cache()
    return {"workload": f"3D Ising {L}^3, beta = {beta}, one lattice, 16^3 tiles", "rows": rows}


def sweep3d(S, W, sizes=(256, 512, 1024), beta=0.2216, flips=8e9, models=("ising", "ea"), tune=True):
    """Plain 3D checkerboard sweeps (Ising, and EA with one coupling sample)
    on one L^3 lattice: ps per attempted flip for the one-pass segment sweep,
    the two half-sweep launches and the per-site kernels, and the rate at
    2 B/flip (one read and one write of every spin per sweep) against 8 TB/s.
    With tune, smc_autotune first measures the launch shapes of both 3D
    paths for each lattice (the rows report them)."""
    import os
    import torch

    rows = []
    # about half a second of sweeps first, so that the short rows of the
    # small lattice are not timed while the clocks ramp up
    w = S.Batch(S.ISING, 3, 256, 1, W.seed_for(103))
    ws = torch.empty(256 ** 3, dtype=torch.int8, device="cuda")
    S.spin_init(w, ws)
    t_end = time.perf_counter() + 0.5
    while time.perf_counter() < t_end:
        S.metropolis_sweep(w, ws, [beta], 0, 64)
        torch.cuda.synchronize()
    del ws
    for L in sizes:
        for model in [m for name, m in (("ising", S.ISING), ("ea", S.EA)) if name in models]:
            b = S.Batch(model, 3, L, 1, W.seed_for(103))
            spins = torch.empty(L ** 3, dtype=torch.int8, device="cuda")
            coup = torch.empty(3 * L ** 3, dtype=torch.int8, device="cuda") if model == S.EA else None
            S.spin_init(b, spins, coup)
            n = max(2, int(flips // L ** 3) // 2 * 2)  # even: the one-pass sweeps end in the caller's buffer
            row = {"model": "EA" if model == S.EA else "Ising", "L": L, "default": S.sweep_plan(b)[1]}
            if tune:
                row["tuned"] = [t for t in autotune_report(S, b, envs=({"SPINMC_SWEEP3D_PASS": "1"},
                                                                      {"SPINMC_SWEEP3D_PASS": "0"}))
                                if t["model"] == row["model"] and t["replicas"] == 1]
            for key, env in (("pass", {"SPINMC_SWEEP3D_PASS": "1"}), ("half", {"SPINMC_SWEEP3D_PASS": "0"}),
                             ("per_site", {"SPINMC_SWEEP3D": "0"})):
                os.environ.update(env)
                S.metropolis_sweep(b, spins, [beta], 0, 2, couplings=coup)
                S.kernel_timing_read()
                S.kernel_timing_enable(True)
                ms = _timed(lambda: S.metropolis_sweep(b, spins, [beta], 2, n, couplings=coup))
                kernel_ms, launches = S.kernel_timing_read()
                S.kernel_timing_enable(False)
                kernel = S.sweep_plan(b)[1]  # the path taken under this row's environment
                for k in env:
                    os.environ.pop(k, None)
                ps = ms * 1e9 / (n * L ** 3)
                row[key] = {"kernel": kernel, "ps_per_flip": round(ps, 4),
                            "hbm_frac_2B": round(2.0 / (ps * 1e-12) / 8e12, 4),
                            "kernel_us_per_sweep": round(kernel_ms * 1e3 / n, 3) if launches else None}
            rows.append(row)
            del spins, coup
            torch.cuda.empty_cache()
    return {"workload": f"3D Ising and EA (one +-J sample) checkerboard sweeps, one L^3 lattice, beta = {beta}",
            "rows": rows}


def heis_dcb2d(S, W, sweeps=4, L=4096, hits=100, tiles=(32, 64)):
    """The paper's Heisenberg benchmark (Sec. 4): 2D, L = 4096, double
    checkerboard with k = 100 hits, in the three arithmetic modes (float32
    with accurate functions, float32 with hardware functions, float64):
    ps per attempted move, from a random start at beta = 1, and the mean and
    largest deviation of |s| from 1 after the run (no renormalisation falls
    in the 5 sweeps; Fig. 12); also small-step proposals (cap 0.3)."""
    import torch

    seed = W.seed_for(91)
    b = S.Batch(S.HEISENBERG, 2, L, 1, seed, renorm_every=16)
    base = torch.empty(L * L * 3, dtype=torch.float32, device="cuda")
    S.spin_init(b, base)
    rows = []
    cases = [(name, mode, tile, 0.0) for name, mode in (("float", S.HEIS_FLOAT), ("fast", S.HEIS_FAST),
                                                         ("double", S.HEIS_DOUBLE)) for tile in tiles
             if not (mode == S.HEIS_DOUBLE and tile > 32)]
    cases += [("fast", S.HEIS_FAST, tiles[0], 0.3), ("double", S.HEIS_DOUBLE, tiles[0], 0.3)]  # small steps
    for name, mode, tile, cap in cases:
        spins = base.double() if mode == S.HEIS_DOUBLE else base.clone()
        acc = torch.zeros(1, dtype=torch.int64, device="cuda")
        S.heis_dcb_sweep(b, spins, [1.0], 0, 1, tile, hits, precision=mode, cap=cap)
        ms = _timed(lambda: S.heis_dcb_sweep(b, spins, [1.0], 1, sweeps, tile, hits, precision=mode, cap=cap,
                                             accepts=acc))
        flips = L * L * hits * sweeps
        # deviation of |s| from 1 after 5 sweeps without renormalisation (Fig. 12)
        dev = (spins.view(-1, 3).double().norm(dim=1) - 1.0).abs()
        rows.append({"mode": name, "tile": tile, "cap": cap, "ms": round(ms, 3),
                     "ps_per_flip": round(ms * 1e9 / flips, 4),
                     "acceptance": round(float(acc.item()) / flips, 4),
                     "norm_dev_mean": float(f"{dev.mean().item():.3g}"),
                     "norm_dev_max": float(f"{dev.max().item():.3g}")})
        del spins
    torch.cuda.empty_cache()
    return {"workload": f"2D Heisenberg {L}x{L}, beta = 1, double checkerboard with T x T tiles and k = {hits} "
                        f"hits, {sweeps} sweeps after one warm-up sweep",
            "kernel": "k_heis_dcb2d", "by_mode": rows}


TABLE1_EXACT = {"e": 1.106079207, "C": 0.8616983594}  # Table 1, row "exact" (L = 1024, beta = 0.4)


def _e_and_c(E, N, beta):
    """e = -E/N and C_V = beta^2 N var(e) per replica (rows of E), their
    means over replicas and the standard errors from the replica spread."""
    import numpy as np

    e = -np.asarray(E, np.float64) / N
    e_r = e.mean(axis=1)
    c_r = beta * beta * N * e.var(axis=1)
    R = e.shape[0]
    return (float(e_r.mean()), float(e_r.std(ddof=1) / np.sqrt(R)), float(c_r.mean()),
            float(c_r.std(ddof=1) / np.sqrt(R)))


def table1(S, W, updates=10_000_000, n_rep=64, L=1024, beta=0.4, therm=2000, every=10):
    """Table 1 with the Philox streams: internal energy e and specific heat
    C_V of the 1024^2 Ising model at beta = 0.4 from `updates` attempts per
    spin in total (n_rep independent replicas), for the plain checkerboard
    sweep (energy every `every` sweeps) and the double checkerboard with
    64 x 64 tiles and one hit (energy after every sweep); Delta_rel =
    (estimate - exact) / standard error against the printed exact values."""
    import numpy as np
    import torch

    N = L * L
    per_rep = updates // n_rep
    rows = []
    for method in ("checkerboard", "double checkerboard 64x64, k = 1"):
        b = S.Batch(S.ISING, 2, L, n_rep, W.seed_for(97))
        spins = torch.empty(n_rep * N, dtype=torch.int8, device="cuda")
        S.spin_init(b, spins)
        S.metropolis_sweep(b, spins, [beta] * n_rep, 0, therm)
        E0 = torch.empty(n_rep, dtype=torch.float64, device="cuda")
        S.measure_energy_magnetisation(b, spins, E0)
        t0 = time.perf_counter()
        if method == "checkerboard":
            calls = per_rep // every
            dE = torch.zeros(n_rep, dtype=torch.int64, device="cuda")
            trace = torch.empty(calls, n_rep, dtype=torch.int64, device="cuda")
            for i in range(calls):
                S.metropolis_sweep(b, spins, [beta] * n_rep, therm + i * every, every, dE_accum=dE)
                trace[i].copy_(dE)
        else:
            chunk = 4096
            n = per_rep
            trace = torch.empty(n, n_rep, dtype=torch.int64, device="cuda")
            done = 0
            base = torch.zeros(n_rep, dtype=torch.int64, device="cuda")
            while done < n:
                m = min(chunk, n - done)
                S.dcb_sweep(b, spins, [beta] * n_rep, therm + done, m, 64, 1, dE_trace=trace[done:done + m])
                trace[done:done + m] += base
                base = trace[done + m - 1].clone()
                done += m
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        E = (E0.cpu().numpy()[None, :] + trace.cpu().numpy()).T  # [replica, time]
        e, de, c, dc = _e_and_c(E, N, beta)
        rows.append({"method": method, "measurements_per_replica": int(E.shape[1]),
                     "e": round(e, 9), "e_err": float(f"{de:.2g}"),
                     "e_delta_rel": round((e - TABLE1_EXACT["e"]) / de, 2),
                     "C": round(c, 7), "C_err": float(f"{dc:.2g}"),
                     "C_delta_rel": round((c - TABLE1_EXACT["C"]) / dc, 2), "seconds": round(secs, 2)})
        del spins, trace
        torch.cuda.empty_cache()
    return {"workload": f"2D Ising {L}x{L}, beta = {beta}, {n_rep} replicas, {updates:.0e} attempts per spin in "
                        f"total after {therm} sweeps of equilibration (Table 1 with Philox4x32-10)",
            "exact": TABLE1_EXACT, "rows": rows}


RNG_STUDY = (("LCG32", 1), ("LCG32, random", 2), ("LCG64", 3), ("LCG64, random", 4), ("Fibonacci, r=521", 5),
             ("Fibonacci, r=1279", 6))


def table1_generators(S, W, updates=10_000_000, n_rep=64, L=1024, beta=0.4, therm=2000, tile=16, k=1,
                      chunk=256):
    """Table 1's generator rows on the GPU: the 1024^2 Ising model at beta =
    0.4 with the double checkerboard (16 x 16 tiles, one hit) drawing from the
    paper's generators (LCG32 / LCG64 with skip-ahead over one global
    sequence or independently seeded per stream, lagged Fibonacci with
    r = 521 and 1279), `updates` attempts per spin in total over n_rep
    replicas, the energy recorded after every sweep; Delta_rel against the
    printed exact values."""
    import torch

    N = L * L
    per_rep = updates // n_rep
    rows = []
    for name, gen in RNG_STUDY:
        b = S.Batch(S.ISING, 2, L, n_rep, W.seed_for(98))
        spins = torch.empty(n_rep * N, dtype=torch.int8, device="cuda")
        S.spin_init(b, spins)
        state = torch.zeros(S.rng_study_state_bytes(b, tile, gen), dtype=torch.uint8, device="cuda")
        S.rng_study_init(b, tile, gen, state)
        S.rng_study_sweep(b, spins, [beta] * n_rep, therm, tile, k, gen, state)
        E0 = torch.empty(n_rep, dtype=torch.float64, device="cuda")
        S.measure_energy_magnetisation(b, spins, E0)
        trace = torch.empty(per_rep, n_rep, dtype=torch.int64, device="cuda")
        dE = torch.zeros(n_rep, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(per_rep):
            S.rng_study_sweep(b, spins, [beta] * n_rep, 1, tile, k, gen, state, dE_accum=dE)
            trace[i].copy_(dE)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        E = (E0.cpu().numpy()[None, :] + trace.cpu().numpy()).T
        e, de, c, dc = _e_and_c(E, N, beta)
        rows.append({"method": f"double checkerboard {tile}x{tile}, k = {k}, {name}",
                     "measurements_per_replica": int(E.shape[1]),
                     "e": round(e, 9), "e_err": float(f"{de:.2g}"),
                     "e_delta_rel": round((e - TABLE1_EXACT["e"]) / de, 2),
                     "C": round(c, 7), "C_err": float(f"{dc:.2g}"),
                     "C_delta_rel": round((c - TABLE1_EXACT["C"]) / dc, 2), "seconds": round(secs, 2),
                     "ps_per_flip": round(secs * 1e12 / (per_rep * n_rep * N), 3)})
        print(f"[bench] table1 {name}: e = {e:.7f} ({rows[-1]['e_delta_rel']} sd), C = {c:.5f} "
              f"({rows[-1]['C_delta_rel']} sd)", file=sys.stderr, flush=True)
        del spins, trace, state
        torch.cuda.empty_cache()
    return rows


def tau_int(series, c=6.0):
    """Integrated autocorrelation time of equilibrium series (rows =
    independent replicas, columns = measurement times), in units of the
    measurement interval: tau = 1/2 + sum_{t=1}^{W} rho(t), with rho the
    normalised autocorrelation function averaged over replicas (the global
    mean subtracted) and Sokal's self-consistent window, the smallest W with
    W >= c tau(W).  Returns (tau, W, the Madras-Sokal error
    tau sqrt(2 (2W + 1) / (n R)))."""
    import numpy as np

    x = np.asarray(series, np.float64)
    R, n = x.shape
    x = x - x.mean()
    f = np.fft.rfft(x, 2 * n, axis=1)
    acov = np.fft.irfft(f * np.conj(f), axis=1)[:, :n].sum(axis=0) / (R * (n - np.arange(n)))
    rho = acov / acov[0]
    tau, W = 0.5, 0
    for W in range(1, n):
        tau += rho[W]
        if W >= c * tau:
            break
    return float(tau), int(W), float(tau * np.sqrt(2.0 * (2 * W + 1) / (n * R)))


def tau_dcb(S, W, L=128, tile=16, hits=(1, 2, 5, 10, 20, 50, 100), n_rep=256, updates=1 << 15,
            therm=1 << 15, betas=(0.35, 0.40, 0.42, 0.43, 0.4406868, 0.45, 0.46, 0.48, 0.55),
            palindromic_betas=(0.4406868,)):
    """Autocorrelation study of the double checkerboard (Sec. 3.4, the
    paper's 128^2 Ising system with 16 x 16 tiles): for each beta, n_rep
    replicas are brought to equilibrium from an ordered start (a random
    start leaves long-lived stripes below T_c), then each hit count k runs
    updates / k sweeps from that state with the energy measured after every
    sweep (dE_trace); tau_int of the energy is reported in attempts per site
    (tau in sweeps times k) next to the plain checkerboard (one tile, k = 1),
    and with the palindromic order at palindromic_betas.  t_flip is the
    measured time per attempted flip of the same batch, and
    tau~ = tau_int t_flip the time per site for an independent sample."""
    import numpy as np
    import torch

    seed = W.seed_for(90)
    b = S.Batch(S.ISING, 2, L, n_rep, seed)
    N = L * L
    # time per flip of every k on this batch (no trace)
    spins = torch.empty(n_rep * N, dtype=torch.int8, device="cuda")
    S.spin_init(b, spins)
    t_flip = {}
    for k in sorted(set(hits) | {1}):
        for T in sorted({tile, L}):
            if T == L and k != 1:
                continue
            n = max(4, 4096 // k)
            S.dcb_sweep(b, spins, [0.44] * n_rep, 0, 2, T, k)
            ms = _timed(lambda: S.dcb_sweep(b, spins, [0.44] * n_rep, 2, n, T, k))
            t_flip[(T, k)] = ms * 1e9 / (n * k * n_rep * N)  # ps
    rows = []
    todo = [(beta, False) for beta in betas] + [(beta, True) for beta in palindromic_betas]
    for beta, pal in todo:
        bl = [beta] * n_rep
        spins.fill_(1)
        S.dcb_sweep(b, spins, bl, 0, therm // 10, tile, 10)  # equilibrate (any valid update will do)
        E0 = torch.empty(n_rep, dtype=torch.float64, device="cuda")
        S.measure_energy_magnetisation(b, spins, E0)
        runs = ([] if pal else [(L, 1)]) + [(tile, k) for k in hits]
        for i, (T, k) in enumerate(runs):
            n = updates // k
            sp = spins.clone()
            trace = torch.empty(n * n_rep, dtype=torch.int64, device="cuda")
            S.dcb_sweep(b, sp, bl, (i + 1) * (1 << 22) // k, n, T, k, palindromic=pal, dE_trace=trace)
            E = (E0.cpu().numpy()[None, :] + trace.view(n, n_rep).cpu().numpy()).T / N
            tau, Wn, err = tau_int(E)
            rows.append({"beta": beta, "palindromic": pal, "tile": T, "hits": k, "sweeps": n,
                         "tau_int_sweeps": round(tau, 3),
                         "tau_int": round(tau * k, 2), "tau_err": round(err * k, 2), "window": Wn,
                         "e_mean": round(float(E.mean()), 5), "t_flip_ps": round(t_flip[(T, k)], 4),
                         "tau_tilde_ps": round(tau * k * t_flip[(T, k)], 3)})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
            del sp, trace
    return {"workload": f"2D Ising {L}x{L}, {n_rep} replicas per beta, double checkerboard with {tile}x{tile} "
                        f"tiles and k hits (plus the plain sweep: one {L}x{L} tile, k = 1), {updates} attempts per "
                        f"site after {therm} of equilibration; energy after every sweep",
            "tau_unit": "attempts per site", "rows": rows}


def tempering_ea2d_uneven(S, W, steps, per_inst_chains=64, per_inst_steps=3):
    """Uneven 2D EA batch, 4096 instances x 16 temperatures, edges from
    {32, ..., 256}: the batch in one call (a graph of steps), against one call
    per instance on a sample of instances (weighted to the batch's edge mix)."""
    import numpy as np
    import torch

    cfg = W.ea2d_uneven(steps=steps)
    nc, nt = cfg.n_chains, cfg.n_temps
    if under_profiler() and os.environ.get("SPINMC_AUTOTUNE", "") != "0":
        raise RuntimeError("tempering.ea2d_uneven: the workgroup-size autotuner queues thousands of small copies; "
                           "set SPINMC_AUTOTUNE=0 for profiled runs")
    profiler_guard("tempering.ea2d_uneven", cfg.steps)
    inst = W.uneven_table(2, cfg.sizes, nt, S.EA)
    b, spins, coup, E, sot = _pt_batch(S, S.EA, 2, 0, nc, nt, cfg.seed, inst=inst)
    sites = int(sum(int(r[0]) ** 2 for r in inst))
    _, kernel = S.pt_plan(b, nc, nt, cfg.betas, cfg.steps)
    # warm-up with the same step graphs as the timed call (32-step graph and the remainder)
    warm = 32 + cfg.steps % 32 if cfg.steps >= 32 else cfg.steps
    S.pt_sweep_swap(b, nc, nt, cfg.betas, spins, sot, E, 0, warm, couplings=coup)
    ms = _timed(lambda: S.pt_sweep_swap(b, nc, nt, cfg.betas, spins, sot, E, warm, cfg.steps, couplings=coup))
    rate = cfg.steps * nc * nt / (ms * 1e-3)
    # one call per instance, sampled evenly over the batch
    picks = np.linspace(0, nc - 1, per_inst_chains).astype(int)

    def per_instance():
        for q in picks:
            L = int(cfg.sizes[q])
            N = L * L
            so, co = int(inst[q * nt][2]), int(inst[q * nt][3])
            one = S.Batch(S.EA, 2, L, nt, cfg.seed, rep_per_sample=nt)
            S.pt_sweep_swap(one, 1, nt, cfg.betas, spins[so:so + nt * N], sot[q * nt:(q + 1) * nt],
                            E[q * nt:(q + 1) * nt], 0, per_inst_steps, couplings=coup[co:co + 2 * N])

    per_instance()
    ms_pi = _timed(per_instance)
    # time per replica-sweep of the sample, scaled to the batch's mean lattice size
    sample_sites = sum(int(cfg.sizes[q]) ** 2 for q in picks) * nt
    rate_pi_sites = per_inst_steps * sample_sites / (ms_pi * 1e-3)
    rate_pi = rate_pi_sites / (sites / (nc * nt))
    # the same calls spread round-robin over four streams (default priority)
    streams = [torch.cuda.Stream() for _ in range(4)]

    def per_instance_4():
        cur = torch.cuda.current_stream()
        for st in streams:
            st.wait_stream(cur)
        for i, q in enumerate(picks):
            L = int(cfg.sizes[q])
            N = L * L
            so, co = int(inst[q * nt][2]), int(inst[q * nt][3])
            one = S.Batch(S.EA, 2, L, nt, cfg.seed, rep_per_sample=nt)
            S.pt_sweep_swap(one, 1, nt, cfg.betas, spins[so:so + nt * N], sot[q * nt:(q + 1) * nt],
                            E[q * nt:(q + 1) * nt], 0, per_inst_steps, couplings=coup[co:co + 2 * N],
                            stream=streams[i % 4])
        for st in streams:
            cur.wait_stream(st)

    pi4 = None  # not run under a profiler (counters, not times, are wanted there)
    if not under_profiler():
        per_instance_4()
        ms_pi4 = _timed(per_instance_4)
        rate_pi4 = per_inst_steps * sample_sites / (ms_pi4 * 1e-3) / (sites / (nc * nt))
        pi4 = {"replica_sweeps_per_s": round(rate_pi4, 1), "speedup": round(rate / rate_pi4, 2),
               "sample": "the same calls, round-robin over four streams"}
    del spins, coup, E, sot
    torch.cuda.empty_cache()
    return {"workload": f"uneven 2D +-J EA, {nc} instances (L from {{32,48,64,96,128,192,256}}) x {nt} "
                        f"temperatures (T geometric 0.5..2.0), {cfg.steps} steps of sweep + exchange",
            "kernel": kernel, "steps": cfg.steps, "ms": round(ms, 3),
            "replica_sweeps_per_s": round(rate, 1), "ns_per_flip": round(ms * 1e6 / (cfg.steps * sites), 6),
            "per_instance": {"replica_sweeps_per_s": round(rate_pi, 1),
                             "sample": f"{per_inst_chains} instances spread over the batch, {per_inst_steps} "
                                       "steps, one call per instance, rate scaled by lattice size"},
            "speedup_vs_per_instance": round(rate / rate_pi, 2),
            "per_instance_4_streams": pi4}


def heisenberg3d(S, W, sweeps):
    """3D Heisenberg 256^3 at beta = 0.693, float32 spins, renormalised every
    16 sweeps: ns per attempted flip and the HBM roof at 24 B/flip (float32
    3-vector read and written once per sweep)."""
    import torch

    cfg = W.heisenberg_3d()
    L = cfg.L
    N = L ** 3
    b = S.Batch(S.HEISENBERG, 3, L, 1, cfg.seed, renorm_every=cfg.renorm_every)
    spins = torch.zeros(3 * N, dtype=torch.float32, device="cuda")
    S.spin_init(b, spins)
    # half a second of untimed sweeps of a scratch copy first, so that the
    # timed sweeps do not start on a cold chip (this section can run alone)
    warm = spins.clone()
    t_end = time.perf_counter() + 0.5
    while time.perf_counter() < t_end:
        S.metropolis_sweep(b, warm, [cfg.betas[0]], 0, 16)
        torch.cuda.synchronize()
    del warm
    S.metropolis_sweep(b, spins, [cfg.betas[0]], 0, 2)
    S.kernel_timing_read()
    S.kernel_timing_enable(True)
    ms = _timed(lambda: S.metropolis_sweep(b, spins, cfg.betas, 2, sweeps))
    kernel_ms, launches = S.kernel_timing_read()
    S.kernel_timing_enable(False)
    E = torch.zeros(1, dtype=torch.float64, device="cuda")
    S.measure_energy_magnetisation(b, spins, E)
    torch.cuda.synchronize()
    _, kernel = S.sweep_plan(b)
    ps = ms * 1e9 / (sweeps * N)
    achieved = 24.0 * N * sweeps / (kernel_ms * 1e-3) / 1e9
    del spins
    torch.cuda.empty_cache()
    return {"workload": f"3D Heisenberg {L}^3, beta={cfg.betas[0]}, float32 spins, renormalised every "
                        f"{cfg.renorm_every} sweeps, {sweeps} sweeps",
            "kernel": kernel, "sweeps": sweeps, "ms": round(ms, 3), "ns_per_flip": round(ps / 1e3, 6),
            "energy_per_spin": round(float(E.item()) / N, 6),
            "hbm_roof_at_24B_per_flip": {"achieved_GBps": round(achieved, 1), "frac": round(achieved / HBM_PEAK_GBS, 4),
                                         "kernel_us_per_sweep": round(kernel_ms * 1e3 / sweeps, 3),
                                         "traffic": traffic_per_launch(kernel, L)}}


def rng_floor(S, n_threads=1 << 20, per_thread=128, reps=5):
    """Philox4x32-10 alone (the generator throughput probe): time per block
    and what it implies for the sweeps, which draw one block per 8 sites
    (Ising/EA heads) or per site (Heisenberg)."""
    import torch

    out = torch.empty(n_threads, dtype=torch.int32, device="cuda")
    S.philox_bench(1, 0, 0, 6, out, per_thread)  # warm-up
    torch.cuda.synchronize()
    best = min(_timed(lambda: S.philox_bench(1, 0, 0, 6, out, per_thread)) for _ in range(reps))
    blocks = n_threads * per_thread
    ps_per_block = best * 1e9 / blocks
    del out
    return {"kernel": "k_philox_bench", "blocks": blocks, "ms": round(best, 4),
            "ps_per_block": round(ps_per_block, 4),
            "ising_sweep_rng_ps_per_flip": round(ps_per_block / 8, 4),
            "heisenberg_sweep_rng_ps_per_flip": round(ps_per_block, 4)}


def single_lattice(S, cfg, sweeps):
    """The sweep kernel on one lattice alone (beta_c): its time per launch and
    HBM fraction, for comparison with the batched launch."""
    import torch

    L = cfg.L
    N = L * L
    b = S.Batch(S.ISING, 2, L, 1, cfg.seed)
    s = torch.empty(N, dtype=torch.int8, device="cuda")
    S.spin_init(b, s)
    S.metropolis_sweep(b, s, [cfg.betas[1]], 0, 3)
    S.kernel_timing_read()
    S.kernel_timing_enable(True)
    S.metropolis_sweep(b, s, [cfg.betas[1]], 3, sweeps)
    torch.cuda.synchronize()
    kernel_ms, launches = S.kernel_timing_read()
    S.kernel_timing_enable(False)
    us = kernel_ms * 1e3 / launches
    del s
    torch.cuda.empty_cache()
    return {"sweeps": sweeps, "kernel_us_per_launch": round(us, 3),
            "frac": round(BYTES_PER_FLIP * N / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}


def summary(out: dict) -> dict:
    """The figures the metric names, flat, as the last key of the line: the
    headline flip time and HBM fraction, the batched tempering against
    per-instance launches, the Heisenberg HBM fraction and the oracle rates."""
    r = {"ns_per_flip": out["value"], "hbm_frac": out["roofline"]["frac"],
         "kernel_us_per_launch": out["roofline"]["kernel_us_per_launch"],
         "conversion_us_per_call": out["roofline"]["conversion_us_per_call"]}
    temp = out.get("tempering") or {}
    for key, short in (("ea3d_L16", "pt3d"), ("ea2d_uneven", "uneven2d")):
        t = temp.get(key)
        if isinstance(t, dict) and "replica_sweeps_per_s" in t:
            r[f"{short}_replica_sweeps_per_s"] = t["replica_sweeps_per_s"]
            r[f"{short}_per_instance_replica_sweeps_per_s"] = t["per_instance"]["replica_sweeps_per_s"]
            r[f"{short}_speedup_vs_per_instance"] = t["speedup_vs_per_instance"]
            if t.get("per_instance_4_streams"):
                r[f"{short}_speedup_vs_per_instance_4_streams"] = t["per_instance_4_streams"]["speedup"]
    h = out.get("heisenberg")
    if isinstance(h, dict) and "hbm_roof_at_24B_per_flip" in h:
        r["heis3d_ns_per_flip"] = h["ns_per_flip"]
        r["heis3d_hbm_frac"] = h["hbm_roof_at_24B_per_flip"]["frac"]
    s3 = out.get("sweep3d")
    if isinstance(s3, dict):
        # the kernel the library takes by default at each edge
        for row in s3.get("rows", []):
            key = "pass" if row.get("default") == "k_ising3d_pass" else "half"
            if key in row:
                name = f"{row['model'].lower()}3d_L{row['L']}"
                r[f"{name}_ps_per_flip"] = row[key]["ps_per_flip"]
                r[f"{name}_hbm_frac_2B"] = row[key]["hbm_frac_2B"]
    cb = out.get("cpu_baseline")
    if isinstance(cb, dict):
        r["oracle_ns_per_flip_2d"] = cb["value"]
        rates = cb.get("rates", {})
        if "heisenberg3d" in rates:
            r["oracle_ns_per_flip_heis3d"] = rates["heisenberg3d"]["ns_per_flip"]
        for key, short in (("ea3d_L16", "pt3d"), ("ea2d_uneven", "uneven2d")):
            if key in rates:
                r[f"oracle_{short}_replica_sweeps_per_s_{rates[key]['aggregate_cores']}_cores"] = \
                    rates[key]["aggregate_replica_sweeps_per_s"]
        r["host_cores_used"] = cb.get("host_cores_used")
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=600)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--L", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tempering", action="store_true", help="skip the parallel-tempering measurements")
    ap.add_argument("--pt3d-steps", type=int, default=10_000)
    ap.add_argument("--uneven-steps", type=int, default=5000)
    ap.add_argument("--heis-sweeps", type=int, default=1000)
    ap.add_argument("--heis-only", action="store_true", help="only the Heisenberg measurement (for profiling)")
    ap.add_argument("--msc-sweeps", type=int, default=2000)
    ap.add_argument("--dcb-sweeps", type=int, default=64)
    ap.add_argument("--dcb-only", action="store_true", help="only the double-checkerboard measurements")
    ap.add_argument("--sweep3d-only", action="store_true", help="only the plain 3D Ising / EA sweep measurements")
    ap.add_argument("--sweep3d-sizes", type=int, nargs="+", default=[256, 512, 1024])
    ap.add_argument("--sweep3d-models", nargs="+", default=["ising", "ea"], choices=["ising", "ea"])
    ap.add_argument("--dcb-scan-flips", type=float, default=4e9,
                    help="attempted flips per lattice size and update in the L scan")
    ap.add_argument("--heis-dcb-sweeps", type=int, default=4)
    ap.add_argument("--heis-dcb-only", action="store_true",
                    help="only the 2D Heisenberg double checkerboard (L = 4096, k = 100, three modes)")
    ap.add_argument("--paper-pt-sizes", default="64,128,256,1024,2048",
                    help="lattice edges of the 20-replica 2D Ising tempering section")
    ap.add_argument("--paper-pt-flips", type=float, default=2e9,
                    help="attempted flips per size and exchange interval in that section")
    ap.add_argument("--pt-ising-only", action="store_true",
                    help="only the 2D Ising tempering benchmark of 20 replicas (L = 64 .. 2048)")
    ap.add_argument("--table1-only", action="store_true",
                    help="only Table 1 with the Philox streams (1024^2, beta = 0.4, 1e7 attempts per spin)")
    ap.add_argument("--table1-updates", type=float, default=1e7,
                    help="attempts per spin in total for each Table 1 row (the paper: 1e7)")
    ap.add_argument("--tau-only", action="store_true",
                    help="only the double-checkerboard autocorrelation study (128^2, 16x16 tiles)")
    ap.add_argument("--tau-updates", type=int, default=1 << 15, help="attempts per site per (beta, k) series")
    ap.add_argument("--tau-replicas", type=int, default=256)
    ap.add_argument("--msc-only", action="store_true", help="only the multi-spin-coded measurement (for profiling)")
    ap.add_argument("--pmc-kernel", default="k_ising2d_split", choices=sorted(KERNEL_SOURCES),
                    help="kernel of the --pmc-summary and --kt-summary")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter scale for the traffic figure)")
    ap.add_argument("--pmc-summary", nargs=4, metavar=("FETCH_DB", "WRITE_DB", "COPY_FETCH_DB", "COPY_WRITE_DB"),
                    help="write the traffic summary of the sweep kernel from rocprofv3 counter databases")
    ap.add_argument("--pmc-grid", choices=["most", "largest"], default="most",
                    help="dispatches of the --pmc-summary: the grid with the most dispatches, or the largest grid")
    ap.add_argument("--pmc-command", action="append", default=[],
                    help="command line recorded in the traffic summary (repeatable)")
    ap.add_argument("--kt-summary", nargs=2, metavar=("KT_DB", "KT_LOG"),
                    help="write the kernel-trace summary from a rocprofv3 database and the run's output")
    ap.add_argument("--kt-command", default="", help="command line recorded in the kernel-trace summary")
    ap.add_argument("--valu-summary", metavar="DB", help="write the VALU utilisation summary from a --pmc database")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes (no smc_autotune before the measurements)")
    ap.add_argument("--preheat-s", type=float, default=1.0,
                    help="seconds of untimed sweeps of the headline batch before the warm-up sweeps")
    ap.add_argument("--oracle-job", nargs=3, metavar=("KIND", "SECONDS", "INDEX"), help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_job:
        kind, sec, idx = args.oracle_job
        print(json.dumps(oracle_job(kind, float(sec), int(idx))))
        return
    if args.valu_summary:
        valu_summary(args.valu_summary, args.pmc_command[0] if args.pmc_command else "")
        return
    kernel_L = {"k_heis3d_tiled": 256, "k_ising3d_half": max(args.sweep3d_sizes),
                "k_ising3d_pass": max(args.sweep3d_sizes), "k_pt3d_chain": 16,
                "k_uneven2d_sweep": 256}.get(args.pmc_kernel, args.L)
    if args.kt_summary:
        kt_summary(*args.kt_summary, kernel=args.pmc_kernel, L=kernel_L, command=args.kt_command)
        return
    if args.pmc_summary:
        pmc_L = kernel_L
        pmc_summary(*args.pmc_summary, kernel=args.pmc_kernel, L=pmc_L,
                    commands=args.pmc_command, grid_rule=args.pmc_grid)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    if args.copy_calibration:
        copy_calibration()
        return
    import paper_1101_1427_amd as S
    import workloads as W

    if args.heis_only:
        print(json.dumps({"heisenberg": heisenberg3d(S, W, args.heis_sweeps)}))
        return
    if args.msc_only:
        print(json.dumps({"msc_ea2d": msc_ea2d(S, W, args.msc_sweeps)}))
        return
    if args.dcb_only:
        print(json.dumps({"dcb2d": dcb2d(S, W, args.dcb_sweeps),
                          "dcb_scan": dcb_scan(S, W, flips=args.dcb_scan_flips),
                          "dcb3d": dcb3d(S, W, flips=args.dcb_scan_flips)}))
        return
    if args.sweep3d_only:
        print(json.dumps({"sweep3d": sweep3d(S, W, sizes=tuple(args.sweep3d_sizes), models=tuple(args.sweep3d_models),
                                             tune=not args.no_autotune)}))
        return
    if args.heis_dcb_only:
        print(json.dumps({"heis_dcb2d": heis_dcb2d(S, W, sweeps=args.heis_dcb_sweeps)}))
        return
    if args.pt_ising_only:
        sizes = tuple(int(x) for x in args.paper_pt_sizes.split(","))
        print(json.dumps({"ising2d_paper": tempering_ising2d(S, W, sizes=sizes, flips=args.paper_pt_flips)}))
        return
    if args.table1_only:
        t1 = table1(S, W, updates=int(args.table1_updates))
        t1["rows"] += table1_generators(S, W, updates=int(args.table1_updates))
        print(json.dumps({"table1": t1}))
        return
    if args.tau_only:
        print(json.dumps({"tau_dcb": tau_dcb(S, W, n_rep=args.tau_replicas, updates=args.tau_updates)}))
        return
    cfg = W.ising_large(args.L)
    L = cfg.L
    N = L * L
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # The workload's three lattices (one per beta) are one batch of three
    # replicas: a step is one sweep of all three (one launch).
    nb = len(cfg.betas)
    b = S.Batch(S.ISING, 2, L, nb, cfg.seed)
    # launch shapes measured for this batch first (untimed; the band height
    # of the one-pass kernel)
    t_tune = time.perf_counter()
    tuned = [] if args.no_autotune else autotune_report(S, b)
    tune_s = time.perf_counter() - t_tune
    spins = torch.empty(nb * N, dtype=torch.int8, device=dev)
    S.spin_init(b, spins)
    dE = torch.zeros(nb, dtype=torch.int64, device=dev)
    steps = max(1, args.steps)
    warm = max(1, args.warmup)
    # Pre-heat: untimed sweeps of the same batch for a stated time, so that the
    # timed sweeps run on a chip at its working clocks (a fresh device starts
    # slow).  The sweep indices continue across pre-heat, warm-up and timing.
    t_pre = time.perf_counter()
    pre = 0
    while True:
        S.metropolis_sweep(b, spins, cfg.betas, pre, 8, dE_accum=dE)
        pre += 8
        torch.cuda.synchronize()
        if time.perf_counter() - t_pre >= args.preheat_s:
            break
    preheat_s = time.perf_counter() - t_pre
    S.metropolis_sweep(b, spins, cfg.betas, pre, warm, dE_accum=dE)
    torch.cuda.synchronize()

    # Timed region: one call.  The library brackets the sweep kernels of the
    # call with HIP events on the stream they run on, which gives the
    # kernel's own time apart from the layout conversions.
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    S.kernel_timing_read()  # drop anything recorded before
    S.kernel_timing_enable(True)
    t_wall = time.perf_counter()
    ev0.record(stream)
    S.metropolis_sweep(b, spins, cfg.betas, pre + warm, steps, dE_accum=dE)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    kernel_ms, launches = S.kernel_timing_read()
    S.kernel_timing_enable(False)
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / steps
    ns_per_flip = gpu_ms * 1e6 / (steps * nb * N)

    launches_per_sweep, kernel = S.sweep_plan(b)
    launch_ms = kernel_ms / launches
    bytes_per_launch = BYTES_PER_FLIP * nb * N / launches_per_sweep
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    conversion_ms = gpu_ms - kernel_ms
    traffic = traffic_per_launch(kernel, L)
    del spins
    torch.cuda.empty_cache()
    single = single_lattice(S, cfg, min(steps, 200))
    rng = rng_floor(S)
    rng["share_of_ising_sweep"] = round(rng["ising_sweep_rng_ps_per_flip"] / (launch_ms * 1e9 / (nb * N)), 4)

    out = {
        "metric": "ns per spin flip (+% HBM roofline); batched PT sweeps/s vs per-instance",
        "value": round(ns_per_flip, 6),
        "unit": "ns/flip",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": f"2D Ising {L}x{L} periodic, int8 spins, random start, three lattices at beta "
                               f"{{0.30, ln(1+sqrt2)/2, 0.50}} swept together as one batch of three replicas "
                               f"(one launch per sweep), {steps} sweeps, Delta E tracked",
                   "L": L, "betas": cfg.betas, "replicas": nb, "sweeps": steps, "seed": cfg.seed},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": kernel, "launches_per_sweep": launches_per_sweep,
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "kernel_us_per_launch": round(launch_ms * 1e3, 3),
                     "conversion_us_per_call": round(conversion_ms * 1e3, 3),
                     "single_lattice": single, "rng_floor": rng,
                     "autotune": {"seconds": round(tune_s, 3), "shapes": tuned}},
        "wall_s": round(wall, 4),
        "preheat_s": round(preheat_s, 3),
        "preheat_sweeps": pre,
    }
    if not args.no_tempering:
        sizes = tuple(int(x) for x in args.paper_pt_sizes.split(","))
        out["heisenberg"] = _section("heisenberg", lambda: heisenberg3d(S, W, args.heis_sweeps))
        out["tempering"] = {
            "ea3d_L16": _section("tempering.ea3d_L16", lambda: tempering_ea3d(S, W, args.pt3d_steps)),
            "ea2d_uneven": _section("tempering.ea2d_uneven", lambda: tempering_ea2d_uneven(S, W, args.uneven_steps)),
            "ising2d_paper": _section("tempering.ising2d_paper",
                                      lambda: tempering_ising2d(S, W, sizes=sizes, flips=args.paper_pt_flips))}
        out["msc_ea2d"] = _section("msc_ea2d", lambda: msc_ea2d(S, W, args.msc_sweeps))
        out["dcb2d"] = _section("dcb2d", lambda: dcb2d(S, W, args.dcb_sweeps))
        out["dcb_scan"] = _section("dcb_scan", lambda: dcb_scan(S, W, flips=args.dcb_scan_flips))
        out["dcb3d"] = _section("dcb3d", lambda: dcb3d(S, W, flips=args.dcb_scan_flips))
        out["sweep3d"] = _section("sweep3d", lambda: sweep3d(S, W, tune=not args.no_autotune))
        out["heis_dcb2d"] = _section("heis_dcb2d", lambda: heis_dcb2d(S, W, sweeps=args.heis_dcb_sweeps))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = _section("cpu_baseline", cpu_baseline)
    out["summary"] = summary(out)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
