"""ctypes binding of the serial CPU oracle (``spinmc_oracle.c``).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use this module to obtain reference results; the product library
never imports it.  The C file is built with plain gcc (``build()``), it
shares no code with the HIP library.

Arrays are numpy arrays in the layouts of the C functions:
  Ising / EA spins   int8  [N]          (x fastest)
  couplings          int8  [d][N]       (bond mu of site i joins i and i+e_mu)
  Heisenberg spins   float64 [N][3]
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "spinmc_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(LIB)
        i8p = np.ctypeslib.ndpointer(np.int8, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(np.uint64, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        vp = C.c_void_p
        I, U32, U64, D, I64 = C.c_int, C.c_uint32, C.c_uint64, C.c_double, C.c_int64
        sig = {
            "orc_philox4x32_10": (None, [u32p, u32p, u32p]),
            "orc_metropolis_u32": (U32, [U64, U32, U32, I, U64]),
            "orc_init_spins": (None, [I, I, U64, U32, i8p]),
            "orc_init_couplings": (None, [I, I, U64, U32, i8p]),
            "orc_init_heis": (None, [I, I, U64, U32, f64p]),
            "orc_thresholds": (None, [D, I, u64p]),
            "orc_half_sweep": (I64, [I, I, vp, i8p, D, U64, U32, U32, I]),
            "orc_sweep": (I64, [I, I, vp, i8p, D, U64, U32, U32]),
            "orc_run": (I64, [I, I, vp, i8p, D, U64, U32, U32, I]),
            "orc_energy": (I64, [I, I, vp, i8p]),
            "orc_magnetisation": (I64, [I, I, i8p]),
            "orc_run_series": (None, [I, I, vp, i8p, D, U64, U32, U32, I, i64p, i64p]),
            "orc_heis_half_sweep": (I64, [I, I, f64p, D, U64, U32, U32, I]),
            "orc_heis_renormalise": (None, [I, I, f64p]),
            "orc_heis_half_sweep_gaps": (I64, [I, I, f64p, D, U64, U32, U32, I, f64p]),
            "orc_heis_sweep": (I64, [I, I, f64p, D, U64, U32, U32, I]),
            "orc_heis_run": (I64, [I, I, f64p, D, U64, U32, U32, I, I]),
            "orc_heis_energy": (D, [I, I, f64p]),
            "orc_heis_magnetisation": (None, [I, I, f64p, f64p]),
            "orc_pt_step": (None, [I, I, vp, i8p, I, f64p, i32p, i64p, U64, U32, U32, U32, I, vp]),
            "orc_pt_run": (None, [I, I, vp, i8p, I, f64p, i32p, i64p, U64, U32, U32, U32, I, I, vp]),
            "orc_swap_u53": (D, [U64, U32, U32, U32]),
            "orc_pt_audit": (None, [u64p, C.POINTER(C.c_double), I]),
            "orc_window_run": (None, [I, I, I, I, i8p, D, U64, U32, U32, I]),
            "orc_dcb_run": (I64, [I, I, I, vp, i8p, D, U64, U32, U32, I, I]),
            "orc_dcb_run3": (I64, [I, I, I, vp, i8p, D, U64, U32, U32, I, I]),
            "orc_heis_dcb_run": (I64, [I, I, I, f64p, D, U64, U32, U32, I, I, I, D]),
            "orc_rng_state_words": (I64, [I, I, I]),
            "orc_rng_init": (None, [I, I, I, U64, U32, u64p]),
            "orc_dcb_run_rng": (I64, [I, I, I, vp, i8p, D, I, u64p, I]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def n_sites(dim: int, L: int) -> int:
    return L ** dim


# ---------------------------------------------------------------- RNG ----
def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(c, k, out)
    return out


def metropolis_u32(seed: int, t: int, r: int, c: int, h: int) -> int:
    return int(lib().orc_metropolis_u32(seed, t, r, c, h))


def swap_u53(seed: int, k: int, t: int, q: int) -> float:
    return float(lib().orc_swap_u53(seed, k, t, q))


# ------------------------------------------------------------ discrete ---
def init_spins(dim: int, L: int, seed: int, r: int) -> np.ndarray:
    s = np.zeros(n_sites(dim, L), np.int8)
    lib().orc_init_spins(dim, L, seed, r, s)
    return s


def init_couplings(dim: int, L: int, seed: int, q: int) -> np.ndarray:
    J = np.zeros(dim * n_sites(dim, L), np.int8)
    lib().orc_init_couplings(dim, L, seed, q, J)
    return J


def thresholds(beta: float, dim: int) -> np.ndarray:
    thr = np.zeros(dim + 1, np.uint64)
    lib().orc_thresholds(beta, dim, thr)
    return thr


def half_sweep(dim, L, J, s, beta, seed, r, t, c) -> int:
    return int(lib().orc_half_sweep(dim, L, _ptr(J), s, beta, seed, r, t, c))


def sweep(dim, L, J, s, beta, seed, r, t) -> int:
    return int(lib().orc_sweep(dim, L, _ptr(J), s, beta, seed, r, t))


def run(dim, L, J, s, beta, seed, r, t0, n) -> int:
    """n sweeps t0..t0+n-1 in place; returns the summed Delta E of accepted flips."""
    return int(lib().orc_run(dim, L, _ptr(J), s, beta, seed, r, t0, n))


def run_series(dim, L, J, s, beta, seed, r, t0, n):
    """n sweeps in place; returns (E, M) int64 arrays recorded after each sweep."""
    E = np.zeros(n, np.int64)
    M = np.zeros(n, np.int64)
    lib().orc_run_series(dim, L, _ptr(J), s, beta, seed, r, t0, n, E, M)
    return E, M


def energy(dim, L, J, s) -> int:
    return int(lib().orc_energy(dim, L, _ptr(J), s))


def magnetisation(dim, L, s) -> int:
    return int(lib().orc_magnetisation(dim, L, s))


# ---------------------------------------------------------- Heisenberg ---
def init_heis(dim: int, L: int, seed: int, r: int) -> np.ndarray:
    s = np.zeros((n_sites(dim, L), 3), np.float64)
    lib().orc_init_heis(dim, L, seed, r, s)
    return s


def heis_half_sweep(dim, L, s, beta, seed, r, t, c) -> int:
    return int(lib().orc_heis_half_sweep(dim, L, s, beta, seed, r, t, c))


def heis_sweep_gaps(dim, L, s, beta, seed, r, t, renorm_every=16):
    """Sweep t (orc_heis_sweep's moves and renormalisation) that also returns,
    per site, the acceptance margin u - exp(-beta Delta E) of its move (+inf
    where Delta E <= 0): (accepted moves, gaps float64 [N])."""
    gap = np.full(n_sites(dim, L), np.inf)
    n = int(lib().orc_heis_half_sweep_gaps(dim, L, s, beta, seed, r, t, 0, gap))
    n += int(lib().orc_heis_half_sweep_gaps(dim, L, s, beta, seed, r, t, 1, gap))
    if renorm_every > 0 and (t + 1) % renorm_every == 0:
        heis_renormalise(dim, L, s)
    return n, gap


def heis_sweep(dim, L, s, beta, seed, r, t, renorm_every=16) -> int:
    return int(lib().orc_heis_sweep(dim, L, s, beta, seed, r, t, renorm_every))


def heis_run(dim, L, s, beta, seed, r, t0, n, renorm_every=16) -> int:
    return int(lib().orc_heis_run(dim, L, s, beta, seed, r, t0, n, renorm_every))


def heis_renormalise(dim, L, s) -> None:
    lib().orc_heis_renormalise(dim, L, s)


def heis_energy(dim, L, s) -> float:
    return float(lib().orc_heis_energy(dim, L, s))


def heis_magnetisation(dim, L, s) -> np.ndarray:
    m = np.zeros(3, np.float64)
    lib().orc_heis_magnetisation(dim, L, s, m)
    return m


# ---------------------------------------------------- parallel tempering --
def pt_run(dim, L, J, spins, beta, slot_of_temp, E, seed, q, r0, t0, n_steps, swap_acc=None, sweeps_per_step=1):
    """n_steps PT steps of one chain in place (each: sweeps_per_step sweeps,
    then an exchange round).

    spins: int8 [n_temps, N]; beta: float64 [n_temps]; slot_of_temp: int32
    [n_temps]; E: int64 [n_temps] (energy per slot); swap_acc: uint64
    [n_temps] or None.
    """
    n_temps = len(beta)
    lib().orc_pt_run(dim, L, _ptr(J), spins.reshape(-1), n_temps, np.ascontiguousarray(beta, np.float64),
                     slot_of_temp, E, seed, q, r0, t0, n_steps, sweeps_per_step, _ptr(swap_acc))


def pt_audit(reset: bool = False) -> dict:
    """Exchange attempts with x < 0 made by the oracle since the last reset,
    how many had |u53 - exp(x)| < 2^-40 (a decision that a one-ulp difference
    in exp could change), and the smallest gap |u53 - exp(x)| seen."""
    counts = np.zeros(2, np.uint64)
    gap = C.c_double(0.0)
    lib().orc_pt_audit(counts, C.byref(gap), 1 if reset else 0)
    return {"attempts": int(counts[0]), "near_ties": int(counts[1]), "min_gap": gap.value}


def dcb_run(L, T, k, J, s, beta, seed, r, t0, n, palindromic=False, dim=2) -> int:
    """n double-checkerboard sweeps (T^dim tiles, k hits per tile) of a 2D or
    3D lattice in place; returns the summed Delta E (orc_dcb_run, orc_dcb_run3)."""
    f = lib().orc_dcb_run if dim == 2 else lib().orc_dcb_run3
    return int(f(L, T, k, _ptr(J), s, beta, seed & 0xFFFFFFFFFFFFFFFF, r, t0, n, 1 if palindromic else 0))


# Generators of the random-number study (Table 1): codes of orc_dcb_run_rng.
GEN_LCG32, GEN_LCG32_RANDOM, GEN_LCG64, GEN_LCG64_RANDOM, GEN_FIB521, GEN_FIB1279 = 1, 2, 3, 4, 5, 6


def rng_init(gen, L, T, seed, rep) -> np.ndarray:
    """Initial state (uint64 words) of a study generator for one replica."""
    n = int(lib().orc_rng_state_words(gen, L, T))
    st = np.zeros(max(n, 1), np.uint64)
    lib().orc_rng_init(gen, L, T, seed & 0xFFFFFFFFFFFFFFFF, rep, st)
    return st


def dcb_run_rng(L, T, k, J, s, beta, gen, state, n) -> int:
    """n double-checkerboard sweeps (T x T tiles, k hits) drawing from a study
    generator whose state advances in place (orc_dcb_run_rng)."""
    return int(lib().orc_dcb_run_rng(L, T, k, _ptr(J), s, beta, gen, state, n))


def heis_dcb_run(L, T, k, s, beta, seed, r, t0, n, palindromic=False, renorm_every=16, cap=0.0) -> int:
    """n double-checkerboard sweeps (T x T tiles, k hits per tile) of a 2D
    Heisenberg lattice (float64 [N*3]) in place, with uniform proposals
    (cap = 0) or small steps on a cap of size cap; returns the number of
    accepted moves (orc_heis_dcb_run)."""
    return int(lib().orc_heis_dcb_run(L, T, k, s, beta, seed & 0xFFFFFFFFFFFFFFFF, r, t0, n,
                                      1 if palindromic else 0, renorm_every, cap))


def window_run(L, x0, y0, win, beta, seed, r, t0, n):
    """n sweeps of a W x W window (site (x0+u, y0+v) mod L at win[v, u]) of a
    2D Ising lattice of edge L, its outer ring held fixed; sites farther than
    2n from the ring end as in the full lattice (orc_window_run)."""
    W = win.shape[0]
    assert win.shape == (W, W) and win.dtype == np.int8 and win.flags.c_contiguous
    lib().orc_window_run(L, W, x0, y0, win.reshape(-1), beta, seed & 0xFFFFFFFFFFFFFFFF, r, t0, n)
