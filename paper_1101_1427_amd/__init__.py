"""Python binding of libspinmc.so (checkerboard Metropolis / parallel tempering on MI355X).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI (``include/spinmc.h``).  Tensors are torch tensors on the
current HIP device; calls are enqueued on ``torch.cuda.current_stream()``
unless a stream is given.  There is no CPU fallback: if the library is
missing, importing the binding's functions raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspinmc.so")

ISING, EA, HEISENBERG = 0, 1, 2
OK, EINVAL, EUNSUPPORTED, EHIP, ENOMEM = 0, -1, -2, -3, -4


class SpinMCError(RuntimeError):
    def __init__(self, code: int, func: str, detail: str):
        self.code = code
        super().__init__(f"{func} failed with status {code}: {detail}")


class Inst(C.Structure):
    _fields_ = [("L", C.c_int32), ("sample", C.c_int32), ("spin_off", C.c_int64), ("coup_off", C.c_int64)]


class Desc(C.Structure):
    _fields_ = [("model", C.c_int32), ("dim", C.c_int32), ("L", C.c_int32), ("n_rep", C.c_int32),
                ("rep_per_sample", C.c_int32), ("renorm_every", C.c_int32), ("seed", C.c_uint64),
                ("inst", C.POINTER(Inst)), ("spins_len", C.c_int64), ("coup_len", C.c_int64)]


class PTDesc(C.Structure):
    _fields_ = [("n_chains", C.c_int32), ("n_temps", C.c_int32), ("beta_per_chain", C.c_int32),
                ("sweeps_per_step", C.c_int32), ("beta", C.POINTER(C.c_double))]


_lib = None


def lib():
    """The loaded libspinmc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1101_1427_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        vp, P = C.c_void_p, C.POINTER
        L.smc_spin_init.argtypes = [P(Desc), vp, vp, vp]
        L.smc_metropolis_sweep.argtypes = [P(Desc), vp, vp, P(C.c_double), C.c_uint64, C.c_int32, vp, vp]
        L.smc_pt_sweep_swap.argtypes = [P(Desc), P(PTDesc), vp, vp, vp, vp, C.c_uint64, C.c_int32, vp, vp]
        L.smc_measure_energy_magnetisation.argtypes = [P(Desc), vp, vp, vp, vp, vp]
        L.smc_measure_energy_magnetisation_noalloc.argtypes = [P(Desc), vp, vp, vp, vp, vp]
        for f in (L.smc_spin_init, L.smc_metropolis_sweep, L.smc_pt_sweep_swap, L.smc_measure_energy_magnetisation,
                  L.smc_measure_energy_magnetisation_noalloc):
            f.restype = C.c_int
        L.smc_sweep_plan.argtypes = [P(Desc), P(C.c_int32), P(C.c_char_p)]
        L.smc_sweep_plan.restype = C.c_int
        L.smc_pt_plan.argtypes = [P(Desc), P(PTDesc), C.c_int32, P(C.c_int32), P(C.c_char_p)]
        L.smc_pt_plan.restype = C.c_int
        L.smc_kernel_timing_enable.argtypes = [C.c_int]
        L.smc_kernel_timing_enable.restype = C.c_int
        L.smc_kernel_timing_read.argtypes = [P(C.c_double), P(C.c_int64)]
        L.smc_kernel_timing_read.restype = C.c_int
        L.smc_msc_sweep.argtypes = [P(Desc), C.c_void_p, C.c_void_p, P(C.c_double), C.c_uint64, C.c_int32,
                                    C.c_int32, C.c_void_p, C.c_void_p]
        L.smc_msc_sweep.restype = C.c_int
        L.smc_msc_plan.argtypes = [P(Desc), C.c_int32, C.c_int32, P(C.c_int32), P(C.c_char_p)]
        L.smc_msc_plan.restype = C.c_int
        L.smc_dcb_sweep.argtypes = [P(Desc), C.c_void_p, C.c_void_p, P(C.c_double), C.c_uint64, C.c_int32,
                                    C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
        L.smc_dcb_sweep.restype = C.c_int
        L.smc_heis_dcb_sweep.argtypes = [P(Desc), C.c_void_p, P(C.c_double), C.c_uint64, C.c_int32, C.c_int32,
                                         C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_void_p, C.c_void_p]
        L.smc_heis_dcb_sweep.restype = C.c_int
        L.smc_autotune.argtypes = [P(Desc), C.c_char_p, C.c_void_p]
        L.smc_autotune.restype = C.c_int
        L.smc_dcb_plan.argtypes = [P(Desc), P(C.c_double), C.c_int32, P(C.c_char_p)]
        L.smc_dcb_plan.restype = C.c_int
        L.smc_rng_study_state_bytes.argtypes = [P(Desc), C.c_int32, C.c_int32, P(C.c_int64)]
        L.smc_rng_study_state_bytes.restype = C.c_int
        L.smc_rng_study_init.argtypes = [P(Desc), C.c_int32, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p]
        L.smc_rng_study_init.restype = C.c_int
        L.smc_rng_study_sweep.argtypes = [P(Desc), C.c_void_p, C.c_void_p, P(C.c_double), C.c_int32, C.c_int32,
                                          C.c_int32, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]
        L.smc_rng_study_sweep.restype = C.c_int
        L.smc_philox_bench.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_int32, C.c_int32,
                                       C.c_void_p, C.c_void_p]
        L.smc_philox_bench.restype = C.c_int
        L.smc_strerror.argtypes = [C.c_int]
        L.smc_strerror.restype = C.c_char_p
        L.smc_last_error.argtypes = []
        L.smc_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc: int, func: str):
    if rc != OK:
        L = lib()
        raise SpinMCError(rc, func, f"{L.smc_strerror(rc).decode()}: {L.smc_last_error().decode()}")


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


@dataclass
class Batch:
    """A batch of replicas.  Uniform (L > 0) or uneven (L == 0 with ``inst``,
    an int64 array of rows (L, sample, spin_off, coup_off))."""
    model: int
    dim: int
    L: int
    n_rep: int
    seed: int
    rep_per_sample: int = 1
    renorm_every: int = 0
    inst: np.ndarray | None = None

    def sites(self, L=None):
        L = self.L if L is None else L
        return L ** self.dim

    def spins_shape(self):
        per = 3 if self.model == HEISENBERG else 1
        if self.L > 0:
            return (self.n_rep * self.sites() * per,)
        ends = [int(r[2]) + self.sites(int(r[0])) for r in self.inst]
        return (max(ends) * per,)

    def coup_len(self):
        if self.model != EA:
            return 0
        if self.L > 0:
            n_samples = -(-self.n_rep // self.rep_per_sample)
            return n_samples * self.dim * self.sites()
        return max(int(r[3]) + self.dim * self.sites(int(r[0])) for r in self.inst)

    def desc(self, spins_len: int, coup_len: int) -> Desc:
        d = Desc(self.model, self.dim, self.L, self.n_rep, self.rep_per_sample, self.renorm_every,
                 self.seed & 0xFFFFFFFFFFFFFFFF, None, spins_len, coup_len)
        if self.L == 0:
            rows = (Inst * self.n_rep)()
            for k, r in enumerate(self.inst):
                rows[k] = Inst(int(r[0]), int(r[1]), int(r[2]), int(r[3]))
            d._inst_keep = rows  # keep alive for the call
            d.inst = C.cast(rows, C.POINTER(Inst))
        return d


def _desc(batch: Batch, spins, couplings):
    return batch.desc(spins.numel(), 0 if couplings is None else couplings.numel())


def spin_init(batch: Batch, spins, couplings=None, stream=None):
    """Random start (and bimodal couplings for EA); see smc_spin_init."""
    d = _desc(batch, spins, couplings)
    _check(lib().smc_spin_init(C.byref(d), _ptr(spins), _ptr(couplings), _stream(stream)), "smc_spin_init")


def metropolis_sweep(batch: Batch, spins, beta, sweep0: int, n_sweeps: int, couplings=None, dE_accum=None,
                     stream=None):
    """n_sweeps checkerboard Metropolis sweeps; beta is a host sequence [n_rep]."""
    d = _desc(batch, spins, couplings)
    b = np.ascontiguousarray(np.broadcast_to(np.asarray(beta, np.float64), (batch.n_rep,)))
    _check(lib().smc_metropolis_sweep(C.byref(d), _ptr(spins), _ptr(couplings),
                                      b.ctypes.data_as(C.POINTER(C.c_double)), sweep0, n_sweeps,
                                      _ptr(dE_accum), _stream(stream)), "smc_metropolis_sweep")


def msc_sweep(batch: Batch, spins, beta, sweep0: int, n_sweeps: int, couplings=None, dE_accum=None,
              word_bits: int = 32, stream=None):
    """n_sweeps sweeps with asynchronous multi-spin coding: replicas in groups of
    word_bits (32 or 64) share their random numbers (see smc_msc_sweep); beta is
    a host sequence [n_rep], equal within each group."""
    d = _desc(batch, spins, couplings)
    b = np.ascontiguousarray(np.broadcast_to(np.asarray(beta, np.float64), (batch.n_rep,)))
    _check(lib().smc_msc_sweep(C.byref(d), _ptr(spins), _ptr(couplings), b.ctypes.data_as(C.POINTER(C.c_double)),
                               sweep0, n_sweeps, word_bits, _ptr(dE_accum), _stream(stream)), "smc_msc_sweep")


def dcb_sweep(batch: Batch, spins, beta, sweep0: int, n_sweeps: int, tile: int, hits: int, palindromic=False,
              couplings=None, dE_accum=None, dE_trace=None, stream=None):
    """n_sweeps double-checkerboard sweeps (tile x tile tiles, `hits` hits per
    tile and sweep; see smc_dcb_sweep); beta is a host sequence [n_rep];
    dE_trace, if given, is an int64 device tensor of n_sweeps * n_rep entries."""
    d = _desc(batch, spins, couplings)
    b = np.ascontiguousarray(np.broadcast_to(np.asarray(beta, np.float64), (batch.n_rep,)))
    if dE_trace is not None:
        import torch

        if dE_trace.dtype != torch.int64 or not dE_trace.is_cuda or not dE_trace.is_contiguous():
            raise TypeError("dE_trace must be a contiguous int64 device tensor")
        if dE_trace.numel() < n_sweeps * batch.n_rep:
            raise ValueError(f"dE_trace holds {dE_trace.numel()} entries, needs n_sweeps * n_rep = "
                             f"{n_sweeps * batch.n_rep}")
    _check(lib().smc_dcb_sweep(C.byref(d), _ptr(spins), _ptr(couplings), b.ctypes.data_as(C.POINTER(C.c_double)),
                               sweep0, n_sweeps, tile, hits, 1 if palindromic else 0, _ptr(dE_accum),
                               _ptr(dE_trace), _stream(stream)), "smc_dcb_sweep")


HEIS_FLOAT, HEIS_FAST, HEIS_DOUBLE = 0, 1, 2


def heis_dcb_sweep(batch: Batch, spins, beta, sweep0: int, n_sweeps: int, tile: int, hits: int,
                   precision: int = HEIS_FAST, palindromic=False, cap: float = 0.0, accepts=None, stream=None):
    """n_sweeps double-checkerboard sweeps of a 2D Heisenberg batch (see
    smc_heis_dcb_sweep); spins float32 [n_rep*N*3] (float64 for HEIS_DOUBLE);
    cap > 0 selects small-step proposals."""
    import torch

    want = torch.float64 if precision == HEIS_DOUBLE else torch.float32
    if spins.dtype != want or not spins.is_cuda or not spins.is_contiguous():
        raise TypeError(f"spins must be a contiguous {want} device tensor for precision {precision}")
    d = _desc(batch, spins, None)
    b = np.ascontiguousarray(np.broadcast_to(np.asarray(beta, np.float64), (batch.n_rep,)))
    _check(lib().smc_heis_dcb_sweep(C.byref(d), _ptr(spins), b.ctypes.data_as(C.POINTER(C.c_double)), sweep0,
                                    n_sweeps, tile, hits, precision, 1 if palindromic else 0, float(cap),
                                    _ptr(accepts), _stream(stream)), "smc_heis_dcb_sweep")


def autotune(batch: Batch, cache_path=None, stream=None):
    """Measure the launch shapes of the batch's 2D kernels (see smc_autotune);
    cache_path: a text file read before and written after tuning, or None."""
    d = batch.desc(batch.spins_shape()[0], batch.coup_len())
    path = None if cache_path is None else os.fsencode(cache_path)
    _check(lib().smc_autotune(C.byref(d), path, _stream(stream)), "smc_autotune")


def dcb_plan(batch: Batch, beta, tile: int) -> str:
    """Name of the kernel smc_dcb_sweep uses for this batch, beta and tile (aligned buffers)."""
    d = batch.desc(batch.spins_shape()[0], batch.coup_len())
    b = np.ascontiguousarray(np.broadcast_to(np.asarray(beta, np.float64), (batch.n_rep,)))
    name = C.c_char_p()
    _check(lib().smc_dcb_plan(C.byref(d), b.ctypes.data_as(C.POINTER(C.c_double)), tile, C.byref(name)),
           "smc_dcb_plan")
    return name.value.decode()


def msc_plan(batch: Batch, n_sweeps: int, word_bits: int = 32):
    """(sweep-kernel launches, kernel name) that smc_msc_sweep uses for n_sweeps sweeps."""
    d = batch.desc(batch.spins_shape()[0], batch.coup_len())
    n = C.c_int32(0)
    name = C.c_char_p()
    _check(lib().smc_msc_plan(C.byref(d), n_sweeps, word_bits, C.byref(n), C.byref(name)), "smc_msc_plan")
    return int(n.value), name.value.decode()


def pt_sweep_swap(batch: Batch, n_chains: int, n_temps: int, beta, spins, slot_of_temp, energy, step0: int,
                  n_steps: int, couplings=None, swap_accepts=None, beta_per_chain: bool = False,
                  sweeps_per_step: int = 1, stream=None):
    """n_steps parallel-tempering steps (sweeps_per_step sweeps, then an exchange
    round); beta is host [n_temps] (or [n_chains, n_temps] with beta_per_chain)."""
    d = _desc(batch, spins, couplings)
    b = np.ascontiguousarray(np.asarray(beta, np.float64).reshape(-1))
    pt = PTDesc(n_chains, n_temps, 1 if beta_per_chain else 0, sweeps_per_step,
                b.ctypes.data_as(C.POINTER(C.c_double)))
    _check(lib().smc_pt_sweep_swap(C.byref(d), C.byref(pt), _ptr(spins), _ptr(couplings), _ptr(slot_of_temp),
                                   _ptr(energy), step0, n_steps, _ptr(swap_accepts), _stream(stream)),
           "smc_pt_sweep_swap")


def measure_energy_magnetisation(batch: Batch, spins, energy, magnetisation=None, couplings=None, stream=None):
    """Energy and magnetisation of every replica into float64 device tensors."""
    d = _desc(batch, spins, couplings)
    _check(lib().smc_measure_energy_magnetisation(C.byref(d), _ptr(spins), _ptr(couplings), _ptr(energy),
                                                  _ptr(magnetisation), _stream(stream)),
           "smc_measure_energy_magnetisation")


def measure_energy_magnetisation_noalloc(batch: Batch, spins, energy, magnetisation=None, couplings=None,
                                        stream=None):
    """As measure_energy_magnetisation, with the library's fixed device array
    for the partial sums (no allocation; uniform batches, bounded size)."""
    d = _desc(batch, spins, couplings)
    _check(lib().smc_measure_energy_magnetisation_noalloc(C.byref(d), _ptr(spins), _ptr(couplings), _ptr(energy),
                                                          _ptr(magnetisation), _stream(stream)),
           "smc_measure_energy_magnetisation_noalloc")


# Generators of the random-number study (smc_rng_generator).
RNG_LCG32, RNG_LCG32_RANDOM, RNG_LCG64, RNG_LCG64_RANDOM, RNG_FIB521, RNG_FIB1279 = 1, 2, 3, 4, 5, 6


def rng_study_state_bytes(batch: Batch, tile: int, generator: int) -> int:
    """Bytes of generator state the study needs for this batch (smc_rng_study_state_bytes)."""
    d = batch.desc(batch.spins_shape()[0], batch.coup_len())
    n = C.c_int64(0)
    _check(lib().smc_rng_study_state_bytes(C.byref(d), tile, generator, C.byref(n)), "smc_rng_study_state_bytes")
    return int(n.value)


def rng_study_init(batch: Batch, tile: int, generator: int, state, stream=None):
    """Seed a study generator's state (a device tensor of rng_study_state_bytes bytes)."""
    d = batch.desc(batch.spins_shape()[0], batch.coup_len())
    _check(lib().smc_rng_study_init(C.byref(d), tile, generator, _ptr(state), state.numel() * state.element_size(),
                                    _stream(stream)), "smc_rng_study_init")


def rng_study_sweep(batch: Batch, spins, beta, n_sweeps: int, tile: int, hits: int, generator: int, state,
                    couplings=None, dE_accum=None, stream=None):
    """n_sweeps double-checkerboard sweeps drawing from a study generator (smc_rng_study_sweep)."""
    d = _desc(batch, spins, couplings)
    b = np.ascontiguousarray(np.broadcast_to(np.asarray(beta, np.float64), (batch.n_rep,)))
    _check(lib().smc_rng_study_sweep(C.byref(d), _ptr(spins), _ptr(couplings), b.ctypes.data_as(C.POINTER(C.c_double)),
                                     n_sweeps, tile, hits, generator, _ptr(state),
                                     state.numel() * state.element_size(), _ptr(dE_accum), _stream(stream)),
           "smc_rng_study_sweep")


def sweep_plan(batch: Batch):
    """(launches per sweep, sweep kernel name) that smc_metropolis_sweep uses for this batch."""
    spins_len = batch.spins_shape()[0]
    d = batch.desc(spins_len, batch.coup_len())
    n = C.c_int32(0)
    name = C.c_char_p()
    _check(lib().smc_sweep_plan(C.byref(d), C.byref(n), C.byref(name)), "smc_sweep_plan")
    return int(n.value), name.value.decode()


def pt_plan(batch: Batch, n_chains: int, n_temps: int, beta, n_steps: int, beta_per_chain: bool = False,
            sweeps_per_step: int = 1):
    """(kernel launches, sweep kernel name) that smc_pt_sweep_swap uses for a call of n_steps steps."""
    spins_len = batch.spins_shape()[0]
    d = batch.desc(spins_len, batch.coup_len())
    b = np.ascontiguousarray(np.asarray(beta, np.float64).reshape(-1))
    pt = PTDesc(n_chains, n_temps, 1 if beta_per_chain else 0, sweeps_per_step,
                b.ctypes.data_as(C.POINTER(C.c_double)))
    n = C.c_int32(0)
    name = C.c_char_p()
    _check(lib().smc_pt_plan(C.byref(d), C.byref(pt), n_steps, C.byref(n), C.byref(name)), "smc_pt_plan")
    return int(n.value), name.value.decode()


def launches_per_sweep(batch: Batch) -> int:
    return sweep_plan(batch)[0]


def sweep_kernel_name(batch: Batch) -> str:
    return sweep_plan(batch)[1]


def kernel_timing_enable(on: bool = True):
    """Bracket the sweep kernels of each smc_metropolis_sweep call with HIP events (profiling aid)."""
    _check(lib().smc_kernel_timing_enable(1 if on else 0), "smc_kernel_timing_enable")


def philox_bench(seed: int, t: int, r: int, tag: int, out, per_thread: int, stream=None):
    """Generator throughput probe: out[i] (uint32 tensor, n_threads entries, given
    as int32) = XOR of the words of blocks (i + k*n_threads, t, r, tag), k < per_thread."""
    import torch

    if out.dtype != torch.int32 or not out.is_cuda or not out.is_contiguous():
        raise TypeError("out must be a contiguous int32 device tensor")
    _check(lib().smc_philox_bench(seed, t, r, tag, out.numel(), per_thread, _ptr(out), _stream(stream)),
           "smc_philox_bench")


def kernel_timing_read():
    """(elapsed ms, sweep-kernel launches) summed over the calls since the last read."""
    ms = C.c_double(0.0)
    n = C.c_int64(0)
    _check(lib().smc_kernel_timing_read(C.byref(ms), C.byref(n)), "smc_kernel_timing_read")
    return float(ms.value), int(n.value)
