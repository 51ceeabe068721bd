"""C-ABI contract checks that need no GPU: the library loads, exports every
function the header declares, and rejects invalid arguments before it
touches the device."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1101_1427_amd as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spinmc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(smc_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for f in ("smc_spin_init", "smc_metropolis_sweep", "smc_pt_sweep_swap", "smc_measure_energy_magnetisation",
              "smc_strerror", "smc_last_error"):
        assert f in names


def test_library_exports_every_declared_symbol():
    lib = C.CDLL(S.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_strerror():
    L = S.lib()
    assert L.smc_strerror(0) == b"success"
    assert L.smc_strerror(-1) == b"invalid argument"
    assert L.smc_strerror(-3) == b"HIP runtime error"
    assert L.smc_strerror(12345) == b"unknown status"


FAKE = C.c_void_p(0x1000)  # never dereferenced: validation fails first


def _desc(**kw):
    base = dict(model=S.ISING, dim=2, L=16, n_rep=1, rep_per_sample=1, renorm_every=0, seed=1, inst=None,
                spins_len=256, coup_len=0)
    base.update(kw)
    return S.Desc(**base)


def _sweep(d, n=1, beta=0.4, spins=FAKE, coup=None, sweep0=0):
    b = (C.c_double * max(1, d.n_rep))(*([beta] * max(1, d.n_rep)))
    return S.lib().smc_metropolis_sweep(C.byref(d), spins, coup, b, sweep0, n, None, None)


@pytest.mark.parametrize("kw,frag", [
    (dict(L=15), b"even"), (dict(L=2), b"even"), (dict(dim=4), b"dim"), (dict(model=7), b"model"),
    (dict(n_rep=0), b"n_rep"), (dict(spins_len=255), b"too small"), (dict(L=0), b"inst"),
    (dict(model=S.EA, rep_per_sample=0, coup_len=512), b"rep_per_sample"),
    (dict(model=S.EA, coup_len=0), b"coup_len"), (dict(model=S.EA, coup_len=511), b"outside"),
    (dict(dim=3, L=2048, spins_len=1 << 40), b"too large"),
])
def test_invalid_descriptors_are_rejected(kw, frag):
    rc = _sweep(_desc(**kw), coup=FAKE)
    assert rc == S.EINVAL
    assert frag in S.lib().smc_last_error()


def test_invalid_call_arguments_are_rejected():
    L = S.lib()
    assert _sweep(_desc(), spins=None) == S.EINVAL
    assert _sweep(_desc(), n=-1) == S.EINVAL
    assert _sweep(_desc(), beta=-0.1) == S.EINVAL
    assert _sweep(_desc(), beta=float("nan")) == S.EINVAL
    assert _sweep(_desc(), sweep0=(1 << 32) - 1, n=2) == S.EINVAL
    assert _sweep(_desc(model=S.EA, coup_len=512), coup=None) == S.EINVAL
    assert L.smc_metropolis_sweep(None, FAKE, None, None, 0, 1, None, None) == S.EINVAL


def test_uneven_batch_bounds_are_checked():
    rows = (S.Inst * 2)(S.Inst(8, 0, 0, 0), S.Inst(6, 1, 64, 0))
    d = _desc(L=0, n_rep=2, spins_len=64 + 35)
    d.inst = C.cast(rows, C.POINTER(S.Inst))
    assert _sweep(d) == S.EINVAL and b"outside" in S.lib().smc_last_error()
    rows[1] = S.Inst(7, 1, 64, 0)
    d.spins_len = 200
    assert _sweep(d) == S.EINVAL and b"even" in S.lib().smc_last_error()


def test_pt_arguments_are_validated():
    L = S.lib()
    beta = (C.c_double * 4)(0.1, 0.2, 0.3, 0.4)
    d = _desc(n_rep=6, spins_len=6 * 256)
    pt = S.PTDesc(2, 4, 0, 0, C.cast(beta, C.POINTER(C.c_double)))
    rc = L.smc_pt_sweep_swap(C.byref(d), C.byref(pt), FAKE, None, FAKE, FAKE, 0, 1, None, None)
    assert rc == S.EINVAL and b"n_chains * n_temps" in L.smc_last_error()
    d = _desc(n_rep=8, spins_len=8 * 256, model=S.HEISENBERG)
    d.spins_len = 8 * 256 * 3
    rc = L.smc_pt_sweep_swap(C.byref(d), C.byref(pt), FAKE, None, FAKE, FAKE, 0, 1, None, None)
    assert rc == S.EUNSUPPORTED
    d = _desc(n_rep=8, spins_len=8 * 256, model=S.EA, rep_per_sample=2, coup_len=8 * 512)
    rc = L.smc_pt_sweep_swap(C.byref(d), C.byref(pt), FAKE, FAKE, FAKE, FAKE, 0, 1, None, None)
    assert rc == S.EINVAL and b"multiple of n_temps" in L.smc_last_error()


def test_binding_has_no_cpu_fallback():
    """The product binding does not import the oracle."""
    src = open(os.path.join(ROOT, "paper_1101_1427_amd", "__init__.py")).read()
    assert "oracle" not in src.replace("oracle (", "")
    for f in os.listdir(os.path.join(ROOT, "paper_1101_1427_amd", "csrc")):
        assert "oracle" not in open(os.path.join(ROOT, "paper_1101_1427_amd", "csrc", f)).read().lower()


def test_kernel_timing_without_calls_reads_zero():
    S.kernel_timing_enable(True)
    assert S.kernel_timing_read() == (0.0, 0)
    S.kernel_timing_enable(False)
    assert S.kernel_timing_read() == (0.0, 0)


def test_philox_bench_arguments_are_validated():
    L = S.lib()
    assert L.smc_philox_bench(1, 0, 0, 0, 16, 4, None, None) == S.EINVAL
    assert L.smc_philox_bench(1, 0, 0, 0, 0, 4, FAKE, None) == S.EINVAL
    assert L.smc_philox_bench(1, 0, 0, 0, 16, 0, FAKE, None) == S.EINVAL
    rc = L.smc_philox_bench(1, 0, 0, 0, 1 << 20, 1 << 13, FAKE, None)
    assert rc == S.EINVAL and b"2^32" in L.smc_last_error()


def test_msc_arguments_are_validated():
    L = S.lib()
    beta = (C.c_double * 128)(*([0.5] * 128))
    d = _desc(n_rep=48, spins_len=48 * 256)
    rc = L.smc_msc_sweep(C.byref(d), FAKE, None, beta, 0, 1, 32, None, None)
    assert rc == S.EINVAL and b"multiple of 32" in L.smc_last_error()
    d = _desc(n_rep=96, spins_len=96 * 256)
    rc = L.smc_msc_sweep(C.byref(d), FAKE, None, beta, 0, 1, 64, None, None)
    assert rc == S.EINVAL and b"multiple of 64" in L.smc_last_error()
    rc = L.smc_msc_sweep(C.byref(d), FAKE, None, beta, 0, 1, 16, None, None)
    assert rc == S.EINVAL and b"word_bits" in L.smc_last_error()
    d = _desc(n_rep=64, spins_len=64 * 256, model=S.EA, coup_len=64 * 512)
    d.rep_per_sample = 2
    rc = L.smc_msc_sweep(C.byref(d), FAKE, FAKE, beta, 0, 1, 32, None, None)
    assert rc == S.EINVAL and b"rep_per_sample" in L.smc_last_error()
    d.rep_per_sample = 1
    beta2 = (C.c_double * 64)(*([0.5] * 40 + [0.6] * 24))
    rc = L.smc_msc_sweep(C.byref(d), FAKE, FAKE, beta2, 0, 1, 32, None, None)
    assert rc == S.EINVAL and b"group of 32" in L.smc_last_error()
    beta3 = (C.c_double * 64)(*([0.5] * 32 + [0.6] * 32))
    rc = L.smc_msc_sweep(C.byref(d), FAKE, FAKE, beta3, 0, 1, 64, None, None)
    assert rc == S.EINVAL and b"group of 64" in L.smc_last_error()
    d = _desc(n_rep=64, spins_len=64 * 256 * 3, model=S.HEISENBERG)
    assert L.smc_msc_sweep(C.byref(d), FAKE, None, beta, 0, 1, 32, None, None) == S.EUNSUPPORTED


def test_dcb_arguments_are_validated():
    L = S.lib()
    beta = (C.c_double * 2)(0.5, 0.5)
    d = _desc(L=64, n_rep=2, spins_len=2 * 64 * 64)
    for tile, frag in ((24, b"multiple of 16"), (48, b"multiple of 16"), (256, b"multiple of 16")):
        rc = L.smc_dcb_sweep(C.byref(d), FAKE, None, beta, 0, 1, tile, 1, 0, None, None, None)
        assert rc == S.EINVAL and frag in L.smc_last_error()
    assert L.smc_dcb_sweep(C.byref(d), FAKE, None, beta, 0, 1, 32, 0, 0, None, None, None) == S.EINVAL
    rc = L.smc_dcb_sweep(C.byref(d), FAKE, None, beta, (1 << 31), 1, 32, 2, 0, None, None, None)
    assert rc == S.EINVAL and b"2^32" in L.smc_last_error()
    d3 = _desc(dim=3, L=32, n_rep=1, spins_len=32 ** 3)
    rc = L.smc_dcb_sweep(C.byref(d3), FAKE, None, beta, 0, 1, 32, 1, 0, None, None, None)
    assert rc == S.EINVAL and b"16 x 16 x 16" in L.smc_last_error()
    d3 = _desc(dim=3, L=32, n_rep=1, spins_len=32 ** 3)
    rc = L.smc_dcb_sweep(C.byref(d3), C.c_void_p(FAKE.value + 1), None, beta, 0, 1, 16, 1, 0, None, None, None)
    assert rc == S.EINVAL and b"16-byte aligned" in L.smc_last_error()
    d3 = _desc(dim=3, L=48, n_rep=1, spins_len=48 ** 3)
    assert L.smc_dcb_sweep(C.byref(d3), FAKE, None, beta, 0, 1, 16, 1, 0, None, None, None) == S.EINVAL
    # only the pointers the kernel reads must be aligned: an Ising call ignores
    # its couplings argument (a zero-sweep call returns after the checks)
    d3 = _desc(dim=3, L=32, n_rep=1, spins_len=32 ** 3)
    unaligned = C.c_void_p(FAKE.value + 3)
    assert L.smc_dcb_sweep(C.byref(d3), FAKE, unaligned, beta, 0, 0, 16, 1, 0, None, None, None) == S.OK
    d3ea = _desc(model=S.EA, dim=3, L=32, n_rep=1, spins_len=32 ** 3, coup_len=3 * 32 ** 3)
    rc = L.smc_dcb_sweep(C.byref(d3ea), FAKE, unaligned, beta, 0, 0, 16, 1, 0, None, None, None)
    assert rc == S.EINVAL and b"16-byte aligned" in L.smc_last_error()
    dh = _desc(model=S.HEISENBERG, dim=3, L=32, n_rep=1, spins_len=3 * 32 ** 3)
    assert L.smc_dcb_sweep(C.byref(dh), FAKE, None, beta, 0, 1, 16, 1, 0, None, None, None) == S.EUNSUPPORTED


def test_dcb_plan_names_the_kernel():
    """smc_dcb_plan: the packed kernel for power-of-two tiles and beta > 0,
    the per-site kernel for other tiles or a replica at beta = 0."""
    L = S.lib()
    name = C.c_char_p()
    d = _desc(L=96, n_rep=2, spins_len=2 * 96 * 96)
    beta = (C.c_double * 2)(0.4, 0.5)
    assert L.smc_dcb_plan(C.byref(d), beta, 48, C.byref(name)) == S.OK and name.value == b"k_dcb2d"
    d = _desc(L=128, n_rep=2, spins_len=2 * 128 * 128)
    for tile in (16, 32, 64, 128):
        assert L.smc_dcb_plan(C.byref(d), beta, tile, C.byref(name)) == S.OK and name.value == b"k_dcb2d_packed"
    beta0 = (C.c_double * 2)(0.4, 0.0)
    assert L.smc_dcb_plan(C.byref(d), beta0, 64, C.byref(name)) == S.OK and name.value == b"k_dcb2d"
    assert L.smc_dcb_plan(C.byref(d), beta, 24, C.byref(name)) == S.EINVAL
    assert L.smc_dcb_plan(C.byref(d), None, 64, C.byref(name)) == S.EINVAL


def test_heis_dcb_arguments_are_validated():
    L = S.lib()
    beta = (C.c_double * 2)(0.5, 0.5)
    d = _desc(model=S.HEISENBERG, L=64, n_rep=2, spins_len=2 * 64 * 64 * 3)
    call = lambda tile, hits, prec, dd=d, sp=FAKE, cap=0.0: L.smc_heis_dcb_sweep(C.byref(dd), sp, beta, 0, 1, tile,
                                                                                  hits, prec, 0, cap, None, None)
    assert call(48, 1, S.HEIS_FAST) == S.EINVAL
    assert call(64, 1, S.HEIS_DOUBLE) == S.EINVAL and b"float modes" in L.smc_last_error()
    assert call(32, 0, S.HEIS_FLOAT) == S.EINVAL
    assert call(32, 1, 3) == S.EINVAL and b"precision" in L.smc_last_error()
    assert call(32, 1, S.HEIS_FAST, cap=2.5) == S.EINVAL and b"cap" in L.smc_last_error()
    assert call(32, 1, S.HEIS_FAST, cap=-0.1) == S.EINVAL
    assert call(32, 1, S.HEIS_FAST, sp=C.c_void_p(FAKE.value + 4)) == S.EINVAL
    assert b"aligned" in L.smc_last_error()
    di = _desc(L=64, n_rep=2, spins_len=2 * 64 * 64)
    assert call(32, 1, S.HEIS_FAST, dd=di) == S.EUNSUPPORTED
    d3 = _desc(model=S.HEISENBERG, dim=3, L=32, n_rep=1, spins_len=3 * 32 ** 3)
    assert call(16, 1, S.HEIS_FAST, dd=d3) == S.EUNSUPPORTED


def test_autotune_has_nothing_to_tune_for_other_batches(tmp_path):
    """Batches none of whose kernels has a launch shape to tune (Heisenberg,
    edges that take the generic kernels, the 2D Ising edge 1000 between the
    LDS-resident and the one-pass kernels): SMC_OK, no device work, no file."""
    L = S.lib()
    path = str(tmp_path / "tune.txt").encode()
    for d in (_desc(dim=3, L=20, n_rep=2, spins_len=2 * 20 ** 3),
              _desc(model=S.HEISENBERG, L=32, n_rep=1, spins_len=3 * 32 * 32),
              _desc(model=S.HEISENBERG, dim=3, L=64, n_rep=1, spins_len=3 * 64 ** 3),
              _desc(L=1000, n_rep=1, spins_len=1000 * 1000)):
        assert L.smc_autotune(C.byref(d), path, None) == S.OK
    assert not (tmp_path / "tune.txt").exists()
    assert L.smc_autotune(None, path, None) == S.EINVAL


def test_sweep_plan_names_the_3d_kernel(monkeypatch):
    """smc_sweep_plan: uniform 3D Ising / EA batches with an edge that is a
    multiple of 16 take the one-pass segment sweep (edges 512 .. 1024 by
    default, 32 .. 1024 with SPINMC_SWEEP3D_PASS=1; one launch) or the
    segment half-sweeps (smaller edges, or SPINMC_SWEEP3D_PASS=0); other
    edges, Heisenberg batches and SPINMC_SWEEP3D=0 the generic kernels."""
    for model, L, want in ((S.ISING, 16, (2, "k_ising3d_half")), (S.EA, 48, (2, "k_ising3d_half")),
                           (S.ISING, 256, (2, "k_ising3d_half")), (S.EA, 512, (1, "k_ising3d_pass")),
                           (S.ISING, 1024, (1, "k_ising3d_pass")),
                           (S.ISING, 20, (2, "k_half_sweep_generic")), (S.EA, 8, (2, "k_half_sweep_generic"))):
        assert S.sweep_plan(S.Batch(model, 3, L, 2, 1)) == want
    assert S.sweep_plan(S.Batch(S.HEISENBERG, 3, 32, 1, 1))[1] not in ("k_ising3d_half", "k_ising3d_pass")
    monkeypatch.setenv("SPINMC_SWEEP3D_PASS", "1")
    assert S.sweep_plan(S.Batch(S.EA, 3, 48, 2, 1)) == (1, "k_ising3d_pass")
    assert S.sweep_plan(S.Batch(S.ISING, 3, 16, 2, 1)) == (2, "k_ising3d_half")
    monkeypatch.setenv("SPINMC_SWEEP3D_PASS", "0")
    assert S.sweep_plan(S.Batch(S.EA, 3, 48, 2, 1)) == (2, "k_ising3d_half")
    assert S.sweep_plan(S.Batch(S.ISING, 3, 1024, 1, 1)) == (2, "k_ising3d_half")
    monkeypatch.setenv("SPINMC_SWEEP3D", "0")
    assert S.sweep_plan(S.Batch(S.ISING, 3, 64, 1, 1)) == (2, "k_half_sweep_generic")


def test_noalloc_measure_checks_before_any_device_work():
    """The allocation-free measurement refuses uneven batches and batches whose
    partial sums exceed its fixed 16 MiB array, on the host."""
    L = S.lib()
    d = _desc(L=16384, n_rep=257, spins_len=257 * 16384 * 16384)  # 257 x 2048 partials x 32 B > 16 MiB
    rc = L.smc_measure_energy_magnetisation_noalloc(C.byref(d), FAKE, None, FAKE, None, None)
    assert rc == S.EINVAL and b"16777216" in L.smc_last_error()
    inst = (S.Inst * 2)(S.Inst(16, 0, 0, 0), S.Inst(32, 0, 256, 0))
    d = _desc(L=0, n_rep=2, inst=C.cast(inst, C.POINTER(S.Inst)), spins_len=256 + 1024)
    assert L.smc_measure_energy_magnetisation_noalloc(C.byref(d), FAKE, None, FAKE, None, None) == S.EUNSUPPORTED
