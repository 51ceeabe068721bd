"""Calls on a stream that is capturing a graph are refused before anything is
issued (they stage host tables and may grow scratch, which a capture cannot
record); the same calls outside the capture run normally."""
import pytest

import paper_1101_1427_amd as S
import workloads as W

pytestmark = pytest.mark.gpu


def test_captured_calls_are_refused_and_leave_the_state_alone():
    import torch

    dev = torch.device("cuda:0")
    b = S.Batch(S.ISING, 2, 64, 2, W.seed_for(71))
    spins = torch.zeros(2 * 64 * 64, dtype=torch.int8, device=dev)
    E = torch.zeros(2, dtype=torch.float64, device=dev)
    S.spin_init(b, spins)
    torch.cuda.synchronize()
    before = spins.clone()
    calls = {
        "smc_metropolis_sweep": lambda: S.metropolis_sweep(b, spins, [0.4, 0.4], 0, 3),
        "smc_measure_energy_magnetisation": lambda: S.measure_energy_magnetisation(b, spins, E),
        "smc_spin_init": lambda: S.spin_init(b, spins),
    }
    errors = {}
    side = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        for name, call in calls.items():
            try:
                call()
            except S.SpinMCError as e:
                errors[name] = str(e)
    torch.cuda.synchronize()
    assert set(errors) == set(calls), errors
    assert all("capturing" in msg for msg in errors.values()), errors
    assert torch.equal(spins, before)
    S.metropolis_sweep(b, spins, [0.4, 0.4], 0, 3)
    S.measure_energy_magnetisation(b, spins, E)
    torch.cuda.synchronize()
    assert not torch.equal(spins, before)
