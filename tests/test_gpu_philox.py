"""GPU generator throughput probe against the oracle's Philox4x32-10: the
XOR of every block a thread draws, bit-exact."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1101_1427_amd as S
import workloads as W
from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n_threads,per_thread", [(300, 4), (257, 7), (64, 1), (1000, 9)])
def test_philox_bench_matches_the_oracle(n_threads, per_thread):
    seed, t, r, tag = W.seed_for(7), 11, 3, 2 * 3 + 1
    out = torch.zeros(n_threads, dtype=torch.int32, device="cuda")
    S.philox_bench(seed, t, r, tag, out, per_thread)
    torch.cuda.synchronize()
    got = out.cpu().numpy().view(np.uint32)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for i in range(n_threads):
        acc = 0
        for k in range(per_thread):
            w = O.philox([i + k * n_threads, t, r, tag], key)
            acc ^= int(w[0]) ^ int(w[1]) ^ int(w[2]) ^ int(w[3])
        assert int(got[i]) == acc, (i, n_threads, per_thread)
