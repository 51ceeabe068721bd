"""The reading of asynchronous multi-spin coding (Sec. 5): the replicas of a
group of 32 share their Metropolis draws, the counters carrying the group
index.  Each replica is then still an exact Metropolis chain of its own
couplings (the paper argues that the shared random numbers leave
disorder averages unbiased); these tests check that on the oracle."""
import math

import numpy as np

from oracle import exact as X
from oracle import oracle as O
import workloads as W

SEED = W.seed_for(61)


def test_group_members_with_equal_inputs_evolve_identically():
    """Same couplings and start: two replicas of one group stay identical;
    in different groups they part."""
    L = 8
    J = O.init_couplings(2, L, SEED, 5)
    s0 = O.init_spins(2, L, SEED, 5)
    a, b, c = s0.copy(), s0.copy(), s0.copy()
    O.run(2, L, J, a, 0.8, SEED, 3, 0, 40)   # group 3
    O.run(2, L, J, b, 0.8, SEED, 3, 0, 40)   # group 3 again
    O.run(2, L, J, c, 0.8, SEED, 4, 0, 40)   # group 4
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)


def test_shared_draws_keep_the_disorder_average():
    """4 x 4 +-J: four groups of 32 samples, each group on shared draws.  The
    replica- and time-averaged energy and its square match the averages of
    the enumerated values over the same samples, within 4.5 standard errors
    taken from the spread of the (independent) group means."""
    L, groups, sweeps, burn = 4, 4, 1500, 100
    for beta in (0.5, 1.0):
        dev_E, dev_E2 = [], []
        for g in range(groups):
            dE, dE2 = [], []
            for k in range(32):
                r = 32 * g + k
                J = O.init_couplings(2, L, SEED, r)
                E_all, M_all = X.enumerate_states(2, L, J)
                ex = X.boltzmann_averages(E_all, M_all, beta)
                s = O.init_spins(2, L, SEED, r)
                E, _ = O.run_series(2, L, J, s, beta, SEED, g, 0, sweeps)
                Ef = E[burn:].astype(np.float64)
                dE.append(Ef.mean() - ex["E"])
                dE2.append((Ef ** 2).mean() - ex["E2"])
            dev_E.append(np.mean(dE))
            dev_E2.append(np.mean(dE2))
        for dev in (np.array(dev_E), np.array(dev_E2)):
            err = dev.std(ddof=1) / math.sqrt(groups)
            assert abs(dev.mean()) < 4.5 * err + 1e-9, (beta, dev)
