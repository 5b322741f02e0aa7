"""Host side over seeded random networks (no GPU): every network sets up,
its pattern has the size the formula gives, and equals the oracle's
Jacobian structure (with and without Q_g slots)."""

import numpy as np
import pytest
import scipy.sparse as sp

from fuzz_nets import random_net
from paper_2011_11880_amd import synth
from paper_2011_11880_amd.api import Plan


@pytest.mark.parametrize("seed", range(40))
def test_random_network_pattern(ora, seed):
    net = random_net(seed)
    p = Plan(net, host_only=True)
    assert p.n == net.n_var
    rp, ci = p.pattern()
    assert rp[0] == 0 and rp[-1] == p.nnz and np.all(np.diff(rp) > 0)
    for r in range(p.n):
        assert np.all(np.diff(ci[rp[r]:rp[r + 1]]) > 0)   # sorted, no duplicates
    y = synth.random_states(net, seed=seed)
    Jo, _ = ora.jacobian(net, y)
    S = sp.csr_matrix((np.ones(Jo.nnz), Jo.indices, Jo.indptr), shape=Jo.shape)
    S.sum_duplicates()
    S.sort_indices()
    assert np.array_equal(rp, S.indptr) and np.array_equal(ci, S.indices)
    pq = Plan(net, host_only=True, q_limits=True)
    assert pq.nnz == p.nnz + net.n_pv
