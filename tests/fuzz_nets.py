"""Seeded random networks for the fuzz tests: random size, a spanning tree
plus extra edges, transformers with taps and phase shifts, parallel
branches, an out-of-service branch, shunts, and extra loads (also at PV and
slack buses).  Only network generation; no evaluation arithmetic."""

import numpy as np

from paper_2011_11880_amd import synth


def random_net(seed):
    rng = np.random.default_rng(10_000 + seed)
    n_bus = int(rng.integers(2, 7)) if rng.random() < 0.2 else int(rng.integers(7, 90))
    max_extra = n_bus * (n_bus - 1) // 2 - (n_bus - 1)
    n_branch = n_bus - 1 + int(min(rng.integers(0, n_bus), max_extra))
    n_pv = int(min(rng.integers(0, max(2, n_bus // 3)), n_bus - 1))
    n_shunt = int(rng.integers(0, n_bus // 4 + 1))
    net = synth.tiny_grid(seed, n_bus=n_bus, n_branch=n_branch, n_pv=n_pv, n_shunt=n_shunt)
    if rng.random() < 0.7:
        net = synth.with_parallel_branches(net, int(min(rng.integers(1, 4), n_branch)), seed)
    nb = synth.non_bridge_branches(net)
    if nb.size and rng.random() < 0.5:
        net = net.copy()
        net.br_status[int(rng.choice(nb))] = 0
    if rng.random() < 0.6:
        k = int(rng.integers(1, 6))
        extra = rng.integers(0, n_bus, k).astype(np.int32)
        net = net.copy()
        net.load_bus = np.concatenate([net.load_bus, extra]).astype(np.int32)
        net.load_p = np.concatenate([net.load_p, rng.uniform(-0.5, 1.0, k)])
        net.load_q = np.concatenate([net.load_q, rng.uniform(-0.3, 0.5, k)])
    return net
