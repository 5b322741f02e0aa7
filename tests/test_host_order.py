"""The locality bus order of the setup (PF_ORDER_LOCALITY), host side: the
order is a breadth-first order over the in-service branches (from bus 0,
then from the lowest-numbered bus not yet reached), the plan equals the
input-order plan of the network renumbered that way, and malformed input is
reported as without the option.  CPU only."""

import numpy as np
import pytest

from paper_2011_11880_amd import capi, synth
from paper_2011_11880_amd.api import Plan
from paper_2011_11880_amd.capi import PFError


def _renumbered(net, order):
    pos = np.empty(net.n_bus, np.int64)
    pos[order] = np.arange(net.n_bus)
    n = net.copy()
    for a in ("br_from", "br_to", "load_bus", "pv_bus", "slack_bus", "shunt_bus"):
        setattr(n, a, pos[getattr(net, a)].astype(np.int32))
    n.coords = None
    return n


def _is_bfs_order(net, order):
    """Every bus is reached from an earlier one in the order, except the
    roots, and each root is the lowest-numbered bus not reached before it;
    positions of each bus's neighbours are what a queue would give."""
    N = net.n_bus
    on = net.br_status != 0
    nb = [[] for _ in range(N)]
    for a, b in zip(net.br_from[on].tolist(), net.br_to[on].tolist()):
        nb[a].append(b)
        nb[b].append(a)
    # replay a queue-based search and require the same sequence
    seen = np.zeros(N, bool)
    out = []
    for s in range(N):
        if seen[s]:
            continue
        seen[s] = True
        q = [s]
        h = 0
        while h < len(q):
            b = q[h]
            h += 1
            out.append(b)
            for c in nb[b]:
                if not seen[c]:
                    seen[c] = True
                    q.append(c)
    return np.array_equal(np.array(out), order)


@pytest.mark.parametrize("which", ["tiny", "70k", "parallel and out of service"])
def test_locality_order_is_breadth_first_and_plan_is_renumbered_plan(which):
    net = {"tiny": lambda: synth.tiny_grid(3, n_shunt=5), "70k": synth.grid_70k,
           "parallel and out of service": lambda: _with_out_of_service()}[which]()
    p = Plan(net, host_only=True, bus_order="locality")
    order = p.bus_order()
    assert np.array_equal(np.sort(order), np.arange(net.n_bus))
    assert _is_bfs_order(net, order)
    q = Plan(_renumbered(net, order), host_only=True)
    rp, ci = p.pattern()
    rq, cq = q.pattern()
    assert np.array_equal(rp, rq) and np.array_equal(ci, cq)
    assert p.info == q.info
    # the input order is the identity
    assert np.array_equal(Plan(net, host_only=True).bus_order(), np.arange(net.n_bus))
    # state conversion round trip
    y = synth.random_states(net, seed=1)
    x = p.to_plan(y)
    assert np.array_equal(p.from_plan(x), y)
    assert np.array_equal(x[:net.n_bus], y[order]) and np.array_equal(x[2 * net.n_bus:],
                                                                       y[2 * net.n_bus:])


def _with_out_of_service():
    net = synth.with_parallel_branches(synth.tiny_grid(5, n_bus=120, n_branch=170, n_pv=12), 6, 2)
    net.br_status[int(synth.non_bridge_branches(net)[3])] = 0
    return net


def test_multi_grid_orders_each_grid():
    nets = [synth.tiny_grid(s, n_bus=40 + 30 * s, n_branch=55 + 40 * s, n_pv=6) for s in range(3)]
    p = Plan.multi(nets, host_only=True, bus_order="locality")
    order = p.bus_order()
    b0 = 0
    for net in nets:
        o = order[b0:b0 + net.n_bus]
        assert _is_bfs_order(net, o)
        b0 += net.n_bus
    q = Plan.multi([_renumbered(n, order[sum(m.n_bus for m in nets[:g]):][:n.n_bus])
                    for g, n in enumerate(nets)], host_only=True)
    assert np.array_equal(p.pattern()[1], q.pattern()[1])


def test_malformed_input_and_unknown_order():
    net = synth.tiny_grid(2)
    bad = net.copy()
    bad.br_to = bad.br_to.copy()
    bad.br_to[3] = net.n_bus + 5
    codes = []
    for order in ("input", "locality"):
        with pytest.raises(PFError) as ei:
            Plan(bad, host_only=True, bus_order=order)
        codes.append(ei.value.code)
    assert codes[0] == codes[1] == capi.PF_EINVAL
    from paper_2011_11880_amd.api import _NetStruct, _opts
    ns = _NetStruct(net)
    o = _opts(host_only=True)
    o.bus_order = 7
    h = capi._P()
    import ctypes
    assert capi.lib().pf_setup(ctypes.byref(ns.s), ctypes.byref(o), ctypes.byref(h)) == \
        capi.PF_EINVAL
