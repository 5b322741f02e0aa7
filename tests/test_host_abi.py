"""Host-side checks of libpf through its C ABI (no GPU needed): symbols,
validation, the fixed Jacobian pattern and its sizes, multi-grid offsets
and schedules.  Plans are built with host_only=1."""

import os
import re

import numpy as np
import pytest

from paper_2011_11880_amd import capi, synth
from paper_2011_11880_amd.api import Plan
from paper_2011_11880_amd.capi import PFError

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "pf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pf_[a-z_]+)\s*\(", src)) - {"pf_linsolve_fn"})


def test_library_exports_every_declared_symbol():
    L = capi.lib()
    names = _declared()
    assert len(names) >= 18
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(capi.SIGNATURES), set(names) ^ set(capi.SIGNATURES)


def _plan(net, **kw):
    return Plan(net, host_only=True, **kw)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_pattern_matches_oracle(ora, seed):
    net = synth.with_parallel_branches(synth.tiny_grid(seed, n_shunt=6), 4, seed)
    p = _plan(net)
    y = synth.random_states(net, seed=seed)
    J, _ = ora.jacobian(net, y)
    rp, ci = p.pattern()
    assert p.n == net.n_var == J.shape[0]
    np.testing.assert_array_equal(rp, J.indptr)
    np.testing.assert_array_equal(ci, J.indices)
    B_u = len({(min(a, b), max(a, b)) for a, b in zip(net.br_from, net.br_to)})
    assert p.nnz == 4 * net.n_bus + 8 * B_u + 2 * net.n_gen + 2 * net.n_slack
    for r in range(p.n):
        assert np.all(np.diff(ci[rp[r]:rp[r + 1]]) > 0)


def test_config_sizes():
    p = _plan(synth.tiny_grid(0))
    assert (p.n, p.nnz) == (442, 3124)
    assert p.info["n_entries"] == 200 + 2 * 280


def test_out_of_service_branch_leaves_pattern():
    net = synth.tiny_grid(0)
    e = int(synth.non_bridge_branches(net)[0])
    p0 = _plan(net)
    p1 = _plan(net.without_branch(e))
    assert p0.nnz - p1.nnz == 8


def _expect(code, net, **kw):
    with pytest.raises(PFError) as ei:
        _plan(net, **kw)
    assert ei.value.code == code, str(ei.value)


def test_validation_errors():
    base = synth.tiny_grid(0)
    n = base.copy(); n.br_to[3] = n.br_from[3]
    _expect(capi.PF_ETOPO, n)
    n = base.copy(); n.br_to[3] = 10_000
    _expect(capi.PF_EINVAL, n)
    n = base.copy(); n.br_from[0] = -1
    _expect(capi.PF_EINVAL, n)
    n = base.copy(); n.br_tap[5] = 0.0
    _expect(capi.PF_EINVAL, n)
    n = base.copy(); n.br_tap[5] = -1.0
    _expect(capi.PF_EINVAL, n)
    n = base.copy(); n.br_r[7] = 0.0; n.br_x[7] = 0.0
    _expect(capi.PF_EINVAL, n)
    n = base.copy(); n.br_x[7] = np.nan
    _expect(capi.PF_EINVAL, n)
    n = base.copy(); n.pv_bus[1] = n.pv_bus[0]
    _expect(capi.PF_ETOPO, n)
    n = base.copy(); n.pv_bus[0] = n.slack_bus[0]
    _expect(capi.PF_ETOPO, n)
    n = base.copy(); n.load_p[2] = np.inf
    _expect(capi.PF_EINVAL, n)
    n = base.copy(); n.br_status[:] = 1; n.br_status[4] = 2
    _expect(capi.PF_EINVAL, n)
    # a bus whose only branch is out of service is isolated
    deg = np.bincount(np.concatenate([base.br_from, base.br_to]), minlength=base.n_bus)
    leaf = int(np.nonzero(deg == 1)[0][0])
    e = int(np.nonzero((base.br_from == leaf) | (base.br_to == leaf))[0][0])
    _expect(capi.PF_ETOPO, base.without_branch(e))


def test_single_bus_network():
    net = synth.Network(n_bus=1, br_from=[], br_to=[], br_r=[], br_x=[], br_b=[], br_tap=[],
                        br_shift_deg=[], br_status=[], load_bus=[], load_p=[], load_q=[],
                        pv_bus=[], pv_p=[], pv_v=[], slack_bus=[0], slack_v=[1.0],
                        slack_theta=[0.0], shunt_bus=[0], shunt_g=[0.1], shunt_b=[0.2])
    p = _plan(net)
    assert (p.n, p.nnz) == (4, 4 + 2 + 2)


def test_batch_spec_validation():
    net = synth.tiny_grid(0)
    with pytest.raises(PFError):
        _plan(net, batch=dict(n_inst=0))
    with pytest.raises(PFError):
        _plan(net, batch=dict(n_inst=2, outage=[0, net.n_branch]))
    e = int(synth.non_bridge_branches(net)[0])
    with pytest.raises(PFError):
        Plan(net.without_branch(e), host_only=True, batch=dict(n_inst=1, outage=[e]))
    ls = np.ones((3, net.n_load)); ls[1, 2] = np.nan
    with pytest.raises(PFError):
        _plan(net, batch=dict(n_inst=3, load_scale=ls))
    p = _plan(net, batch=dict(n_inst=3, outage=[-1, e, -1]))
    assert p.info["kind"] == "batch" and p.n_inst == 3 and p.ld == 3
    with pytest.raises(PFError):
        _plan(net, batch=dict(n_inst=3, inst_stride=2))
    assert _plan(net, batch=dict(n_inst=3, inst_stride=16)).ld == 16


def test_multi_grid_offsets(ora):
    nets = [synth.tiny_grid(s, n_bus=30 + 10 * s, n_branch=40 + 12 * s, n_pv=5) for s in range(4)]
    p = Plan.multi(nets, host_only=True)
    assert p.info["kind"] == "multi" and p.info["n_grids"] == 4
    rp, ci = p.pattern()
    for g, net in enumerate(nets):
        y = synth.random_states(net, seed=g)
        J, _ = ora.jacobian(net, y)
        x0, x1 = p.x_off[g], p.x_off[g + 1]
        assert x1 - x0 == net.n_var
        sub_rp = rp[x0:x1 + 1] - rp[x0]
        np.testing.assert_array_equal(sub_rp, J.indptr)
        np.testing.assert_array_equal(ci[rp[x0]:rp[x1]] - x0, J.indices)
        assert rp[x0] == p.j_off[g]


def test_schedule_roundtrip_and_tiles():
    net = synth.grid_10k()
    p = _plan(net)
    s = p.schedule
    assert s["tile_entries"] % 64 == 0
    p.schedule = dict(s, tile_entries=64)
    t64 = p.info["n_tiles"]
    p.schedule = dict(s, tile_entries=1024)
    assert p.info["n_tiles"] < t64
    with pytest.raises(PFError):
        p.schedule = dict(s, tile_entries=100)
    with pytest.raises(PFError):
        p.schedule = dict(s, waves_per_block=9)


def test_eval_on_host_only_plan_fails():
    p = _plan(synth.tiny_grid(0))
    L = capi.lib()
    rc = L.pf_eval(p._h, None, None, None, None)
    assert rc == capi.PF_EINVAL
