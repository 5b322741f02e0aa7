"""GPU parity of the batched kernel (pf_eval_batch): random states as
instances (bit-identical to the single-instance kernel), load/PV scenario
overlays and N-1 outages (against the oracle on the modified network),
ragged instance counts, residual-only and Jacobian-only launches, schedule
invariance, graph replay, every instance of the 10,000-bus x 1024-instance
batch against the oracle, and the benchmark's 70,000-bus x 1000-state launch
(every instance bit-identical to the single-instance kernel, a wide sample
against the oracle)."""

import numpy as np
import pytest

from paper_2011_11880_amd import synth
from parity import (check_close, check_jacobian, check_jacobian_triplets, pattern_keys,
                    triplet_positions)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _Plan():
    from paper_2011_11880_amd.api import Plan
    return Plan


def _net():
    net = synth.tiny_grid(4, n_bus=150, n_branch=210, n_pv=25, n_shunt=12)
    return synth.with_parallel_branches(net, 8, 3)


def _batch_eval(plan, Y, cuda):
    X = torch.from_numpy(np.ascontiguousarray(Y.T)).to(cuda)
    F, J = plan.eval_batch(X)
    torch.cuda.synchronize()
    return F.cpu().numpy(), J.cpu().numpy()


def _instance_net(net, spec, k):
    n = net.copy()
    if spec.get("load_scale") is not None:
        n.load_p = net.load_p * spec["load_scale"][k]
        n.load_q = net.load_q * spec["load_scale"][k]
    if spec.get("pv_scale") is not None:
        n.pv_p = net.pv_p * spec["pv_scale"][k]
    if spec.get("outage") is not None and spec["outage"][k] >= 0:
        n = n.without_branch(int(spec["outage"][k]))
    return n


@pytest.mark.parametrize("n_inst", [1, 63, 64, 65, 130])
def test_states_as_instances_bitwise_equal_single(cuda, n_inst):
    Plan = _Plan()
    net = _net()
    Y = synth.random_states(net, n_inst, seed=n_inst)
    bp = Plan(net, batch=dict(n_inst=n_inst))
    Fb, Jb = _batch_eval(bp, Y, cuda)
    sp = Plan(net)
    for k in sorted({0, n_inst // 2, n_inst - 1}):
        F, J = sp.eval(torch.from_numpy(Y[k]).to(cuda))
        torch.cuda.synchronize()
        assert np.array_equal(F.cpu().numpy(), Fb[:, k])
        assert np.array_equal(J.cpu().numpy(), Jb[:, k])


def test_scenarios_and_outages_vs_oracle(ora, cuda):
    Plan = _Plan()
    net = _net()
    I = 48
    ls, ps = synth.batch_scenarios(net, I, seed=5)
    cand = synth.non_bridge_branches(net)
    par = np.arange(net.n_branch - 8, net.n_branch)   # parallel branches
    out = np.full(I, -1, np.int32)
    out[16:] = np.concatenate([par[:4], cand[:I - 20]])[:I - 16]
    ls[16:24] = 1.0
    spec = dict(n_inst=I, load_scale=ls, pv_scale=ps, outage=out)
    bp = Plan(net, batch=spec)
    Y = synth.random_states(net, I, seed=6)
    Fb, Jb = _batch_eval(bp, Y, cuda)
    rp, ci = bp.pattern()
    for k in range(I):
        nk = _instance_net(net, spec, k)
        Fo, So = ora.residual(nk, Y[k])
        Jo, Ao = ora.jacobian(nk, Y[k])
        check_close(Fb[:, k], Fo, So, f"inst {k} F")
        check_jacobian(rp, ci, Jb[:, k], Jo, Ao, f"inst {k} J")


@pytest.mark.parametrize("overlay", [False, True])
def test_residual_only_and_jacobian_only_equal_fused(cuda, overlay):
    """The residual-only and Jacobian-only launches write exactly what the
    fused launch writes, without an overlay and with scenarios and outages,
    on a grid whose longest admittance rows need more than one group of
    four entries."""
    Plan = _Plan()
    net = _net()
    pairs = {(min(f, t), max(f, t)) for f, t in zip(net.br_from, net.br_to)}
    deg = np.bincount(np.array([b for p in pairs for b in p]), minlength=net.n_bus)
    assert deg.max() + 1 > 4
    I = 70
    spec = dict(n_inst=I)
    if overlay:
        ls, ps = synth.batch_scenarios(net, I, seed=8)
        out = np.full(I, -1, np.int32)
        out[35:] = synth.non_bridge_branches(net)[:I - 35]
        spec.update(load_scale=ls, pv_scale=ps, outage=out)
    bp = Plan(net, batch=spec)
    Y = synth.random_states(net, I, seed=9)
    X = torch.from_numpy(bp.to_batch(Y)).to(cuda)
    F0, J0 = bp.eval_batch(X)
    F1, none_j = bp.eval_batch(X, want_J=False)
    none_f, J1 = bp.eval_batch(X, want_F=False)
    torch.cuda.synchronize()
    assert none_j is None and none_f is None
    assert np.array_equal(bp.from_batch(F1), bp.from_batch(F0))
    assert np.array_equal(bp.from_batch(J1), bp.from_batch(J0))


@pytest.mark.parametrize("I,LD", [(70, 72), (70, 71), (69, 70), (130, 130)])
def test_lane_pairing_paths_equal_single(cuda, I, LD):
    """Without overlays, even instance counts and pitches take two instances
    per lane, odd ones one: both bit-identical to the single-instance kernel
    for every instance, under several schedules (residual-only and
    Jacobian-only launches included), padding columns untouched."""
    Plan = _Plan()
    net = _net()
    Y = synth.random_states(net, I, seed=I + LD)
    bp = Plan(net, batch=dict(n_inst=I, inst_stride=LD))
    Xp = np.full((net.n_var, LD), np.nan)
    Xp[:, :I] = Y.T
    X = torch.from_numpy(Xp).to(cuda)
    sp = Plan(net)
    ref = [sp.eval(torch.from_numpy(Y[k]).to(cuda)) for k in range(I)]
    for sched in (None, dict(batch_buses=1, batch_group=1, waves_per_block=1),
                  dict(batch_buses=7, batch_group=2, grid_blocks=5),
                  dict(batch_buses=64, batch_order=1, batch_group=64)):
        if sched:
            bp.schedule = dict(bp.schedule, **sched)
        F = torch.full((bp.n, LD), 7.0, dtype=torch.float64, device=cuda)
        J = torch.full((bp.nnz, LD), 7.0, dtype=torch.float64, device=cuda)
        bp.eval_batch(X, F, J)
        F1 = torch.full_like(F, 7.0)
        J1 = torch.full_like(J, 7.0)
        bp.eval_batch(X, F1, None, want_J=False)
        bp.eval_batch(X, None, J1, want_F=False)
        torch.cuda.synchronize()
        for k in range(I):
            assert torch.equal(F[:, k], ref[k][0]) and torch.equal(J[:, k], ref[k][1]), (sched, k)
        assert torch.equal(F1, F) and torch.equal(J1, J), sched
        assert torch.all(F[:, I:] == 7.0) and torch.all(J[:, I:] == 7.0), sched


def test_outage_slots_are_exact_zero(cuda):
    """Taking out a branch with no parallel partner zeroes its eight
    off-diagonal slots exactly."""
    Plan = _Plan()
    net = synth.tiny_grid(0)
    e = int(synth.non_bridge_branches(net)[7])
    f, t = int(net.br_from[e]), int(net.br_to[e])
    bp = Plan(net, batch=dict(n_inst=2, outage=[-1, e]))
    Y = synth.random_states(net, 2, seed=1)
    Y[1] = Y[0]
    _, Jb = _batch_eval(bp, Y, cuda)
    rp, ci = bp.pattern()
    N = net.n_bus
    slots = []
    for r, c in [(f, t), (f, N + t), (N + f, t), (N + f, N + t),
                 (t, f), (t, N + f), (N + t, f), (N + t, N + f)]:
        row = ci[rp[r]:rp[r + 1]]
        slots.append(rp[r] + int(np.nonzero(row == c)[0][0]))
    assert np.all(Jb[slots, 1] == 0.0)
    assert np.all(Jb[slots, 0] != 0.0)


def test_schedules_bitwise(cuda):
    Plan = _Plan()
    net = synth.grid_10k()
    I = 100
    ls, ps = synth.batch_scenarios(net, I, seed=2)
    out = np.full(I, -1, np.int32)
    out[::3] = synth.contingencies(net, len(out[::3]), seed=2)
    bp = Plan(net, batch=dict(n_inst=I, load_scale=ls, pv_scale=ps, outage=out))
    X = torch.from_numpy(np.ascontiguousarray(synth.random_states(net, I, seed=3).T)).to(cuda)
    F0, J0 = bp.eval_batch(X)
    for s in [dict(batch_buses=1, batch_order=1, waves_per_block=1, grid_blocks=-1, xcd_remap=2),
              dict(batch_buses=7, batch_order=2, waves_per_block=8, grid_blocks=5, xcd_remap=1),
              dict(batch_buses=64, batch_order=1, waves_per_block=2, grid_blocks=1000, xcd_remap=1),
              dict(batch_buses=3, batch_order=2, waves_per_block=4, grid_blocks=-1, xcd_remap=1)]:
        bp.schedule = dict(bp.schedule, **s)
        F, J = bp.eval_batch(X)
        torch.cuda.synchronize()
        assert torch.equal(F, F0) and torch.equal(J, J0), s


def test_graph_replay_matches_eager(cuda):
    Plan = _Plan()
    net = _net()
    I = 70
    bp = Plan(net, batch=dict(n_inst=I))
    X = torch.from_numpy(np.ascontiguousarray(synth.random_states(net, I, seed=9).T)).to(cuda)
    F0, J0 = bp.eval_batch(X)
    F = torch.zeros_like(F0)
    J = torch.zeros_like(J0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            bp.eval_batch(X, F, J)
    torch.cuda.synchronize()
    for r in range(3):
        F.zero_()
        J.fill_(7.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(F, F0) and torch.equal(J, J0), r
        X.add_(0.0)   # eager work between replays


def test_10k_1024_scenarios_and_contingencies(ora, cuda):
    """512 load/renewable scenarios and 512 N-1 contingencies of the
    10,000-bus grid in one launch; every instance against the oracle on its
    own modified network."""
    Plan = _Plan()
    net = synth.grid_10k()
    I = 1024
    ls = np.ones((I, net.n_load))
    ps = np.ones((I, net.n_pv))
    a, b = synth.batch_scenarios(net, 512, seed=2001)
    ls[:512], ps[:512] = a, b
    out = np.full(I, -1, np.int32)
    out[512:] = synth.contingencies(net, 512, seed=2002)
    spec = dict(n_inst=I, load_scale=ls, pv_scale=ps, outage=out)
    bp = Plan(net, batch=spec)
    Y = synth.random_states(net, I, seed=2003)
    Fb, Jb = _batch_eval(bp, Y, cuda)
    Fb = np.ascontiguousarray(Fb.T)
    Jb = np.ascontiguousarray(Jb.T)
    rp, ci = bp.pattern()
    keys = pattern_keys(rp, ci)
    base_pos = None
    for k in range(I):
        nk = _instance_net(net, spec, k)
        Fo, So = ora.residual(nk, Y[k])
        check_close(Fb[k], Fo, So, f"inst {k} F")
        r, c, v, m = ora.jacobian_coo(nk, Y[k], scales=True)
        if out[k] < 0:
            if base_pos is None:
                base_pos = triplet_positions(keys, bp.n, r, c)
            pos = base_pos
        else:
            pos = triplet_positions(keys, bp.n, r, c)
        check_jacobian_triplets(Jb[k], keys, pos, v, m, f"inst {k} J")


def test_padded_instance_stride(cuda):
    """Rows padded to inst_stride: results equal the unpadded layout bit for
    bit and the padding columns are left untouched."""
    Plan = _Plan()
    net = _net()
    I, LD = 70, 80
    Y = synth.random_states(net, I, seed=12)
    ls, ps = synth.batch_scenarios(net, I, seed=12)
    out = np.full(I, -1, np.int32)
    out[::5] = synth.contingencies(net, len(out[::5]), seed=12)
    spec = dict(n_inst=I, load_scale=ls, pv_scale=ps, outage=out)
    ref = Plan(net, batch=spec)
    F0, J0 = _batch_eval(ref, Y, cuda)
    pp = Plan(net, batch=dict(spec, inst_stride=LD))
    assert pp.ld == LD and pp.n_inst == I
    Xp = np.full((net.n_var, LD), np.nan)
    Xp[:, :I] = Y.T
    X = torch.from_numpy(Xp).to(cuda)
    F = torch.full((pp.n, LD), 7.0, dtype=torch.float64, device=cuda)
    J = torch.full((pp.nnz, LD), 7.0, dtype=torch.float64, device=cuda)
    pp.eval_batch(X, F, J)
    torch.cuda.synchronize()
    F, J = F.cpu().numpy(), J.cpu().numpy()
    assert np.array_equal(F[:, :I], F0) and np.array_equal(J[:, :I], J0)
    assert np.all(F[:, I:] == 7.0) and np.all(J[:, I:] == 7.0)


def test_instance_views_are_zero_copy(cuda):
    """States written through an (n_inst, n) view with strides (1, ld) of a
    padded (n, ld) allocation evaluate in place: the returned F and J are
    views of the same kind, equal bit for bit to the contiguous layout's
    columns, and share storage with the allocation they view."""
    Plan = _Plan()
    net = _net()
    I, LD = 70, 80
    Y = synth.random_states(net, I, seed=31)
    pp = Plan(net, batch=dict(n_inst=I, inst_stride=LD))
    buf = torch.zeros((pp.n, LD), dtype=torch.float64, device=cuda)
    Xv = pp.instances(buf)
    assert Xv.shape == (I, pp.n) and Xv.stride() == (1, LD) and Xv.data_ptr() == buf.data_ptr()
    Xv.copy_(torch.from_numpy(Y).to(cuda))
    Fv, Jv = pp.eval_batch(Xv)
    assert Fv.shape == (I, pp.n) and Fv.stride() == (1, LD)
    assert Jv.shape == (I, pp.nnz) and Jv.stride() == (1, LD)
    F, J = pp.eval_batch(buf)
    torch.cuda.synchronize()
    assert torch.equal(Fv, F[:, :I].T) and torch.equal(Jv, J[:, :I].T)
    sp = Plan(net)
    Fs, Js = sp.eval(torch.from_numpy(Y[5]).to(cuda))
    assert torch.equal(Fv[5], Fs) and torch.equal(Jv[5], Js)
    with pytest.raises(ValueError):
        pp.eval_batch(Xv, F=F)           # outputs must follow the input's form
    with pytest.raises(ValueError):
        pp.eval_batch(Xv[:, :-1])


def test_panel_layout_matches_rows(cuda):
    """Panels of 64 instances hold exactly the values of the row layout;
    padding columns of the last panel stay untouched; every schedule agrees."""
    Plan = _Plan()
    net = _net()
    I = 130
    Y = synth.random_states(net, I, seed=21)
    ls, ps = synth.batch_scenarios(net, I, seed=21)
    out = np.full(I, -1, np.int32)
    out[1::4] = synth.contingencies(net, len(out[1::4]), seed=21)
    spec = dict(n_inst=I, load_scale=ls, pv_scale=ps, outage=out)
    F0, J0 = _batch_eval(Plan(net, batch=spec), Y, cuda)
    pp = Plan(net, batch=dict(spec, layout="panels"))
    assert pp.panels and pp.batch_shape(pp.n) == (3, pp.n, 64)
    X = torch.from_numpy(pp.to_batch(Y)).to(cuda)
    for s in [dict(batch_group=1), dict(batch_group=2, batch_order=2, batch_buses=3),
              dict(batch_group=64, waves_per_block=1, grid_blocks=7)]:
        pp.schedule = dict(pp.schedule, **s)
        F = torch.full(pp.batch_shape(pp.n), 7.0, dtype=torch.float64, device=cuda)
        J = torch.full(pp.batch_shape(pp.nnz), 7.0, dtype=torch.float64, device=cuda)
        pp.eval_batch(X, F, J)
        torch.cuda.synchronize()
        assert np.array_equal(pp.from_batch(F), F0.T), s
        assert np.array_equal(pp.from_batch(J), J0.T), s
        Fn, Jn = F.cpu().numpy(), J.cpu().numpy()
        assert np.all(Fn[2, :, I - 128:] == 7.0) and np.all(Jn[2, :, I - 128:] == 7.0)


def test_70k_x1000_bench_configuration(ora, cuda):
    """The benchmark's batched launch as timed (70,000-bus grid, 1000 random
    states in rows padded to 1008, default schedule): every instance
    bit-identical to the single-instance kernel, every residual and every
    eighth Jacobian (plus the chunk edges) against the oracle."""
    Plan = _Plan()
    net = synth.grid_70k()
    S = 1000
    Y = synth.random_states(net, S, seed=1001)
    bp = Plan(net, batch=dict(n_inst=S, inst_stride=1008))
    X = torch.from_numpy(bp.to_batch(Y)).to(cuda)
    F, J = bp.eval_batch(X)
    sp = Plan(net)
    Xs = torch.from_numpy(Y).to(cuda)
    Fs = torch.empty(sp.n, dtype=torch.float64, device=cuda)
    Js = torch.empty(sp.nnz, dtype=torch.float64, device=cuda)
    for k in range(S):
        sp.eval(Xs[k], Fs, Js)
        assert torch.equal(Fs, F[:, k]) and torch.equal(Js, J[:, k]), k
    Fh = np.ascontiguousarray(F[:, :S].cpu().numpy().T)
    for k in range(S):
        Fo, So = ora.residual(net, Y[k])
        check_close(Fh[k], Fo, So, f"inst {k} F")
    del Fh
    rp, ci = bp.pattern()
    keys = pattern_keys(rp, ci)
    pos = None
    ks = sorted(set(range(0, S, 8)) | {63, 64, 511, 959, 960, 999})
    for g in range(0, len(ks), 64):
        kk = ks[g:g + 64]
        Jh = np.ascontiguousarray(J[:, kk].cpu().numpy().T)
        for q, k in enumerate(kk):
            r, c, v, m = ora.jacobian_coo(net, Y[k], scales=True)
            if pos is None:
                pos = triplet_positions(keys, bp.n, r, c)
            check_jacobian_triplets(Jh[q], keys, pos, v, m, f"inst {k} J")
    del F, J, X
    torch.cuda.empty_cache()
