"""Plans set up with the locality bus order (PF_ORDER_LOCALITY): single,
batched (scenarios and outages), multi-grid and adjoint evaluations against
the oracle on the input network, through the plan's state permutation."""

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2011_11880_amd import synth
from parity import check_close, check_jacobian

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _oracle_in_plan_order(ora, net, y, perm):
    """Oracle F, S, J, scale at y (input numbering), rows and columns taken
    to the plan's order: F_plan = F[perm], J_plan = J[perm][:, perm]."""
    Fo, So = ora.residual(net, y)
    Jo, Ao = ora.jacobian(net, y)
    Jp = Jo[perm][:, perm].tocsr()
    Ap = Ao[perm][:, perm].tocsr()
    Jp.sort_indices()
    Ap.sort_indices()
    return Fo[perm], So[perm], Jp, Ap


@pytest.mark.parametrize("which", ["tiny", "10k", "70k"])
def test_single_instance_locality_order(ora, cuda, which):
    from paper_2011_11880_amd.api import Plan
    net = {"tiny": lambda: synth.tiny_grid(3, n_shunt=5), "10k": synth.grid_10k,
           "70k": synth.grid_70k}[which]()
    p = Plan(net, bus_order="locality")
    perm = p.state_perm()
    y = synth.random_states(net, seed=7)
    F, J = p.eval(torch.from_numpy(p.to_plan(y)).to(cuda))
    torch.cuda.synchronize()
    Fo, So, Jo, Ao = _oracle_in_plan_order(ora, net, y, perm)
    check_close(F.cpu().numpy(), Fo, So, f"{which} F")
    rp, ci = p.pattern()
    check_jacobian(rp, ci, J.cpu().numpy(), Jo, Ao, f"{which} J")


def test_batched_locality_order(ora, cuda):
    from paper_2011_11880_amd.api import Plan
    import test_gpu_batch as TB
    net = TB._net()
    I = 70
    ls, ps = synth.batch_scenarios(net, I, seed=5)
    out = np.full(I, -1, np.int32)
    out[35:] = synth.non_bridge_branches(net)[:I - 35]
    spec = dict(n_inst=I, load_scale=ls, pv_scale=ps, outage=out)
    bp = Plan(net, batch=spec, bus_order="locality")
    perm = bp.state_perm()
    Y = synth.random_states(net, I, seed=6)
    X = torch.from_numpy(bp.to_batch(bp.to_plan(Y))).to(cuda)
    F, J = bp.eval_batch(X)
    torch.cuda.synchronize()
    Fh, Jh = bp.from_batch(F), bp.from_batch(J)
    rp, ci = bp.pattern()
    for k in (0, 1, 34, 35, 36, 69):
        nk = TB._instance_net(net, spec, k)
        Fo, So, Jo, Ao = _oracle_in_plan_order(ora, nk, Y[k], perm)
        check_close(Fh[k], Fo, So, f"inst {k} F")
        check_jacobian(rp, ci, Jh[k], Jo, Ao, f"inst {k} J")


def test_multi_grid_locality_order(ora, cuda):
    from paper_2011_11880_amd.api import Plan
    nets = synth.uneven_grids(12, seed=3000)
    mp = Plan.multi(nets, bus_order="locality")
    ys = [synth.random_states(n, seed=60 + g) for g, n in enumerate(nets)]
    y = np.concatenate(ys)
    F, J = mp.eval(torch.from_numpy(mp.to_plan(y)).to(cuda))
    torch.cuda.synchronize()
    F = mp.from_plan(F.cpu().numpy())
    J = J.cpu().numpy()
    order = mp.bus_order()
    b0 = 0
    for g, net in enumerate(nets):
        x0, x1 = mp.x_off[g], mp.x_off[g + 1]
        Fo, So = ora.residual(net, ys[g])
        check_close(F[x0:x1], Fo, So, f"grid {g} F")
        single = Plan(net, host_only=True, bus_order="locality")
        assert np.array_equal(single.bus_order(), order[b0:b0 + net.n_bus])
        perm = single.state_perm()
        _, _, Jo, Ao = _oracle_in_plan_order(ora, net, ys[g], perm)
        rp, ci = single.pattern()
        check_jacobian(rp, ci, J[mp.j_off[g]:mp.j_off[g + 1]], Jo, Ao, f"grid {g} J")
        b0 += net.n_bus


def test_adjoint_locality_order(ora, cuda):
    """J^T W in the plan's order is the oracle's J^T W with both the
    cotangent and the result permuted; parameter gradients keep the
    branch and load order."""
    from paper_2011_11880_amd.api import Plan
    import test_gpu_vjp as V
    net = V._net()
    p = Plan(net, bus_order="locality")
    perm = p.state_perm()
    y = synth.random_states(net, seed=9)
    Wn = np.random.default_rng(9).standard_normal((net.n_var, 5))
    gx, gp = p.vjp(torch.from_numpy(p.to_plan(y)).to(cuda),
                   torch.from_numpy(np.ascontiguousarray(Wn[perm])).to(cuda))
    torch.cuda.synchronize()
    gx, gp = gx.cpu().numpy(), gp.cpu().numpy()
    Jo, Ao = ora.jacobian(net, y)
    B, L = net.n_branch, net.n_load
    for k in range(5):
        go = Jo.T @ Wn[:, k]
        check_close(gx[:, k], go[perm], (Ao.T @ np.abs(Wn[:, k]))[perm], f"gx[{k}]")
        gpo = ora.vjp_params(net, y, Wn[:, k])
        sc = ora.vjp_params_scale(net, y, Wn[:, k])
        for q, name in enumerate(V.PNAMES):
            check_close(gp[q * B:(q + 1) * B, k], gpo[name], sc[name], f"{name}[{k}]")
        np.testing.assert_array_equal(gp[5 * B:5 * B + L, k], gpo["load_p"])
        np.testing.assert_array_equal(gp[5 * B + L:, k], gpo["load_q"])


def test_70k_x1000_bench_configuration_locality_order(ora, cuda, tmp_path):
    """The benchmark's headline launch as timed (70,000-bus grid numbered
    breadth-first at setup, 1000 random states in rows padded to 1008, the
    schedule from the tune cache): every instance bit-identical to the
    single-instance kernel on the same plan order, every residual and every
    eighth Jacobian (plus the chunk edges) against the oracle through the
    plan's permutation."""
    import os
    from paper_2011_11880_amd.api import Plan
    from parity import check_jacobian_triplets, pattern_keys, triplet_positions
    net = synth.grid_70k()
    S = 1000
    Y = synth.random_states(net, S, seed=1001)
    bp = Plan(net, batch=dict(n_inst=S, inst_stride=1008), bus_order="locality")
    perm = bp.state_perm()
    inv = np.empty_like(perm)
    inv[perm] = np.arange(perm.size)
    X = torch.from_numpy(bp.to_batch(bp.to_plan(Y))).to(cuda)
    F = torch.empty((bp.n, 1008), dtype=torch.float64, device=cuda)
    J = torch.empty((bp.nnz, 1008), dtype=torch.float64, device=cuda)
    # the committed tune cache's schedule (a copy: a miss appends to the file)
    import shutil
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune_cache.txt"
    shutil.copy(os.path.join(root, "paper_2011_11880_amd", "tune_cache.txt"), cache)
    bp.autotune(X, F, J, reps=3, cache=str(cache))
    bp.eval_batch(X, F, J)
    sp = Plan(net, bus_order="locality")
    Xs = torch.from_numpy(bp.to_plan(Y)).to(cuda)
    Fs = torch.empty(sp.n, dtype=torch.float64, device=cuda)
    Js = torch.empty(sp.nnz, dtype=torch.float64, device=cuda)
    for k in range(S):
        sp.eval(Xs[k], Fs, Js)
        assert torch.equal(Fs, F[:, k]) and torch.equal(Js, J[:, k]), k
    Fh = np.ascontiguousarray(F[:, :S].cpu().numpy().T)
    for k in range(S):
        Fo, So = ora.residual(net, Y[k])
        check_close(Fh[k], Fo[perm], So[perm], f"inst {k} F")
    del Fh
    rp, ci = bp.pattern()
    keys = pattern_keys(rp, ci)
    pos = None
    ks = sorted(set(range(0, S, 8)) | {63, 64, 127, 128, 511, 959, 960, 999})
    for g in range(0, len(ks), 64):
        kk = ks[g:g + 64]
        Jh = np.ascontiguousarray(J[:, kk].cpu().numpy().T)
        for q, k in enumerate(kk):
            r, c, v, m = ora.jacobian_coo(net, Y[k], scales=True)
            if pos is None:
                pos = triplet_positions(keys, bp.n, inv[r], inv[c])
            check_jacobian_triplets(Jh[q], keys, pos, v, m, f"inst {k} J")
    del F, J, X
    torch.cuda.empty_cache()
