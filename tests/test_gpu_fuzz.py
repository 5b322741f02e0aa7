"""GPU parity over seeded random networks (fuzz_nets.random_net: random
size from 2 buses up, transformers with taps and shifts, parallel and
out-of-service branches, shunts, several loads per bus): for each network
the single-instance kernel against the oracle, a batch of random states
bit-identical to single evaluations, held PV units against the oracle with
the same modes, the adjoint against the oracle, and the breadth-first bus
numbering (single against the oracle, batch bit-identical to single); and
the networks together as one multi-grid launch, bit-identical to their own
plans."""

import numpy as np
import pytest

from fuzz_nets import random_net
from paper_2011_11880_amd import synth
from parity import check_close, check_jacobian

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEEDS = range(24)


@pytest.fixture(scope="module")
def cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@pytest.mark.parametrize("seed", SEEDS)
def test_random_network(ora, cuda, seed):
    from paper_2011_11880_amd.api import Plan
    from test_gpu_vjp import _check_vjp
    print(f"fuzz seed {seed}", flush=True)
    net = random_net(seed)
    rng = np.random.default_rng(seed)
    p = Plan(net)
    rp, ci = p.pattern()
    # single instance against the oracle
    y = synth.random_states(net, seed=seed)
    F, J = p.eval(torch.from_numpy(y).to(cuda))
    torch.cuda.synchronize()
    F, J = F.cpu().numpy(), J.cpu().numpy()
    Fo, So = ora.residual(net, y)
    Jo, Ao = ora.jacobian(net, y)
    check_close(F, Fo, So, f"seed {seed} F")
    check_jacobian(rp, ci, J, Jo, Ao, f"seed {seed} J")
    # a batch of states: every instance bit-identical to its single evaluation
    I = int(rng.integers(1, 70))
    Y = synth.random_states(net, I, seed=seed + 100)
    bp = Plan(net, batch=dict(n_inst=I))
    Fb, Jb = bp.eval_batch(torch.from_numpy(np.ascontiguousarray(Y.T)).to(cuda))
    torch.cuda.synchronize()
    Fb, Jb = Fb.cpu().numpy(), Jb.cpu().numpy()
    for k in range(I):
        Fs, Js = p.eval(torch.from_numpy(Y[k]).to(cuda))
        torch.cuda.synchronize()
        assert np.array_equal(Fs.cpu().numpy(), Fb[:, k]), (seed, k)
        assert np.array_equal(Js.cpu().numpy(), Jb[:, k]), (seed, k)
    # PV units held at reactive targets
    if net.n_pv:
        mode = (rng.random(net.n_pv) < 0.5).astype(np.int32)
        qt = np.where(mode == 1, rng.normal(0, 0.5, net.n_pv), 0.0)
        pq = Plan(net, q_limits=True)
        pq.set_gen_modes(mode, qt)
        Fq, Jq = pq.eval(torch.from_numpy(y).to(cuda))
        torch.cuda.synchronize()
        Fo, So = ora.residual(net, y, modes=(mode, qt))
        Jo, Ao = ora.jacobian(net, y, modes=(mode, qt))
        rq, cq = pq.pattern()
        check_close(Fq.cpu().numpy(), Fo, So, f"seed {seed} held F")
        check_jacobian(rq, cq, Jq.cpu().numpy(), Jo, Ao, f"seed {seed} held J")
    # adjoint
    K = int(rng.integers(1, 6))
    Wn = rng.standard_normal((net.n_var, K))
    _check_vjp(ora, p, net, y, Wn, cuda, f"seed {seed} vjp")
    # buses numbered breadth-first at setup: the single kernel against the
    # oracle through the plan's permutation, a batch bit-identical to it
    pl = Plan(net, bus_order="locality")
    perm = pl.state_perm()
    Fl, Jl = pl.eval(torch.from_numpy(pl.to_plan(y)).to(cuda))
    torch.cuda.synchronize()
    Fo, So = ora.residual(net, y)
    Jo, Ao = ora.jacobian(net, y)
    Jp, Ap = Jo[perm][:, perm].tocsr(), Ao[perm][:, perm].tocsr()
    Jp.sort_indices()
    Ap.sort_indices()
    rl, cl = pl.pattern()
    check_close(Fl.cpu().numpy(), Fo[perm], So[perm], f"seed {seed} locality F")
    check_jacobian(rl, cl, Jl.cpu().numpy(), Jp, Ap, f"seed {seed} locality J")
    bl = Plan(net, batch=dict(n_inst=I), bus_order="locality")
    Fb, Jb = bl.eval_batch(torch.from_numpy(np.ascontiguousarray(bl.to_plan(Y).T)).to(cuda))
    torch.cuda.synchronize()
    Fb, Jb = Fb.cpu().numpy(), Jb.cpu().numpy()
    for k in range(I):
        Fs, Js = pl.eval(torch.from_numpy(pl.to_plan(Y[k])).to(cuda))
        torch.cuda.synchronize()
        assert np.array_equal(Fs.cpu().numpy(), Fb[:, k]), (seed, k)
        assert np.array_equal(Js.cpu().numpy(), Jb[:, k]), (seed, k)


def test_random_networks_as_one_multi_grid_launch(ora, cuda):
    from paper_2011_11880_amd.api import Plan
    nets = [random_net(s) for s in SEEDS]
    mp = Plan.multi(nets)
    ys = [synth.random_states(n, seed=500 + g) for g, n in enumerate(nets)]
    F, J = mp.eval(torch.from_numpy(np.concatenate(ys)).to(cuda))
    torch.cuda.synchronize()
    F, J = F.cpu().numpy(), J.cpu().numpy()
    for g, net in enumerate(nets):
        x0, x1 = mp.x_off[g], mp.x_off[g + 1]
        j0, j1 = mp.j_off[g], mp.j_off[g + 1]
        sp_ = Plan(net)
        Fs, Js = sp_.eval(torch.from_numpy(ys[g]).to(cuda))
        torch.cuda.synchronize()
        assert np.array_equal(Fs.cpu().numpy(), F[x0:x1]), g
        assert np.array_equal(Js.cpu().numpy(), J[j0:j1]), g
        Fo, So = ora.residual(net, ys[g])
        check_close(F[x0:x1], Fo, So, f"multi grid {g} F")
