"""GPU parity of the adjoint (pf_vjp): J^T W and (dF/dp)^T W against the
oracle's explicit transposed-Jacobian product and parameter gradients, the
adjoint as benchmarked (70,000 buses, 64 cotangents) column by column and
gradient by gradient with the dot-product identity <W, J V> = <J^T W, V>,
torch.autograd.gradcheck of PFResidual on the 200-bus grid, and batched
cotangents through torch.func.vmap."""

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2011_11880_amd import synth
from parity import check_close

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PNAMES = ("br_r", "br_x", "br_b", "br_tap", "br_shift_deg")


@pytest.fixture(scope="module")
def cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _net():
    net = synth.tiny_grid(6, n_bus=160, n_branch=230, n_pv=25, n_shunt=10)
    net = synth.with_parallel_branches(net, 6, 2)
    e = int(synth.non_bridge_branches(net)[4])
    net.br_status[e] = 0
    return net


def _check_vjp(ora, plan, net, y, Wn, cuda, what, params_too=True):
    x = torch.from_numpy(y).to(cuda)
    W = torch.from_numpy(np.ascontiguousarray(Wn)).to(cuda)
    gx, gp = plan.vjp(x, W)
    torch.cuda.synchronize()
    gx, gp = gx.cpu().numpy(), gp.cpu().numpy()
    J, A = ora.jacobian(net, y)
    B, L = net.n_branch, net.n_load
    for k in range(Wn.shape[1]):
        w = Wn[:, k]
        go, gpo = ora.vjp(net, y, w)
        scale = A.T @ np.abs(w)
        check_close(gx[:, k], go, scale, f"{what} gx[{k}]")
        if not params_too:
            continue
        sc = ora.vjp_params_scale(net, y, w)
        for q, name in enumerate(PNAMES):
            check_close(gp[q * B:(q + 1) * B, k], gpo[name], sc[name], f"{what} {name}[{k}]")
        np.testing.assert_array_equal(gp[5 * B:5 * B + L, k], gpo["load_p"])
        np.testing.assert_array_equal(gp[5 * B + L:, k], gpo["load_q"])
    return gx, gp


@pytest.mark.parametrize("k", [1, 5, 64, 65, 130])
def test_vjp_vs_oracle(ora, cuda, k):
    from paper_2011_11880_amd.api import Plan
    net = _net()
    p = Plan(net)
    y = synth.random_states(net, seed=k)
    Wn = np.random.default_rng(k).standard_normal((net.n_var, k))
    _check_vjp(ora, p, net, y, Wn, cuda, f"k{k}", params_too=(k <= 65))


def test_vjp_several_loads_per_bus(ora, cuda):
    """Buses with two and three loads (also at PV and slack buses), reversed
    and same-direction parallel branches and an out-of-service branch: every
    gradient row is written (outputs start as NaN) and matches the oracle."""
    from paper_2011_11880_amd.api import Plan
    net = _net()
    rng = np.random.default_rng(21)
    extra = np.concatenate([net.load_bus[:6], net.load_bus[:3], net.pv_bus[:2],
                            net.slack_bus[:1]]).astype(np.int32)
    net = net.copy()
    net.load_bus = np.concatenate([net.load_bus, extra]).astype(np.int32)
    net.load_p = np.concatenate([net.load_p, rng.uniform(0, 1, extra.size)])
    net.load_q = np.concatenate([net.load_q, rng.uniform(-0.2, 0.3, extra.size)])
    p = Plan(net)
    y = synth.random_states(net, seed=22)
    K = 3
    Wn = rng.standard_normal((net.n_var, K))
    x = torch.from_numpy(y).to(cuda)
    W = torch.from_numpy(np.ascontiguousarray(Wn)).to(cuda)
    gx = torch.full((p.n, K), float("nan"), dtype=torch.float64, device=cuda)
    gp = torch.full((p.n_params, K), float("nan"), dtype=torch.float64, device=cuda)
    p.vjp(x, W, gx, gp)
    gp_only = torch.full_like(gp, float("nan"))
    p.vjp(x, W, None, gp_only, want_gx=False)
    gx_only = torch.full_like(gx, float("nan"))
    p.vjp(x, W, gx_only, None, want_gparam=False)
    torch.cuda.synchronize()
    gx, gp = gx.cpu().numpy(), gp.cpu().numpy()
    assert not np.isnan(gx).any() and not np.isnan(gp).any()
    assert np.array_equal(gp, gp_only.cpu().numpy())
    assert np.array_equal(gx, gx_only.cpu().numpy())
    J, A = ora.jacobian(net, y)
    B, L = net.n_branch, net.n_load
    for k in range(K):
        go, gpo = ora.vjp(net, y, Wn[:, k])
        check_close(gx[:, k], go, A.T @ np.abs(Wn[:, k]), f"gx[{k}]")
        sc = ora.vjp_params_scale(net, y, Wn[:, k])
        for q, name in enumerate(PNAMES):
            check_close(gp[q * B:(q + 1) * B, k], gpo[name], sc[name], f"{name}[{k}]")
        np.testing.assert_array_equal(gp[5 * B:5 * B + L, k], gpo["load_p"])
        np.testing.assert_array_equal(gp[5 * B + L:, k], gpo["load_q"])


def test_vjp_hub_rows_and_schedules(ora, cuda):
    from paper_2011_11880_amd.api import Plan
    import test_gpu_eval as E
    net = E._hub_grid()
    y = synth.random_states(net, seed=3)
    Wn = np.random.default_rng(3).standard_normal((net.n_var, 3))
    outs = []
    for te in (64, 512):
        p = Plan(net, schedule=dict(tile_entries=te))
        outs.append(_check_vjp(ora, p, net, y, Wn, cuda, f"hub te{te}"))
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])


def test_vjp_multi_grid(ora, cuda):
    from paper_2011_11880_amd.api import Plan
    nets = [synth.tiny_grid(s, n_bus=40 + 30 * s, n_branch=55 + 40 * s, n_pv=6, n_shunt=3)
            for s in range(3)]
    mp = Plan.multi(nets)
    ys = [synth.random_states(n, seed=g) for g, n in enumerate(nets)]
    y = np.concatenate(ys)
    Wn = np.random.default_rng(9).standard_normal((y.size, 4))
    gx, gp = mp.vjp(torch.from_numpy(y).to(cuda), torch.from_numpy(Wn).to(cuda))
    gx, gp = gx.cpu().numpy(), gp.cpu().numpy()
    Btot = sum(n.n_branch for n in nets)
    boff = 0
    for g, net in enumerate(nets):
        x0, x1 = mp.x_off[g], mp.x_off[g + 1]
        J, A = ora.jacobian(net, ys[g])
        for k in range(4):
            w = Wn[x0:x1, k]
            go, gpo = ora.vjp(net, ys[g], w)
            check_close(gx[x0:x1, k], go, A.T @ np.abs(w), f"grid {g} gx")
            sc = ora.vjp_params_scale(net, ys[g], w)
            for q, name in enumerate(PNAMES):
                seg = gp[q * Btot + boff:q * Btot + boff + net.n_branch, k]
                check_close(seg, gpo[name], sc[name], f"grid {g} {name}")
        boff += net.n_branch


def test_adjoint_70k_64_cotangents(ora, cuda):
    """The adjoint as benchmarked (70,000-bus grid, 64 cotangents, one
    launch): every column of J^T W against the oracle's explicit transposed
    Jacobian, every parameter gradient (r, x, b, tap, shift, load P and Q)
    against the oracle's pi-model partials, and the dot-product identity
    <W_k, J V> = <(J^T W)_k, V> with J from pf_eval."""
    from paper_2011_11880_amd.api import Plan
    net = synth.grid_70k()
    p = Plan(net)
    y = synth.random_states(net, seed=4000)
    rng = np.random.default_rng(4001)
    K = 64
    Wn = rng.standard_normal((net.n_var, K))
    V = rng.standard_normal(net.n_var)
    x = torch.from_numpy(y).to(cuda)
    _, Jv = p.eval(x)
    gx, gp = p.vjp(x, torch.from_numpy(Wn).to(cuda))
    torch.cuda.synchronize()
    rp, ci = p.pattern()
    J = sp.csr_matrix((Jv.cpu().numpy(), ci, rp), shape=(p.n, p.n))
    gx, gp = gx.cpu().numpy(), gp.cpu().numpy()
    JV = J @ V
    absJ = abs(J)
    for k in range(K):
        lhs = Wn[:, k] @ JV
        rhs = gx[:, k] @ V
        scale = np.abs(Wn[:, k]) @ (absJ @ np.abs(V))
        assert abs(lhs - rhs) <= 1e-12 * scale, k
    Jo, Ao = ora.jacobian(net, y)
    GX = Jo.T @ Wn                  # the oracle's J^T w, all columns at once
    SX = Ao.T @ np.abs(Wn)
    B, L = net.n_branch, net.n_load
    for k in range(K):
        check_close(gx[:, k], GX[:, k], SX[:, k], f"70k gx[{k}]")
        gpo = ora.vjp_params(net, y, Wn[:, k])
        sc = ora.vjp_params_scale(net, y, Wn[:, k])
        for q, name in enumerate(PNAMES):
            check_close(gp[q * B:(q + 1) * B, k], gpo[name], sc[name], f"70k {name}[{k}]")
        np.testing.assert_array_equal(gp[5 * B:5 * B + L, k], gpo["load_p"])
        np.testing.assert_array_equal(gp[5 * B + L:, k], gpo["load_q"])


def test_gradcheck_residual(cuda):
    from paper_2011_11880_amd.api import Plan, params_vector
    from paper_2011_11880_amd.autograd import PFResidual
    net = synth.tiny_grid(0, n_shunt=4)
    p = Plan(net)
    x = torch.from_numpy(synth.random_states(net, seed=8)).to(cuda).requires_grad_(True)
    prm = torch.from_numpy(params_vector(net)).to(cuda).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda a, b: PFResidual.apply(a, b, p), (x, prm),
                                    eps=1e-6, atol=1e-6, rtol=1e-5, fast_mode=True)


def test_vmapped_cotangents_reach_multi_cotangent_kernel(cuda):
    """torch.func.vmap over the vjp function hands all cotangents to one
    pf_vjp launch (the inner Function's vmap rule); results equal the
    one-at-a-time backward."""
    from paper_2011_11880_amd.api import Plan, params_vector
    from paper_2011_11880_amd.autograd import PFResidual
    net = synth.tiny_grid(2)
    p = Plan(net)
    x = torch.from_numpy(synth.random_states(net, seed=2)).to(cuda)
    prm = torch.from_numpy(params_vector(net)).to(cuda)
    F, vjp_fn = torch.func.vjp(lambda a, b: PFResidual.apply(a, b, p), x, prm)
    Wb = torch.randn(7, p.n, dtype=torch.float64, device=cuda)
    gx_b, gp_b = torch.func.vmap(vjp_fn)(Wb)
    xr = x.clone().requires_grad_(True)
    pr = prm.clone().requires_grad_(True)
    Fr = PFResidual.apply(xr, pr, p)
    assert torch.equal(F, Fr.detach())
    for i in range(7):
        gx, gp = torch.autograd.grad(Fr, (xr, pr), grad_outputs=Wb[i], retain_graph=True)
        assert torch.equal(gx, gx_b[i]) and torch.equal(gp, gp_b[i])
