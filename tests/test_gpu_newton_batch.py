"""Batched Newton (pf_batch_lu_* + pf_newton_batch): every instance of a
batched plan factorised on the device along one shared LU pattern.  Solves
against host sparse solves of each instance's own network (oracle J and F),
and Newton per instance against the oracle's Newton on that network."""

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from paper_2011_11880_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _instance_net(net, outage, ls=None, ps=None, k=None):
    v = net if outage < 0 else net.without_branch(int(outage))
    if ls is not None:
        v = v.copy()
        v.load_p = net.load_p * ls[k]
        v.load_q = net.load_q * ls[k]
        v.pv_p = net.pv_p * ps[k]
    return v


@pytest.mark.parametrize("which", ["tiny", "10k"])
def test_batched_solves_match_host(ora, cuda, which):
    """Random states, 70 instances (N-1 outages and the base case):
    factorise every instance along the pattern of instance 0's LU and solve
    J_i d = F_i; compare with the oracle's J_i, F_i and a host solve."""
    from paper_2011_11880_amd.api import Plan
    net = synth.tiny_grid(9) if which == "tiny" else synth.grid_10k()
    I = 70
    out = np.full(I, -1, np.int32)
    out[1:] = synth.contingencies(net, I - 1, seed=77)
    p = Plan(net, batch=dict(n_inst=I, outage=out))
    Y = synth.random_states(net, I, seed=78)
    X = torch.from_numpy(p.to_batch(Y)).to(cuda)
    lu = p.batch_lu(X)
    F, J = p.eval_batch(X)
    lu.factor(J)
    D = lu.solve(F)
    torch.cuda.synchronize()
    Dh = p.from_batch(D)
    for i in (0, 1, 33, 63, 64, 69):
        v = _instance_net(net, out[i])
        Jo, _ = ora.jacobian(v, Y[i])
        Fo, _ = ora.residual(v, Y[i])
        d = Dh[i]
        res = np.max(np.abs(Jo @ d - Fo))
        assert res <= 1e-10 * (abs(Jo).max() * np.max(np.abs(d)) + np.max(np.abs(Fo))), (i, res)
        ref = spla.spsolve(Jo.tocsc(), Fo)
        assert np.max(np.abs(d - ref)) <= 1e-7 * np.max(np.abs(ref)), i


def test_newton_batch_contingencies_10k(ora, cuda):
    """N-1 contingency analysis on the 10k grid: 130 outages (plus the base
    case), every instance warm-started at the base solution.  Each
    instance's convergence, step count and end state match the oracle's
    Newton on that instance's network."""
    from paper_2011_11880_amd.api import Plan
    import test_gpu_newton_device as D
    net, ystar, _ = D._manufactured(ora, synth.grid_10k(), 3, ang=0.03, pert=(0, 0))
    I = 131
    out = np.full(I, -1, np.int32)
    out[1:] = synth.contingencies(net, I - 1, seed=2002)
    p = Plan(net, batch=dict(n_inst=I, outage=out))
    X = torch.from_numpy(p.to_batch(np.tile(ystar, (I, 1)))).to(cuda)
    rep = p.newton_batch(X, tol=1e-10, max_iter=12)
    Xh = p.from_batch(X)
    assert rep["inst_iterations"][0] == 0          # the base case is already solved
    n_ok = 0
    for i in range(0, I, 10):
        v = _instance_net(net, out[i])
        y, norms, _ = ora.newton(v, ystar, tol=1e-10, max_iter=12)
        conv_o = norms[-1] < 1e-10
        conv = rep["inst_norm"][i] < 1e-10
        assert conv == conv_o, (i, norms, rep["inst_norm"][i])
        if conv:
            n_ok += 1
            assert abs(int(rep["inst_iterations"][i]) - (len(norms) - 1)) <= 1, i
            np.testing.assert_allclose(Xh[i], y, rtol=0, atol=1e-8)
    assert n_ok >= 10
    assert rep["n_converged"] == int(np.sum(rep["inst_norm"] < 1e-10))


def test_newton_batch_tiny_scenarios(ora, cuda):
    """200-bus grid: 70 instances with load and PV scale factors (a width
    that leaves a partial chunk) from a perturbed start; every instance
    against the oracle's Newton."""
    from paper_2011_11880_amd.api import Plan
    import test_gpu_newton_device as D
    net, ystar, y0 = D._manufactured(ora, synth.tiny_grid(10), 10)
    I = 70
    rng = np.random.default_rng(11)
    ls = np.exp(0.02 * rng.normal(size=(I, net.n_load)))
    ps = rng.uniform(0.97, 1.03, (I, net.n_pv))
    p = Plan(net, batch=dict(n_inst=I, load_scale=ls, pv_scale=ps))
    X = torch.from_numpy(p.to_batch(np.tile(y0, (I, 1)))).to(cuda)
    rep = p.newton_batch(X, tol=1e-10, max_iter=12)
    Xh = p.from_batch(X)
    assert rep["n_converged"] == I
    for i in range(I):
        v = _instance_net(net, -1, ls, ps, i)
        y, norms, _ = ora.newton(v, y0, tol=1e-10, max_iter=12)
        assert norms[-1] < 1e-10
        assert abs(int(rep["inst_iterations"][i]) - (len(norms) - 1)) <= 1, i
        np.testing.assert_allclose(Xh[i], y, rtol=0, atol=1e-9)


def test_newton_batch_failure_paths(ora, cuda):
    from paper_2011_11880_amd.api import Plan
    from paper_2011_11880_amd.capi import PF_EINVAL, PFError
    net = synth.tiny_grid(12)
    I = 5
    p = Plan(net, batch=dict(n_inst=I))
    q = Plan(net, batch=dict(n_inst=I))
    X = torch.from_numpy(p.to_batch(synth.random_states(net, I, seed=1))).to(cuda)
    lu_q = q.batch_lu(X)
    with pytest.raises(PFError) as ei:
        p.newton_batch(X, lu_q)
    assert ei.value.code == PF_EINVAL
    with pytest.raises(PFError) as ei:
        q.newton_batch(X, lu_q, max_iter=65)
    assert ei.value.code == PF_EINVAL
    # a random state on this grid does not converge in 2 steps: no error
    rep = q.newton_batch(X, lu_q, max_iter=2)
    assert rep["n_converged"] < I and rep["iterations"] == 2
    # a NaN in one instance: its norm and the largest norm are NaN
    Y = synth.random_states(net, I, seed=1)
    Y[2, 3] = np.nan
    X = torch.from_numpy(q.to_batch(Y)).to(cuda)
    rep = q.newton_batch(X, lu_q, max_iter=1)
    assert np.isnan(rep["inst_norm"][2]) and np.isnan(rep["norms"][0])
    assert np.all(np.isfinite(np.delete(rep["inst_norm"], 2)))
    q.close()
    assert lu_q._h is None


@pytest.mark.parametrize("which", ["tiny", "10k"])
def test_one_instance_plan_solves_match_host(ora, cuda, which):
    """A single-instance plan is one instance of the batched factorisation:
    factorise and solve at a random state, against a host solve of the
    oracle's J and F."""
    from paper_2011_11880_amd.api import Plan
    net = synth.tiny_grid(9) if which == "tiny" else synth.grid_10k()
    p = Plan(net)
    y = synth.random_states(net, seed=41)
    x = torch.from_numpy(y).to(cuda)
    lu = p.batch_lu(x)
    F, J = p.eval(x)
    lu.factor(J)
    d = lu.solve(F)
    torch.cuda.synchronize()
    assert tuple(d.shape) == (p.n,)
    d = d.cpu().numpy()
    Jo, _ = ora.jacobian(net, y)
    Fo, _ = ora.residual(net, y)
    ref = spla.spsolve(Jo.tocsc(), Fo)
    np.testing.assert_allclose(d, ref, rtol=0, atol=1e-7 * np.max(np.abs(ref)))


@pytest.mark.parametrize("which", ["tiny", "10k", "70k"])
def test_one_instance_newton_matches_oracle(ora, cuda, which):
    """Device-resident Newton of a single-instance plan on the library's own
    factorisation: the oracle's step count and end state (200 and 10k
    buses), convergence to the manufactured solution at 70k."""
    from paper_2011_11880_amd.api import Plan
    import test_gpu_newton_device as D
    if which == "tiny":
        net, ystar, y0 = D._manufactured(ora, synth.tiny_grid(7), 7)
    else:
        net0 = synth.grid_10k() if which == "10k" else synth.grid_70k()
        net, ystar, y0 = D._manufactured(ora, net0, 3, ang=0.03, pert=(1e-4, 2.5e-4))
    p = Plan(net)
    x = torch.from_numpy(y0).to(cuda)
    rep = p.newton_batch(x, tol=1e-10, max_iter=12)
    assert rep["n_converged"] == 1 and rep["inst_norm"][0] < 1e-10
    xh = x.cpu().numpy()
    if which != "70k":
        y, norms, _ = ora.newton(net, y0, tol=1e-10, max_iter=12)
        assert norms[-1] < 1e-10
        assert abs(rep["iterations"] - (len(norms) - 1)) <= 1
        np.testing.assert_allclose(xh, y, rtol=0, atol=1e-9)
    np.testing.assert_allclose(xh, ystar, rtol=0, atol=1e-6)


def test_one_instance_multi_grid_newton(ora, cuda):
    """Two grids in one multi-grid plan, solved together as one instance."""
    from paper_2011_11880_amd.api import Plan
    import test_gpu_newton_device as D
    cases = [D._manufactured(ora, synth.tiny_grid(s, n_bus=60 + 40 * s, n_branch=85 + 55 * s,
                                                  n_pv=8), 30 + s) for s in range(2)]
    nets = [c[0] for c in cases]
    mp = Plan.multi(nets)
    x = torch.from_numpy(np.concatenate([c[2] for c in cases])).to(cuda)
    rep = mp.newton_batch(x, tol=1e-10, max_iter=12)
    assert rep["n_converged"] == 1
    xh = x.cpu().numpy()
    for g, (net, ystar, y0) in enumerate(cases):
        y, norms, _ = ora.newton(net, y0, tol=1e-10, max_iter=12)
        assert norms[-1] < 1e-10
        np.testing.assert_allclose(xh[mp.x_off[g]:mp.x_off[g + 1]], y, rtol=0, atol=1e-9)


def test_one_instance_failure_paths(ora, cuda):
    """A single-instance plan's Newton on its own factorisation: a
    factorisation of another plan is refused, a start that does not converge
    in the allowed steps reports it without error, and a NaN state gives a
    NaN norm."""
    from paper_2011_11880_amd.api import Plan
    from paper_2011_11880_amd.capi import PF_EINVAL, PFError
    net = synth.tiny_grid(12)
    p, q = Plan(net), Plan(net)
    y = synth.random_states(net, seed=5)
    x = torch.from_numpy(y).to(cuda)
    lu_q = q.batch_lu(x)
    with pytest.raises(PFError) as ei:
        p.newton_batch(x, lu_q)
    assert ei.value.code == PF_EINVAL
    rep = q.newton_batch(x, lu_q, max_iter=1)
    assert rep["n_converged"] == 0 and rep["iterations"] == 1
    y[3] = np.nan
    x = torch.from_numpy(y).to(cuda)
    rep = q.newton_batch(x, lu_q, max_iter=1)
    assert np.isnan(rep["inst_norm"][0]) and np.isnan(rep["norms"][0])
    q.close()
    assert lu_q._h is None
