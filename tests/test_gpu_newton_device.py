"""Device-resident Newton (pf_refact_* + pf_newton_device): the linear solve
on the GPU by re-factorisation along the pattern of one host LU.  Checked
against the oracle's Jacobian and residual (host sparse solves), against
the oracle's Newton iterates, and for convergence on manufactured solutions
up to the 70k-bus grid."""

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


def _grid(which):
    return {"tiny": lambda: synth.tiny_grid(7), "10k": synth.grid_10k,
            "70k": synth.grid_70k}[which]()


def _manufactured(ora, net0, seed, ang=0.3, pert=(0.02, 0.05)):
    """Network and solution y* with F(y*) = 0, and a perturbed start y0.
    The synthetic geometric grids join dense regions by thin corridors, so
    their Jacobians are nearly singular along relative shifts of a region's
    angles; the large ones take small angles at y* (ang) and a start within
    1e-4 of it, where Newton from the oracle reaches y* in a few steps."""
    import test_oracle_pins as P
    net0 = synth.fill_zero_injection_buses(net0)
    N = net0.n_bus
    ystar = synth.random_states(net0, seed=21 + seed)
    ystar[:N] *= ang
    net, ystar = P.manufactured(ora, net0, ystar)
    F, S = ora.residual(net, ystar)
    assert np.max(np.abs(F)) <= 1e-12 * max(1.0, np.max(S))
    rng = np.random.default_rng(seed)
    y0 = ystar + np.concatenate([rng.normal(0, pert[0], 2 * N),
                                 rng.normal(0, pert[1], net.n_var - 2 * N)])
    return net, ystar, y0


@pytest.mark.parametrize("which", ["tiny", "10k"])
def test_device_solve_matches_host_solve(ora, cuda, which):
    """LU pattern and pivots from J(y0); refactorise at another state y1 and
    solve J(y1) d = F(y1) on the device; compare with the oracle's J(y1),
    F(y1) and a host sparse solve."""
    from paper_2011_11880_amd.api import Plan
    net = _grid(which)
    y0 = synth.random_states(net, seed=11)
    y1 = synth.random_states(net, seed=12)
    p = Plan(net)
    lu = p.device_lu(torch.from_numpy(y0).to(cuda))
    F1, J1 = p.eval(torch.from_numpy(y1).to(cuda))
    d = F1.clone()
    lu.solve(J1, d)
    torch.cuda.synchronize()
    d = d.cpu().numpy()
    Jo, _ = ora.jacobian(net, y1)
    Fo, _ = ora.residual(net, y1)
    dh = spla.spsolve(Jo.tocsc(), Fo)
    res = np.max(np.abs(Jo @ d - Fo))
    scale = abs(Jo).max() * np.max(np.abs(d)) + np.max(np.abs(Fo))
    assert res <= 1e-11 * scale, (res, scale)
    assert np.max(np.abs(d - dh)) <= 1e-8 * np.max(np.abs(dh)), np.max(np.abs(d - dh))
    # a second solve with the same object and another right-hand side
    b = torch.from_numpy(Fo[::-1].copy()).to(cuda)
    lu.solve(J1, b)
    torch.cuda.synchronize()
    dh2 = spla.spsolve(Jo.tocsc(), Fo[::-1].copy())
    assert np.max(np.abs(b.cpu().numpy() - dh2)) <= 1e-8 * np.max(np.abs(dh2))


def test_newton_device_iterates_match_oracle(ora, cuda):
    """Iterate m of the device Newton equals iterate m of the oracle's Newton
    (host sparse solves) to 1e-9, for every m up to convergence."""
    from paper_2011_11880_amd.api import Plan
    net, ystar, y0 = _manufactured(ora, synth.tiny_grid(5), 5)
    p = Plan(net)
    _, norms_o, iters_o = ora.newton(net, y0, tol=1e-10, max_iter=10)
    lu = p.device_lu(torch.from_numpy(y0).to(cuda))
    for m in range(1, len(iters_o)):
        x = torch.from_numpy(y0).to(cuda)
        rep = p.newton_device(x, lu, tol=1e-300, max_iter=m)
        assert rep["iterations"] == m and not rep["converged"]
        np.testing.assert_allclose(x.cpu().numpy(), iters_o[m], rtol=1e-9, atol=1e-11)
        np.testing.assert_allclose(rep["norms"][:m + 1], norms_o[:m + 1], rtol=1e-6, atol=1e-13)


@pytest.mark.parametrize("which", ["tiny", "10k", "70k"])
def test_newton_device_converges(ora, cuda, which):
    from paper_2011_11880_amd.api import Plan
    if which == "tiny":
        net, ystar, y0 = _manufactured(ora, _grid(which), 3)
    else:
        net, ystar, y0 = _manufactured(ora, _grid(which), 3, ang=0.03, pert=(1e-4, 2.5e-4))
    p = Plan(net)
    x = torch.from_numpy(y0).to(cuda)
    rep = p.newton_device(x, tol=1e-10, max_iter=10)
    assert rep["converged"], rep
    assert rep["norms"][-1] < 1e-10 and len(rep["norms"]) == rep["iterations"] + 1
    assert np.max(np.abs(x.cpu().numpy() - ystar)) < 1e-8
    if which == "tiny":
        big = [v for v in rep["norms"] if v > 1e-8]
        for a, b in zip(big, big[1:]):  # quadratic: the error exponent doubles
            assert b <= 50 * a * a + 1e-11, rep["norms"]
    # the oracle's Newton (host sparse solves) takes as many steps, to one
    _, norms_o, _ = ora.newton(net, y0, tol=1e-10, max_iter=10)
    assert abs((len(norms_o) - 1) - rep["iterations"]) <= 1, (norms_o, rep["norms"])
    assert abs(rep["norms"][0] - norms_o[0]) <= 1e-12 * norms_o[0]


def test_newton_device_failure_paths(ora, cuda):
    from paper_2011_11880_amd.api import Plan
    from paper_2011_11880_amd.capi import PF_EINVAL, PFError
    net, ystar, y0 = _manufactured(ora, synth.tiny_grid(8), 8)
    p, q = Plan(net), Plan(net)
    x = torch.from_numpy(y0).to(cuda)
    lu_q = q.device_lu(x)
    with pytest.raises(PFError) as ei:
        p.newton_device(x, lu_q)
    assert ei.value.code == PF_EINVAL
    with pytest.raises(PFError) as ei:
        q.newton_device(x, lu_q, max_iter=65)
    assert ei.value.code == PF_EINVAL
    # a NaN in the state: the norm is NaN, no convergence, no error
    y = y0.copy()
    y[3] = np.nan
    xn = torch.from_numpy(y).to(cuda)
    rep = q.newton_device(xn, lu_q, max_iter=2)
    assert not rep["converged"] and np.isnan(rep["norms"][0])
    # the object is still usable afterwards
    x = torch.from_numpy(y0).to(cuda)
    rep = q.newton_device(x, lu_q)
    assert rep["converged"]
    q.close()  # releases the refactorisation first
    assert lu_q._h is None
