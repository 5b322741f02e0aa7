"""GPU parity of reactive-limit support: evaluation with PV units held at
reactive targets (single, batched, multi-grid, adjoint) against the
oracle, the library's limit check against the oracle's rule, and Newton
with limits (host and device solves) against the oracle's outer loop."""

import numpy as np
import pytest

from paper_2011_11880_amd import synth
from parity import check_close, check_jacobian
from test_oracle_pins import _net_with_everything

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _modes(net, seed, frac=0.4):
    rng = np.random.default_rng(seed)
    mode = (rng.random(net.n_pv) < frac).astype(np.int32)
    qt = np.where(mode == 1, rng.normal(0, 0.5, net.n_pv), 0.0)
    return mode, qt


@pytest.mark.parametrize("which", ["tiny", "everything", "10k"])
def test_eval_with_held_units(ora, cuda, which):
    from paper_2011_11880_amd.api import Plan
    net = {"tiny": lambda: synth.tiny_grid(6), "everything": _net_with_everything,
           "10k": synth.grid_10k}[which]()
    p = Plan(net, q_limits=True)
    rp, ci = p.pattern()
    y = synth.random_states(net, seed=8)
    x = torch.from_numpy(y).to(cuda)
    for mode, qt in ((np.zeros(net.n_pv, np.int32), np.zeros(net.n_pv)), _modes(net, 1),
                     (np.ones(net.n_pv, np.int32), np.linspace(-1, 1, net.n_pv))):
        p.set_gen_modes(mode, qt)
        F, J = p.eval(x)
        torch.cuda.synchronize()
        Fo, So = ora.residual(net, y, modes=(mode, qt))
        Jo, Ao = ora.jacobian(net, y, modes=(mode, qt))
        check_close(F.cpu().numpy(), Fo, So, f"{which} F")
        check_jacobian(rp, ci, J.cpu().numpy(), Jo, Ao, f"{which} J")
    # voltage control with the slot present equals the plain plan's values
    p.set_gen_modes(np.zeros(net.n_pv, np.int32))
    F1, J1 = p.eval(x)
    p0 = Plan(net)
    F0, J0 = p0.eval(x)
    torch.cuda.synchronize()
    assert torch.equal(F0, F1)
    rp0, ci0 = p0.pattern()
    N = net.n_bus
    extra = np.zeros(p.nnz, bool)
    for k in range(net.n_pv):
        extra[rp[2 * N + k] + 1] = True
    assert torch.equal(J0.cpu(), J1.cpu()[torch.from_numpy(~extra)])
    assert not J1.cpu()[torch.from_numpy(extra)].any()


def test_batched_and_multi_with_held_units(ora, cuda):
    from paper_2011_11880_amd.api import Plan
    net = synth.tiny_grid(12)
    mode, qt = _modes(net, 3)
    I = 70
    Y = synth.random_states(net, I, seed=9)
    bp = Plan(net, batch=dict(n_inst=I), q_limits=True)
    bp.set_gen_modes(mode, qt)
    F, J = bp.eval_batch(torch.from_numpy(bp.to_batch(Y)).to(cuda))
    torch.cuda.synchronize()
    Fi, Ji = bp.from_batch(F), bp.from_batch(J)
    sp_ = Plan(net, q_limits=True)
    sp_.set_gen_modes(mode, qt)
    rp, ci = sp_.pattern()
    for i in (0, 33, 69):
        Fs, Js = sp_.eval(torch.from_numpy(Y[i]).to(cuda))
        torch.cuda.synchronize()
        assert np.array_equal(Fs.cpu().numpy(), Fi[i]) and np.array_equal(Js.cpu().numpy(), Ji[i])
        Fo, So = ora.residual(net, Y[i], modes=(mode, qt))
        Jo, Ao = ora.jacobian(net, Y[i], modes=(mode, qt))
        check_close(Fi[i], Fo, So, f"inst {i} F")
        check_jacobian(rp, ci, Ji[i], Jo, Ao, f"inst {i} J")
    # two grids: modes over the concatenated PV units
    nets = [synth.tiny_grid(13, n_bus=60, n_branch=80, n_pv=9), net]
    mp = Plan.multi(nets, q_limits=True)
    m2, q2 = _modes(nets[0], 5)
    mp.set_gen_modes(np.concatenate([m2, mode]), np.concatenate([q2, qt]))
    ys = [synth.random_states(n, seed=20 + g) for g, n in enumerate(nets)]
    F, J = mp.eval(torch.from_numpy(np.concatenate(ys)).to(cuda))
    torch.cuda.synchronize()
    F, J = F.cpu().numpy(), J.cpu().numpy()
    for g, (n, md) in enumerate(zip(nets, [(m2, q2), (mode, qt)])):
        Fo, So = ora.residual(n, ys[g], modes=md)
        Jo, Ao = ora.jacobian(n, ys[g], modes=md)
        check_close(F[mp.x_off[g]:mp.x_off[g + 1]], Fo, So, f"grid {g} F")
        pg = Plan(n, host_only=True, q_limits=True)
        rpg, cig = pg.pattern()
        check_jacobian(rpg, cig, J[mp.j_off[g]:mp.j_off[g + 1]], Jo, Ao, f"grid {g} J")


def test_adjoint_with_held_units(ora, cuda):
    from paper_2011_11880_amd.api import Plan
    net = _net_with_everything()
    mode, qt = _modes(net, 7, frac=0.5)
    p = Plan(net, q_limits=True)
    p.set_gen_modes(mode, qt)
    y = synth.random_states(net, seed=3)
    K = 5
    W = np.random.default_rng(2).normal(size=(p.n, K))
    gx, _ = p.vjp(torch.from_numpy(y).to(cuda), torch.from_numpy(W).to(cuda))
    torch.cuda.synchronize()
    gx = gx.cpu().numpy()
    Jo, Ao = ora.jacobian(net, y, modes=(mode, qt))
    for k in range(K):
        ref = Jo.T @ W[:, k]
        scale = abs(Ao).T @ np.abs(W[:, k])
        check_close(gx[:, k], ref, scale, f"J^T w[{k}]")


def test_limit_check_matches_oracle_rule(ora, cuda):
    from paper_2011_11880_amd.api import Plan
    net = synth.tiny_grid(14)
    N = net.n_bus
    p = Plan(net, q_limits=True)
    rng = np.random.default_rng(6)
    y = synth.random_states(net, seed=6)
    qmin = rng.uniform(-1.0, -0.2, net.n_pv)
    qmax = rng.uniform(0.2, 1.0, net.n_pv)
    # start: some units held at either limit, the rest under voltage control
    mode0 = np.zeros(net.n_pv, np.int32)
    qt0 = np.zeros(net.n_pv)
    mode0[::5] = 1
    qt0[::10] = qmax[::10]
    qt0[5::10] = qmin[5::10]
    for trial in range(3):
        y[2 * N:2 * N + net.n_pv] = rng.uniform(-1.5, 1.5, net.n_pv)
        y[N + net.pv_bus] = net.pv_v + rng.uniform(-0.02, 0.02, net.n_pv)
        p.set_gen_modes(mode0, qt0)
        ns = p.q_limit_check(torch.from_numpy(y).to(cuda), qmin, qmax, tol=1e-9)
        m_o, qt_o, ns_o = ora.q_limit_switch(net, y, mode0, qt0, qmin, qmax, tol=1e-9)
        m, qt = p.gen_modes()
        assert ns == ns_o and ns > 0
        assert np.array_equal(m, m_o) and np.array_equal(qt, qt_o)


def _limits_case(ora, net0, seed, ang, pert, lo_idx, hi_idx, margin):
    import test_gpu_newton_device as D
    net, ystar, y0 = D._manufactured(ora, net0, seed, ang=ang, pert=pert)
    N, NPV = net.n_bus, net.n_pv
    q = ystar[2 * N:2 * N + NPV]
    qmin, qmax = q - 10.0, q + 10.0
    qmax[hi_idx] = q[hi_idx] - margin
    qmin[lo_idx] = q[lo_idx] + margin
    return net, y0, qmin, qmax


@pytest.mark.parametrize("device", [False, True, "rocsolver"])
def test_newton_with_limits_matches_oracle(ora, cuda, device):
    from paper_2011_11880_amd.api import Plan
    net, y0, qmin, qmax = _limits_case(ora, synth.tiny_grid(11), 11, 0.3, (0.02, 0.05),
                                       [2, 30], [1, 4, 9, 20], 0.05)
    y_o, m_o, qt_o, outer_o, ok_o = ora.newton_qlim(net, y0, qmin, qmax)
    assert ok_o and m_o.any()
    p = Plan(net, q_limits=True)
    x = torch.from_numpy(y0).to(cuda)
    rep = p.newton_qlim(x, qmin, qmax, device=device)
    assert rep["converged"] and rep["outer"] == outer_o
    m, qt = p.gen_modes()
    assert np.array_equal(m, m_o) and np.array_equal(qt, qt_o)
    np.testing.assert_allclose(x.cpu().numpy(), y_o, rtol=0, atol=1e-9)


@pytest.mark.parametrize("device", [True, "rocsolver"])
def test_newton_with_limits_10k_device(ora, cuda, device):
    """10k grid: ten units above their upper limit at the solution, by
    0.002.  Larger shifts of held outputs make Newton wander on the
    synthetic grid's weak corridors. The plain switching rule can also
    cycle: a unit forced up by its lower limit raises a capped neighbour's
    voltage, and on some corridors a unit's voltage rises as its output is
    cut. So upper limits only, on units where the oracle's outer loop
    settles. Device Newton with limits ends where that loop does."""
    from paper_2011_11880_amd.api import Plan
    net0 = synth.grid_10k()
    rng = np.random.default_rng(16)
    pick = rng.choice(net0.n_pv, 10, replace=False)
    net, y0, qmin, qmax = _limits_case(ora, net0, 3, 0.03, (1e-4, 2.5e-4),
                                       [], pick, 0.002)
    y_o, m_o, qt_o, outer_o, ok_o = ora.newton_qlim(net, y0, qmin, qmax)
    assert ok_o and m_o.sum() >= 10
    p = Plan(net, q_limits=True)
    x = torch.from_numpy(y0).to(cuda)
    rep = p.newton_qlim(x, qmin, qmax, device=device)
    assert rep["converged"] and rep["outer"] == outer_o
    m, qt = p.gen_modes()
    assert np.array_equal(m, m_o) and np.array_equal(qt, qt_o)
    np.testing.assert_allclose(x.cpu().numpy(), y_o, rtol=0, atol=1e-8)


def _inner_case(which):
    """(network, seed, angle scale, perturbation, units pushed above their
    lower limit, units pushed below their upper limit, margin, state
    tolerance); on the 10k grid ten upper limits only, as in the outer-loop
    test above."""
    if which == "tiny":
        return synth.tiny_grid(11), 11, 0.3, (0.02, 0.05), [2, 30], [1, 4, 9, 20], 0.05, 1e-9
    net0 = synth.grid_10k()
    hi = np.random.default_rng(16).choice(net0.n_pv, 10, replace=False)
    return net0, 3, 0.03, (1e-4, 2.5e-4), [], hi, 0.002, 1e-8


@pytest.mark.parametrize("which", ["tiny", "10k"])
def test_newton_with_limits_checked_in_the_iterations(ora, cuda, which):
    """pf_newton with q_min/q_max: the limits are checked at every iterate
    whose mismatch is below 1e-3, inside one Newton run.  The iterations at
    which units switch, the final modes and targets, the iteration count and
    the end state equal the oracle's in-iteration Newton; the norms agree
    wherever they are above rounding."""
    from paper_2011_11880_amd.api import Plan
    net0, seed, ang, pert, lo, hi, margin, atol = _inner_case(which)
    net, y0, qmin, qmax = _limits_case(ora, net0, seed, ang, pert, lo, hi, margin)
    y_o, m_o, qt_o, norms_o, sw_o, ok_o = ora.newton_qlim_inner(net, y0, qmin, qmax)
    assert ok_o and len(sw_o) >= 1
    p = Plan(net, q_limits=True)
    x = torch.from_numpy(y0).to(cuda)
    rep = p.newton(x, q_min=qmin, q_max=qmax, max_iter=20)
    assert rep["converged"]
    assert [k for k, s in enumerate(rep["switched"]) if s] == sw_o
    assert rep["n_switches"] == sum(rep["switched"]) == int(m_o.sum())
    assert rep["iterations"] == len(norms_o) - 1
    m, qt = p.gen_modes()
    assert np.array_equal(m, m_o) and np.array_equal(qt, qt_o)
    np.testing.assert_allclose(x.cpu().numpy(), y_o, rtol=0, atol=atol)
    big = np.array(norms_o) > 1e-8
    np.testing.assert_allclose(np.array(rep["norms"])[big], np.array(norms_o)[big], rtol=1e-6)
    # the same run through newton_qlim(inner=True), from the same start
    p.set_gen_modes(np.zeros(net.n_pv, np.int32))
    x2 = torch.from_numpy(y0).to(cuda)
    r2 = p.newton_qlim(x2, qmin, qmax, inner=True, max_iter=20)
    assert r2["converged"] and r2["rounds"][0]["switched"] == rep["switched"]
    assert torch.equal(x, x2)


@pytest.mark.parametrize("solver", ["library", "rocsolver"])
@pytest.mark.parametrize("which", ["tiny", "10k"])
def test_device_newton_with_limits_checked_in_the_iterations(ora, cuda, which, solver):
    """Device Newton with the limits checked inside the iterations, on
    pivots from pf_jacobian_switch_order: pf_newton_batch on a plan of one
    instance (this library's factorisation) and pf_newton_device
    (rocSOLVER's re-factorisation).  The iterates at which units switch, the
    final modes and targets, the iteration count and the end state equal
    the oracle's in-iteration Newton, with one host LU for the whole run;
    the norms agree wherever they are above rounding.  newton_qlim(inner=True)
    on the same device path gives the same state bit for bit."""
    from paper_2011_11880_amd.api import Plan, BatchLU, DeviceLU
    net0, seed, ang, pert, lo, hi, margin, atol = _inner_case(which)
    net, y0, qmin, qmax = _limits_case(ora, net0, seed, ang, pert, lo, hi, margin)
    y_o, m_o, qt_o, norms_o, sw_o, ok_o = ora.newton_qlim_inner(net, y0, qmin, qmax)
    assert ok_o and len(sw_o) >= 1
    p = Plan(net, q_limits=True)
    x = torch.from_numpy(y0).to(cuda)
    if solver == "library":
        lu = BatchLU(p, x, switchable=True)
        rep = p.newton_batch(x, lu, q_min=qmin, q_max=qmax, max_iter=20)
        rep["converged"] = rep["n_converged"] == 1
    else:
        lu = DeviceLU(p, x, switchable=True)
        rep = p.newton_device(x, lu, q_min=qmin, q_max=qmax, max_iter=20)
    lu.close()
    assert rep["converged"]
    assert [k for k, s in enumerate(rep["switched"]) if s] == sw_o
    assert rep["n_switches"] == sum(rep["switched"]) == int(m_o.sum())
    assert rep["iterations"] == len(norms_o) - 1
    m, qt = p.gen_modes()
    assert np.array_equal(m, m_o) and np.array_equal(qt, qt_o)
    np.testing.assert_allclose(x.cpu().numpy(), y_o, rtol=0, atol=atol)
    big = np.array(norms_o) > 1e-8
    np.testing.assert_allclose(np.array(rep["norms"])[big], np.array(norms_o)[big], rtol=1e-6)
    p.set_gen_modes(np.zeros(net.n_pv, np.int32))
    x2 = torch.from_numpy(y0).to(cuda)
    r2 = p.newton_qlim(x2, qmin, qmax, device=True if solver == "library" else "rocsolver",
                       inner=True, max_iter=20)
    assert r2["converged"] and r2["rounds"][0]["switched"] == rep["switched"]
    assert torch.equal(x, x2)


def test_device_newton_with_limits_in_the_iterations_70k(ora, cuda):
    """The benchmark's shape at full size: the 70k grid, 20 PV units capped
    0.002 below their output at the manufactured solution, limits checked
    inside the iterations of the device Newton on switch-proof pivots.  The
    switches, iteration count, final modes and end state equal the
    oracle's in-iteration Newton on the same case."""
    from paper_2011_11880_amd.api import Plan
    net0 = synth.grid_70k()
    pick = np.random.default_rng(4103).choice(net0.n_pv, 20, replace=False)
    net, y0, qmin, qmax = _limits_case(ora, net0, 5, 0.03, (1e-4, 2.5e-4), [], pick, 0.002)
    y_o, m_o, qt_o, norms_o, sw_o, ok_o = ora.newton_qlim_inner(net, y0, qmin, qmax)
    assert ok_o and int(m_o.sum()) == 20
    p = Plan(net, q_limits=True)
    x = torch.from_numpy(y0).to(cuda)
    r = p.newton_qlim(x, qmin, qmax, device=True, inner=True, max_iter=30)
    rep = r["rounds"][0]
    assert r["converged"] and [k for k, v in enumerate(rep["switched"]) if v] == sw_o
    assert rep["iterations"] == len(norms_o) - 1
    m, qt = p.gen_modes()
    assert np.array_equal(m, m_o) and np.array_equal(qt, qt_o)
    np.testing.assert_allclose(x.cpu().numpy(), y_o, rtol=0, atol=1e-8)


def test_limit_checks_rejected_where_pivots_are_fixed(cuda):
    """Limit fields are refused by the device Newtons whose pivots a switch
    breaks (either factorisation made without pf_jacobian_switch_order's
    pairing), by the batched Newton on a batched plan, by the fast decoupled
    method, and by pf_newton on a plan without Q_g slots or with
    q_min > q_max."""
    import ctypes
    from paper_2011_11880_amd import capi
    from paper_2011_11880_amd.api import Plan, BatchLU
    from paper_2011_11880_amd.capi import PFError
    net = synth.tiny_grid(11)
    y = synth.random_states(net, seed=1)
    y[:net.n_bus] *= 0.1
    lo = np.full(net.n_pv, -1.0)
    hi = np.full(net.n_pv, 1.0)
    x = torch.from_numpy(y).to(cuda)
    with pytest.raises(PFError, match="q_limits"):
        Plan(net).newton(x.clone(), q_min=lo, q_max=hi)
    p = Plan(net, q_limits=True)
    with pytest.raises(PFError, match="q_min"):
        p.newton(x.clone(), q_min=hi, q_max=lo)
    with pytest.raises(ValueError):
        p.newton(x.clone(), q_min=lo)
    opts = capi.pf_newton_opts(tol=1e-10, max_iter=5)
    opts.q_min = lo.ctypes.data_as(capi._pd)
    opts.q_max = hi.ctypes.data_as(capi._pd)
    rep = capi.pf_newton_report()
    L = capi.lib()
    xd = x.clone()
    lu = BatchLU(p, xd)
    rc = L.pf_newton_batch(p._h, lu._h, ctypes.c_void_p(xd.data_ptr()), ctypes.byref(opts),
                           None, None, ctypes.byref(rep), None)
    assert rc == capi.PF_EINVAL and b"survive a switch" in L.pf_last_error()
    lu.close()
    # a batched plan never qualifies: its modes would be every instance's
    bp = Plan(net, batch=dict(n_inst=2), q_limits=True)
    X2 = torch.from_numpy(bp.to_batch(np.stack([y, y]))).to(cuda)
    blu = BatchLU(bp, X2)
    rc = L.pf_newton_batch(bp._h, blu._h, ctypes.c_void_p(X2.data_ptr()), ctypes.byref(opts),
                           None, None, ctypes.byref(rep), None)
    assert rc == capi.PF_EINVAL and b"non-batched" in L.pf_last_error()
    blu.close()
    with pytest.raises(ValueError, match="one instance"):
        BatchLU(bp, X2, switchable=True)
    dl = p.device_lu(xd)
    rc = L.pf_newton_device(p._h, dl._h, ctypes.c_void_p(xd.data_ptr()), ctypes.byref(opts),
                            ctypes.byref(rep), None)
    assert rc == capi.PF_EINVAL and b"survive a switch" in L.pf_last_error()
    dl.close()
    p.fdlf(xd, max_iter=1)   # creates the fast decoupled object
    rc = L.pf_fdlf_solve(p._fd[0], ctypes.c_void_p(xd.data_ptr()), ctypes.byref(opts),
                         ctypes.byref(rep), None)
    assert rc == capi.PF_EINVAL and b"Newton solvers only" in L.pf_last_error()


@pytest.mark.parametrize("solver", ["host", "device"])
def test_newton_with_limits_in_the_iterations_multi_grid(ora, cuda, solver):
    """pf_newton (host solve) and pf_newton_batch (this library's
    factorisation, pivots that survive a switch) with limits checked inside
    the iterations on a multi-grid plan (two manufactured 200-bus cases,
    limits binding on both): the run converges, and each grid ends feasible
    under its own modes -- F = 0 per the oracle, free units inside their
    limits, held ones at a limit with the voltage on the justifying side --
    in the modes the oracle's in-iteration Newton reaches on that grid
    alone."""
    from paper_2011_11880_amd.api import Plan
    cases = [_limits_case(ora, synth.tiny_grid(11), 11, 0.3, (0.02, 0.05), [2, 30],
                          [1, 4, 9, 20], 0.05),
             _limits_case(ora, synth.tiny_grid(12), 12, 0.3, (0.02, 0.05), [], [3, 7], 0.05)]
    nets = [c[0] for c in cases]
    mp = Plan.multi(nets, q_limits=True)
    x = torch.from_numpy(np.concatenate([c[1] for c in cases])).to(cuda)
    qmin = np.concatenate([c[2] for c in cases])
    qmax = np.concatenate([c[3] for c in cases])
    if solver == "host":
        rep = mp.newton(x, q_min=qmin, q_max=qmax, max_iter=30)
    else:
        rep = mp.newton_batch(x, q_min=qmin, q_max=qmax, max_iter=30)
        rep["converged"] = rep["n_converged"] == 1
    assert rep["converged"] and rep["n_switches"] >= 1
    m, qt = mp.gen_modes()
    xh = x.cpu().numpy()
    k0 = 0
    for g, (net, y0, lo, hi) in enumerate(cases):
        NPV, N = net.n_pv, net.n_bus
        mg, qg_t = m[k0:k0 + NPV], qt[k0:k0 + NPV]
        y = xh[mp.x_off[g]:mp.x_off[g + 1]]
        F, _ = ora.residual(net, y, modes=(mg, qg_t))
        assert np.max(np.abs(F)) < 1e-9, g
        Qg = y[2 * N:2 * N + NPV]
        V = y[N + net.pv_bus]
        free = mg == 0
        assert np.all(Qg[free] <= hi[free] + 1e-9) and np.all(Qg[free] >= lo[free] - 1e-9)
        held = ~free
        assert np.all((qg_t[held] == hi[held]) | (qg_t[held] == lo[held]))
        up = held & (qg_t == hi)
        dn = held & (qg_t == lo)
        assert np.all(V[up] <= net.pv_v[up] + 1e-9) and np.all(V[dn] >= net.pv_v[dn] - 1e-9)
        _, m_o, qt_o, _, _, ok_o = ora.newton_qlim_inner(net, y0, lo, hi)
        assert ok_o and np.array_equal(mg, m_o) and np.array_equal(qg_t, qt_o), g
        k0 += NPV
