"""Pins of the oracle's reactive-limit handling (CPU only).

Section II-A: in the extended formulation one set of equations covers a PV
unit under voltage control and held at a reactive target, so reactive limits
can be checked during the iterations.  A held generator keeps its Q_g variable
and its control row becomes Q_g - Q_target.  The pins tie that to the
classical treatment (the generator replaced by a constant PQ injection), to
complex-step derivatives, and to the switching rule's plain definition."""

import numpy as np
import pytest

from paper_2011_11880_amd import synth
from test_oracle_pins import _net_with_everything, manufactured


def _solution(ora, seed=9):
    net0 = synth.tiny_grid(seed)
    N = net0.n_bus
    ystar = synth.random_states(net0, seed=30 + seed)
    ystar[:N] *= 0.3
    return manufactured(ora, net0, ystar)


def _as_pq(net, pick, qt):
    """The same network with the PV generators in ``pick`` replaced by loads
    drawing (-P_set, -Q_target)."""
    keep = np.setdiff1d(np.arange(net.n_pv), pick)
    out = net.copy()
    out.pv_bus, out.pv_p, out.pv_v = net.pv_bus[keep], net.pv_p[keep], net.pv_v[keep]
    out.load_bus = np.concatenate([net.load_bus, net.pv_bus[pick]]).astype(np.int32)
    out.load_p = np.concatenate([net.load_p, -net.pv_p[pick]])
    out.load_q = np.concatenate([net.load_q, -qt[pick]])
    return out, keep


def test_held_output_equals_pq_injection(ora):
    """Holding three PV generators at reactive targets gives the same bus
    voltages and angles as the network in which they are PQ injections
    (solved by the oracle's Newton in the plain formulation)."""
    net, ystar = _solution(ora)
    N, NPV = net.n_bus, net.n_pv
    pick = np.array([0, 5, 17])
    mode = np.zeros(NPV, np.int32)
    mode[pick] = 1
    qt = np.zeros(NPV)
    qt[pick] = ystar[2 * N + pick] + np.array([0.05, -0.08, 0.03])
    y1, norms, _ = ora.newton(net, ystar, tol=1e-12, max_iter=12, modes=(mode, qt))
    assert norms[-1] < 1e-12
    np.testing.assert_allclose(y1[2 * N + pick], qt[pick], rtol=0, atol=1e-13)
    net2, keep = _as_pq(net, pick, qt)
    y2 = np.concatenate([ystar[:2 * N], ystar[2 * N + keep], ystar[2 * N + NPV:]])
    y2, norms2, _ = ora.newton(net2, y2, tol=1e-12, max_iter=12)
    assert norms2[-1] < 1e-12
    np.testing.assert_allclose(y1[:2 * N], y2[:2 * N], rtol=0, atol=1e-10)
    np.testing.assert_allclose(y1[2 * N + keep], y2[2 * N:2 * N + keep.size], rtol=0, atol=1e-10)
    np.testing.assert_allclose(y1[2 * N + NPV:], y2[2 * N + keep.size:], rtol=0, atol=1e-10)
    # the held generators' buses no longer sit at their voltage set points
    assert np.min(np.abs(y1[N + net.pv_bus[pick]] - net.pv_v[pick])) > 1e-6


def test_holding_the_solution_output_keeps_the_solution(ora):
    net, ystar = _solution(ora, seed=10)
    N = net.n_bus
    mode = np.ones(net.n_pv, np.int32)
    qt = ystar[2 * N:2 * N + net.n_pv].copy()
    F, S = ora.residual(net, ystar, modes=(mode, qt))
    assert np.max(np.abs(F) - 1e-12 * (S + 1)) <= 0


@pytest.mark.parametrize("which", ["tiny", "everything"])
def test_jacobian_complex_step_with_held_outputs(ora, which):
    net = synth.tiny_grid(2) if which == "tiny" else _net_with_everything()
    rng = np.random.default_rng(4)
    mode = (rng.random(net.n_pv) < 0.5).astype(np.int32)
    qt = rng.normal(0, 0.5, net.n_pv)
    yv = synth.random_states(net, seed=13)
    J, A = ora.jacobian(net, yv, modes=(mode, qt))
    Jd, Ad = J.toarray(), A.toarray()
    h = 1e-30
    for j in range(yv.size):
        yz = yv.astype(complex)
        yz[j] += 1j * h
        col = ora.residual_complex(net, yz, modes=(mode, qt)).imag / h
        np.testing.assert_array_less(np.abs(col - Jd[:, j]), 1e-13 * (Ad[:, j] + 1))
    # a held row has its single +1 on the Q_g column, a controlled row on V
    N = net.n_bus
    for k in range(net.n_pv):
        row = Jd[2 * N + k]
        col = 2 * N + k if mode[k] else N + net.pv_bus[k]
        assert row[col] == 1.0 and np.count_nonzero(row) == 1


def test_switching_rule_cases(ora):
    """Each branch of the rule on one generator at a time."""
    net = synth.tiny_grid(0)
    N = net.n_bus
    k = 3
    bus = net.pv_bus[k]
    vset = net.pv_v[k]
    qmin = np.full(net.n_pv, -1.0)
    qmax = np.full(net.n_pv, 1.0)
    y = synth.random_states(net, seed=1)
    y[2 * N:2 * N + net.n_pv] = 0.0

    def run(q, v, mode_k, qt_k):
        yy = y.copy()
        yy[2 * N + k] = q
        yy[N + bus] = v
        mode = np.zeros(net.n_pv, np.int32)
        qt = np.zeros(net.n_pv)
        mode[k], qt[k] = mode_k, qt_k
        m, t, ns = ora.q_limit_switch(net, yy, mode, qt, qmin, qmax)
        others = np.delete(np.arange(net.n_pv), k)
        assert not m[others].any()
        return int(m[k]), float(t[k]), ns

    assert run(0.5, vset, 0, 0.0) == (0, 0.0, 0)          # inside: stays
    assert run(1.2, vset, 0, 0.0) == (1, 1.0, 1)          # above qmax: held at qmax
    assert run(-1.3, vset, 0, 0.0) == (1, -1.0, 1)        # below qmin: held at qmin
    assert run(1.0, vset - 0.01, 1, 1.0) == (1, 1.0, 0)   # at qmax, V below set: stays
    assert run(1.0, vset + 0.01, 1, 1.0) == (0, 0.0, 1)   # at qmax, V above set: released
    assert run(-1.0, vset + 0.01, 1, -1.0) == (1, -1.0, 0)
    assert run(-1.0, vset - 0.01, 1, -1.0) == (0, 0.0, 1)


def test_newton_with_limits_ends_feasible(ora):
    """After the outer loop: F = 0 under the final modes, controlled
    generators inside their limits, held ones at a limit with the bus
    voltage on the side that justifies holding."""
    net, ystar = _solution(ora, seed=11)
    N, NPV = net.n_bus, net.n_pv
    q = ystar[2 * N:2 * N + NPV]
    qmin = q - 10.0
    qmax = q + 10.0
    qmax[[1, 4, 9, 20]] = q[[1, 4, 9, 20]] - 0.05   # four generators above their upper limit
    qmin[[2, 30]] = q[[2, 30]] + 0.05               # two below their lower limit
    y, mode, qt, outer, ok = ora.newton_qlim(net, ystar, qmin, qmax)
    assert ok and outer >= 2 and mode.sum() >= 1
    F, S = ora.residual(net, y, modes=(mode, qt))
    assert np.max(np.abs(F)) < 1e-10
    Qg = y[2 * N:2 * N + NPV]
    V = y[N + net.pv_bus]
    free = mode == 0
    assert np.all(Qg[free] <= qmax[free] + 1e-9) and np.all(Qg[free] >= qmin[free] - 1e-9)
    held = ~free
    assert np.all((qt[held] == qmax[held]) | (qt[held] == qmin[held]))
    np.testing.assert_allclose(Qg[held], qt[held], rtol=0, atol=1e-12)
    up = held & (qt == qmax)
    lo = held & (qt == qmin)
    assert np.all(V[up] <= net.pv_v[up] + 1e-9) and np.all(V[lo] >= net.pv_v[lo] - 1e-9)


def test_newton_with_limits_checked_in_the_iterations_ends_feasible(ora):
    """Limits checked at every iterate once the mismatch is below 1e-3 (no
    outer loop): the end state is feasible in the same sense as the outer
    loop's (F = 0 under the final modes, free generators inside their
    limits, held ones at a limit with the voltage on the justifying side),
    the switches happen inside the iterations, and for this case the final
    modes and state agree with the outer loop's."""
    net, ystar = _solution(ora, seed=11)
    N, NPV = net.n_bus, net.n_pv
    q = ystar[2 * N:2 * N + NPV]
    qmin = q - 10.0
    qmax = q + 10.0
    qmax[[1, 4, 9, 20]] = q[[1, 4, 9, 20]] - 0.05
    qmin[[2, 30]] = q[[2, 30]] + 0.05
    rng = np.random.default_rng(4)
    y0 = ystar + np.concatenate([rng.normal(0, 0.01, 2 * N), np.zeros(net.n_var - 2 * N)])
    y, mode, qt, norms, sw, ok = ora.newton_qlim_inner(net, y0, qmin, qmax)
    assert ok and len(sw) >= 1 and mode.sum() >= 1
    assert sw[0] > 0 and norms[0] >= 1e-3                # first checked below 1e-3
    assert sw[-1] < len(norms) - 1                       # the last check switched nothing
    F, S = ora.residual(net, y, modes=(mode, qt))
    assert np.max(np.abs(F)) < 1e-10
    Qg = y[2 * N:2 * N + NPV]
    V = y[N + net.pv_bus]
    free = mode == 0
    assert np.all(Qg[free] <= qmax[free] + 1e-9) and np.all(Qg[free] >= qmin[free] - 1e-9)
    held = ~free
    assert np.all((qt[held] == qmax[held]) | (qt[held] == qmin[held]))
    np.testing.assert_allclose(Qg[held], qt[held], rtol=0, atol=1e-12)
    up = held & (qt == qmax)
    lo = held & (qt == qmin)
    assert np.all(V[up] <= net.pv_v[up] + 1e-9) and np.all(V[lo] >= net.pv_v[lo] - 1e-9)
    y2, mode2, qt2, _, ok2 = ora.newton_qlim(net, y0, qmin, qmax)
    assert ok2 and np.array_equal(mode, mode2) and np.array_equal(qt, qt2)
    np.testing.assert_allclose(y, y2, rtol=0, atol=1e-9)
