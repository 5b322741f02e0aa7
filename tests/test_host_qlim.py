"""Host side of reactive-limit support (no GPU): the pattern of a plan set
up with q_limits, and the mode entry points' checks."""

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2011_11880_amd import capi, synth
from paper_2011_11880_amd.api import Plan
from paper_2011_11880_amd.capi import PFError
from test_oracle_pins import _net_with_everything


@pytest.mark.parametrize("which", ["tiny", "everything"])
def test_pattern_is_union_of_both_modes(ora, which):
    net = synth.tiny_grid(3) if which == "tiny" else _net_with_everything()
    p0 = Plan(net, host_only=True)
    p = Plan(net, host_only=True, q_limits=True)
    assert p.nnz == p0.nnz + net.n_pv and p.n == p0.n
    y = synth.random_states(net, seed=2)
    ones = np.ones(net.n_pv, np.int32)
    J0, _ = ora.jacobian(net, y)
    J1, _ = ora.jacobian(net, y, modes=(ones, np.zeros(net.n_pv)))
    U = (abs(J0) + abs(J1)).tocsr()
    U.data[:] = 1
    U.sort_indices()
    rp, ci = p.pattern()
    # structural pattern of the union (explicit zeros of either side kept)
    S0 = sp.csr_matrix((np.ones(J0.nnz), J0.indices, J0.indptr), shape=J0.shape)
    S1 = sp.csr_matrix((np.ones(J1.nnz), J1.indices, J1.indptr), shape=J1.shape)
    Su = (S0 + S1).tocsr()
    Su.sort_indices()
    assert np.array_equal(rp, Su.indptr) and np.array_equal(ci, Su.indices)
    # each PV control row: V column, then the unit's own Q_g column
    N = net.n_bus
    for k in range(net.n_pv):
        r = 2 * N + k
        assert list(ci[rp[r]:rp[r + 1]]) == [N + net.pv_bus[k], 2 * N + k]


def test_multi_grid_pattern_with_slots():
    nets = [synth.tiny_grid(1, n_bus=30, n_branch=40, n_pv=4), synth.tiny_grid(2)]
    p0 = Plan.multi(nets, host_only=True)
    p = Plan.multi(nets, host_only=True, q_limits=True)
    assert p.nnz == p0.nnz + sum(n.n_pv for n in nets)


def test_mode_entry_points():
    net = synth.tiny_grid(4)
    p = Plan(net, host_only=True, q_limits=True)
    m, qt = p.gen_modes()
    assert not m.any() and not qt.any()
    mode = np.zeros(net.n_pv, np.int32)
    mode[[0, 7]] = 1
    target = np.linspace(-1, 1, net.n_pv)
    p.set_gen_modes(mode, target)
    m, qt = p.gen_modes()
    assert np.array_equal(m, mode)
    assert qt[0] == target[0] and qt[7] == target[7] and not np.delete(qt, [0, 7]).any()
    p.set_gen_modes(np.zeros(net.n_pv, np.int32))   # all back to voltage control
    assert not p.gen_modes()[0].any()
    bad = mode.copy()
    bad[3] = 2
    with pytest.raises(PFError) as ei:
        p.set_gen_modes(bad, target)
    assert ei.value.code == capi.PF_EINVAL
    with pytest.raises(PFError):
        p.set_gen_modes(mode, None)           # held without a target
    t2 = target.copy()
    t2[7] = np.nan
    with pytest.raises(PFError):
        p.set_gen_modes(mode, t2)
    assert not p.gen_modes()[0].any()         # a rejected call changes nothing
    plain = Plan(net, host_only=True)
    with pytest.raises(PFError) as ei:
        plain.set_gen_modes(mode, target)
    assert "q_limits" in str(ei.value)
    with pytest.raises(PFError) as ei:          # the check needs a device plan
        p.q_limit_check(None, np.zeros(net.n_pv), np.ones(net.n_pv))
    assert ei.value.code == capi.PF_EINVAL


def test_row_order_follows_modes(ora):
    """Held units keep their control row (its +1 at the unit's own Q_g is
    then the diagonal); units under voltage control trade rows with their
    bus's Q row.  Every diagonal entry of the reordered Jacobian is nonzero
    in both modes."""
    net = synth.tiny_grid(4)
    p = Plan(net, host_only=True, q_limits=True)
    N = net.n_bus
    mode = np.zeros(net.n_pv, np.int32)
    mode[[0, 3]] = 1
    qt = np.zeros(net.n_pv)
    p.set_gen_modes(mode, qt)
    R = p.jacobian_row_order()
    for k in range(net.n_pv):
        if mode[k]:
            assert R[2 * N + k] == 2 * N + k and R[N + net.pv_bus[k]] == N + net.pv_bus[k]
        else:
            assert R[2 * N + k] == N + net.pv_bus[k] and R[N + net.pv_bus[k]] == 2 * N + k
    y = synth.random_states(net, seed=2)
    J, _ = ora.jacobian(net, y, modes=(mode, qt))
    rp, ci = p.pattern()
    from parity import oracle_on_pattern
    v, _, _ = oracle_on_pattern(rp, ci, J, abs(J))
    import scipy.sparse as sp
    Jp = sp.csr_matrix((v, ci, rp), shape=(p.n, p.n))
    assert np.all(Jp[R].diagonal() != 0)


def test_newton_limit_arguments_checked_before_any_call():
    net = synth.tiny_grid(4)
    p = Plan(net, host_only=True, q_limits=True)
    lo = np.full(net.n_pv, -1.0)
    with pytest.raises(ValueError, match="together"):
        p.newton(None, q_min=lo)
    with pytest.raises(ValueError, match="one entry per PV unit"):
        p.newton(None, q_min=lo[:-1], q_max=lo[:-1] + 2)
    with pytest.raises(ValueError, match="together"):
        p.newton_batch(None, lu=object(), q_max=lo)
    with pytest.raises(ValueError, match="together"):
        p.newton_device(None, lu=object(), q_min=lo)
    with pytest.raises(ValueError, match="one entry per PV unit"):
        p.newton_device(None, lu=object(), q_min=lo[1:], q_max=lo[1:])


def _lu_no_pivoting(A):
    """Dense LU of A in its given order (packed L - I + U) and the smallest
    |pivot| met; (None, 0.0) at an exactly zero pivot."""
    A = np.array(A, dtype=np.float64)
    smallest = np.inf
    for k in range(A.shape[0]):
        piv = A[k, k]
        if piv == 0.0:
            return None, 0.0
        smallest = min(smallest, abs(piv))
        A[k + 1:, k] /= piv
        A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
    return A, smallest


@pytest.mark.parametrize("seed", [1, 3])
def test_switch_safe_pivots_hold_in_both_modes(ora, seed):
    """Pivots paired by pf_jacobian_switch_order, each PV unit's Q_g column
    eliminated ahead of its bus voltage column, factorise the Jacobian
    without pivoting whatever the units' modes (all under voltage control,
    all held, mixed): no pivot vanishes, the factors stay inside the filled
    pattern that pf_lu_symbolic gives for them, and the solve equals a dense
    solve.  SuperLU's own column order on the same rows, which puts some
    voltage columns first, meets an exactly zero pivot once every unit is
    held -- the case the reordering exists for."""
    import scipy.sparse as sp
    from parity import oracle_on_pattern
    from paper_2011_11880_amd.api import host_lu, lu_pattern, switch_safe_pivots
    net = synth.tiny_grid(seed, n_bus=120, n_branch=170, n_pv=25)
    N, NPV = net.n_bus, net.n_pv
    p = Plan(net, host_only=True, q_limits=True)
    n = p.n
    rp, ci = p.pattern()
    order, qv = p.jacobian_switch_order()
    assert np.array_equal(qv[:, 0], 2 * N + np.arange(NPV))
    assert np.array_equal(qv[:, 1], N + net.pv_bus)
    assert np.array_equal(order[qv[:, 0]], qv[:, 1]) and np.array_equal(order[qv[:, 1]], qv[:, 0])
    assert np.array_equal(np.sort(order), np.arange(n))
    # the order does not follow the modes
    held = np.zeros(NPV, np.int32)
    held[::3] = 1
    p.set_gen_modes(held, np.zeros(NPV))
    o2, qv2 = p.jacobian_switch_order()
    assert np.array_equal(o2, order) and np.array_equal(qv2, qv)
    assert not np.array_equal(p.jacobian_row_order(), order)
    y = synth.random_states(net, seed=seed)

    def dense(mode):
        J, _ = ora.jacobian(net, y, modes=(mode, np.full(NPV, 0.1)))
        v, _, _ = oracle_on_pattern(rp, ci, J, abs(J))
        return sp.csr_matrix((v, ci, rp), shape=(n, n)).toarray()

    M0 = dense(np.zeros(NPV, np.int32))
    v0 = M0[np.repeat(np.arange(n), np.diff(rp)), ci]
    _, _, _, _, q0 = host_lu(rp, ci, v0, n, None, row_order=order)
    at0 = np.argsort(q0)
    assert np.any(at0[qv[:, 0]] > at0[qv[:, 1]])      # some units need the move
    pivP, pivQ = switch_safe_pivots(q0, order, qv)
    at = np.argsort(pivQ)
    assert np.all(at[qv[:, 0]] < at[qv[:, 1]])
    assert np.array_equal(pivP, order[pivQ])
    trp, tci = lu_pattern(rp, ci, n, pivP, pivQ)
    inside = sp.csr_matrix((np.ones(tci.size), tci, trp), shape=(n, n)).toarray() != 0
    rng = np.random.default_rng(seed)
    b = rng.normal(size=n)
    for mode in (np.zeros(NPV, np.int32), np.ones(NPV, np.int32),
                 (rng.random(NPV) < 0.5).astype(np.int32)):
        M = dense(mode)
        LU, smallest = _lu_no_pivoting(M[pivP][:, pivQ])
        assert LU is not None and smallest > 1e-3, mode
        assert np.all(inside | (LU == 0.0))
        L = np.tril(LU, -1) + np.eye(n)
        z = np.linalg.solve(np.triu(LU), np.linalg.solve(L, b[pivP]))
        x = np.empty(n)
        x[pivQ] = z
        ref = np.linalg.solve(M, b)
        assert np.max(np.abs(x - ref)) <= 1e-9 * np.max(np.abs(ref))
    LU, smallest = _lu_no_pivoting(dense(np.ones(NPV, np.int32))[order[q0]][:, q0])
    assert LU is None and smallest == 0.0
    # the same pivots with SuperLU's values of T, for the rocSOLVER path:
    # T = (L - I) + U on the full pattern, L U = M[pivP][:, pivQ]
    from paper_2011_11880_amd.api import host_lu_switchable
    t_rp, t_ci, t_v, sP, sQ = host_lu_switchable(rp, ci, v0, n, order, qv)
    at = np.argsort(sQ)
    assert np.all(at[qv[:, 0]] < at[qv[:, 1]]) and np.array_equal(sP, order[sQ])
    T = sp.csr_matrix((t_v, t_ci, t_rp), shape=(n, n)).toarray()
    L = np.tril(T, -1) + np.eye(n)
    A0 = M0[sP][:, sQ]
    assert np.max(np.abs(L @ np.triu(T) - A0)) <= 1e-12 * np.max(np.abs(A0))
    LU, _ = _lu_no_pivoting(A0)
    assert np.max(np.abs(LU - T)) <= 1e-10 * np.max(np.abs(LU))


def test_switch_order_needs_q_limits():
    net = synth.tiny_grid(4)
    with pytest.raises(PFError, match="q_limits"):
        Plan(net, host_only=True).jacobian_switch_order()


def test_switch_order_without_pv_units_and_on_multi_grid():
    """No PV unit: no pairs, and the order is pf_jacobian_row_order's.  Two
    grids: the pairs of each grid's units sit at that grid's offsets."""
    net = synth.tiny_grid(5, n_bus=30, n_branch=40, n_pv=0)
    p = Plan(net, host_only=True, q_limits=True)
    order, qv = p.jacobian_switch_order()
    assert qv.shape == (0, 2) and np.array_equal(order, p.jacobian_row_order())
    nets = [synth.tiny_grid(1, n_bus=30, n_branch=40, n_pv=4), synth.tiny_grid(2)]
    mp = Plan.multi(nets, host_only=True, q_limits=True)
    order, qv = mp.jacobian_switch_order()
    k = 0
    for g, n in enumerate(nets):
        xo = mp.x_off[g]
        N = n.n_bus
        assert np.array_equal(qv[k:k + n.n_pv, 0], xo + 2 * N + np.arange(n.n_pv))
        assert np.array_equal(qv[k:k + n.n_pv, 1], xo + N + n.pv_bus)
        k += n.n_pv
    assert np.array_equal(order[qv[:, 0]], qv[:, 1]) and np.array_equal(order[qv[:, 1]], qv[:, 0])
