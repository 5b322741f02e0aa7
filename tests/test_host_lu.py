"""Host side of the device-resident Newton: the form in which one host LU is
handed to the device re-factorisation, and the argument checks of
pf_refact_create (no GPU needed)."""

import ctypes

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2011_11880_amd import capi, synth
from paper_2011_11880_amd.api import Plan, host_lu


def _csr(ora, net, seed):
    J, _ = ora.jacobian(net, synth.random_states(net, seed=seed))
    return J


@pytest.mark.parametrize("which", ["tiny", "10k"])
def test_host_lu_reassembles_the_matrix(ora, which):
    """M[pivP][:, pivQ] = L U with L = I + strict lower part of T, U = upper
    part of T (the re-factorisation's convention for P M Q = L U)."""
    net = synth.tiny_grid(4) if which == "tiny" else synth.grid_10k()
    M = _csr(ora, net, 5)
    n = M.shape[0]
    trp, tci, tv, pivP, pivQ = host_lu(M.indptr, M.indices, M.data, n)
    assert sorted(pivP) == list(range(n)) and sorted(pivQ) == list(range(n))
    T = sp.csr_matrix((tv, tci, trp), shape=(n, n))
    for i in range(n):  # strictly increasing columns, diagonal present
        cols = tci[trp[i]:trp[i + 1]]
        assert np.all(np.diff(cols) > 0)
        assert i in cols
    L = sp.tril(T, -1) + sp.identity(n)
    U = sp.triu(T)
    lhs = M[pivP][:, pivQ]
    err = abs(lhs - L @ U).max()
    assert err <= 1e-12 * abs(M).max(), err
    # the factors solve the system: x = Q U^-1 L^-1 P b
    import scipy.sparse.linalg as spla
    b = np.random.default_rng(1).normal(size=n)
    y = spla.spsolve_triangular(L.tocsr(), b[pivP], lower=True)
    z = spla.spsolve_triangular(U.tocsr(), y, lower=False)
    x = np.empty(n)
    x[pivQ] = z
    assert np.max(np.abs(M @ x - b)) <= 1e-9 * (abs(M).max() * np.max(np.abs(x)) + 1)


def _create(plan, Jv, trp, tci, tv, pivP, pivQ, nnzT=None):
    h = capi._vp()
    arr = [np.ascontiguousarray(a) for a in (Jv, trp, tci, tv, pivP, pivQ)]
    Jv, trp, tci, tv, pivP, pivQ = arr
    rc = capi.lib().pf_refact_create(
        plan._h, Jv.ctypes.data_as(capi._pd), int(trp[-1] if nnzT is None else nnzT),
        trp.ctypes.data_as(capi._pi32), tci.ctypes.data_as(capi._pi32),
        tv.ctypes.data_as(capi._pd), pivP.ctypes.data_as(capi._pi32),
        pivQ.ctypes.data_as(capi._pi32), ctypes.byref(h))
    msg = capi.lib().pf_last_error().decode()
    return rc, msg, h


def test_refact_create_argument_checks(ora):
    net = synth.tiny_grid(6)
    plan = Plan(net, host_only=True)
    M = _csr(ora, net, 2)
    rp, ci = plan.pattern()
    assert np.array_equal(rp, M.indptr) and np.array_equal(ci, M.indices)
    Jv = M.data
    trp, tci, tv, pivP, pivQ = host_lu(M.indptr, M.indices, M.data, plan.n)

    # well-formed factors: rejected only because the plan has no device side
    rc, msg, h = _create(plan, Jv, trp, tci, tv, pivP, pivQ)
    assert rc == capi.PF_EINVAL and "host-only" in msg and not h.value

    bad = pivP.copy()
    bad[0] = bad[1]
    rc, msg, _ = _create(plan, Jv, trp, tci, tv, bad, pivQ)
    assert rc == capi.PF_EINVAL and "permutation" in msg

    rc, msg, _ = _create(plan, Jv, trp, tci, tv, pivP, pivQ, nnzT=int(trp[-1]) - 1)
    assert rc == capi.PF_EINVAL and "nnzT" in msg

    # a row without its diagonal: drop the diagonal entry of row 0
    k = trp[0] + int(np.nonzero(tci[trp[0]:trp[1]] == 0)[0][0])
    tci2 = np.delete(tci, k)
    tv2 = np.delete(tv, k)
    trp2 = trp.copy()
    trp2[1:] -= 1
    rc, msg, _ = _create(plan, Jv, trp2, tci2, tv2, pivP, pivQ)
    assert rc == capi.PF_EINVAL and "diagonal" in msg

    # unsorted columns in the first row with two entries
    r = int(np.nonzero(np.diff(trp) >= 2)[0][0])
    tci3 = tci.copy()
    tci3[trp[r]], tci3[trp[r] + 1] = tci3[trp[r] + 1], tci3[trp[r]]
    rc, msg, _ = _create(plan, Jv, trp, tci3, tv, pivP, pivQ)
    assert rc == capi.PF_EINVAL and "increasing" in msg

    tci4 = tci.copy()
    tci4[-1] = plan.n
    rc, msg, _ = _create(plan, Jv, trp, tci4, tv, pivP, pivQ)
    assert rc == capi.PF_EINVAL and "range" in msg


def test_refact_create_rejects_batched_plan(ora):
    net = synth.tiny_grid(6)
    plan = Plan(net, host_only=True, batch=dict(n_inst=3))
    M = _csr(ora, net, 2)
    trp, tci, tv, pivP, pivQ = host_lu(M.indptr, M.indices, M.data, plan.n)
    rc, msg, _ = _create(plan, M.data, trp, tci, tv, pivP, pivQ)
    assert rc == capi.PF_EINVAL and "non-batched" in msg


def test_newton_device_argument_checks():
    L = capi.lib()
    assert L.pf_newton_device(None, None, None, None, None, None) == capi.PF_EINVAL
    assert L.pf_refact_solve(None, None, None, None) == capi.PF_EINVAL
    L.pf_refact_destroy(None)


def _eliminate(A, trp, tci):
    """Plain row-by-row elimination of the dense matrix A along the pattern
    (trp, tci); returns the factor values (a test reference)."""
    n = A.shape[0]
    T = np.zeros(trp[-1])
    diag = np.zeros(n, int)
    for r in range(n):
        cols = tci[trp[r]:trp[r + 1]]
        pos = {int(c): q for q, c in enumerate(cols)}
        row = A[r, cols].astype(float)
        diag[r] = trp[r] + pos[r]
        for q, k in enumerate(cols):
            if k >= r:
                break
            row[q] /= T[diag[k]]
            for f in range(diag[k] + 1, trp[k + 1]):
                row[pos[int(tci[f])]] -= row[q] * T[f]
        T[trp[r]:trp[r + 1]] = row
    return T


def test_symbolic_pattern_is_closed(ora):
    """The pattern from pf_lu_symbolic holds SuperLU's factors and every
    entry that elimination along it reaches: refactorising another Jacobian
    of the same grid along it with the same orders reproduces P J Q = L U."""
    net = synth.tiny_grid(3)
    J, _ = ora.jacobian(net, synth.random_states(net, seed=1))
    n = J.shape[0]
    trp, tci, tv, P, Q = host_lu(J.indptr, J.indices, J.data, n)
    import scipy.sparse.linalg as spla
    lu = spla.splu(J.tocsc(), permc_spec="COLAMD")
    assert trp[-1] >= lu.L.nnz + lu.U.nnz - n
    # the values placed in the pattern still factor J
    T = sp.csr_matrix((tv, tci, trp), shape=(n, n))
    L = sp.tril(T, -1) + sp.identity(n)
    U = sp.triu(T)
    assert abs(J[P][:, Q] - L @ U).max() <= 1e-12 * abs(J).max()
    J2, _ = ora.jacobian(net, synth.random_states(net, seed=2))
    A2 = J2.toarray()[P][:, Q]
    T2 = sp.csr_matrix((_eliminate(A2, trp, tci), tci, trp), shape=(n, n))
    L2 = sp.tril(T2, -1) + sp.identity(n)
    U2 = sp.triu(T2)
    assert np.abs(A2 - (L2 @ U2).toarray()).max() <= 1e-12 * np.abs(A2).max()


def test_symbolic_argument_checks():
    L = capi.lib()
    rp = np.array([0, 1, 2], np.int32)
    ci = np.array([0, 1], np.int32)
    p = np.array([0, 0], np.int32)
    q = np.array([0, 1], np.int32)
    nz = ctypes.c_int64(0)
    rc = L.pf_lu_symbolic(2, rp.ctypes.data_as(capi._pi32), ci.ctypes.data_as(capi._pi32),
                          p.ctypes.data_as(capi._pi32), q.ctypes.data_as(capi._pi32),
                          ctypes.byref(nz), None, None)
    assert rc == capi.PF_EINVAL and "permutation" in L.pf_last_error().decode()
    p[1] = 1
    rc = L.pf_lu_symbolic(2, rp.ctypes.data_as(capi._pi32), ci.ctypes.data_as(capi._pi32),
                          p.ctypes.data_as(capi._pi32), q.ctypes.data_as(capi._pi32),
                          ctypes.byref(nz), None, None)
    assert rc == capi.PF_OK and nz.value == 2


def test_batch_lu_create_checks(ora):
    net = synth.tiny_grid(6)
    single = Plan(net, host_only=True)
    batch = Plan(net, host_only=True, batch=dict(n_inst=5))
    M = _csr(ora, net, 2)
    trp, tci, _, pivP, pivQ = host_lu(M.indptr, M.indices, M.data, single.n)
    L = capi.lib()

    def create(plan, P=pivP):
        h = capi._vp()
        rc = L.pf_batch_lu_create(plan._h, int(trp[-1]), trp.ctypes.data_as(capi._pi32),
                                  tci.ctypes.data_as(capi._pi32), P.ctypes.data_as(capi._pi32),
                                  pivQ.ctypes.data_as(capi._pi32), ctypes.byref(h))
        return rc, L.pf_last_error().decode()

    # a single-instance plan is accepted (one instance); host-only plans are not
    rc, msg = create(single)
    assert rc == capi.PF_EINVAL and "host-only" in msg
    bad = pivP.copy()
    bad[0] = bad[1]
    rc, msg = create(batch, bad)
    assert rc == capi.PF_EINVAL and "permutation" in msg
    rc, msg = create(batch)
    assert rc == capi.PF_EINVAL and "host-only" in msg
    assert L.pf_newton_batch(None, None, None, None, None, None, None, None) == capi.PF_EINVAL
    assert L.pf_batch_lu_factor(None, None, None) == capi.PF_EINVAL
    L.pf_batch_lu_destroy(None)


@pytest.mark.parametrize("which", ["tiny", "everything", "10k"])
def test_jacobian_row_order_gives_robust_diagonal(ora, which):
    """Under pf_jacobian_row_order every diagonal entry of the Jacobian is a
    structural nonzero: constant +-1 on the control rows' new places, a sum
    over branches elsewhere.  An LU pivoting on that diagonal factors J."""
    from test_oracle_pins import _net_with_everything
    net = {"tiny": lambda: synth.tiny_grid(5), "everything": _net_with_everything,
           "10k": synth.grid_10k}[which]()
    p = Plan(net, host_only=True)
    R = p.jacobian_row_order()
    assert sorted(R) == list(range(p.n))
    J, _ = ora.jacobian(net, synth.random_states(net, seed=3))
    d = J.tocsr()[R].diagonal()
    assert np.all(d != 0)
    N = net.n_bus
    moved = R != np.arange(p.n)
    assert moved.sum() == 2 * (net.n_gen + net.n_slack)
    assert np.all(np.abs(d[moved]) == 1.0)
    trp, tci, tv, pivP, pivQ = host_lu(J.indptr, J.indices, J.data, p.n, row_order=R)
    assert np.array_equal(pivP, R[pivQ])          # pivots on the reordered diagonal
    T = sp.csr_matrix((tv, tci, trp), shape=(p.n, p.n))
    L = sp.tril(T, -1) + sp.identity(p.n)
    U = sp.triu(T)
    assert abs(J[pivP][:, pivQ] - L @ U).max() <= 1e-12 * abs(J).max()
    # multi-grid plans: the order stays inside each grid's block
    nets = [synth.tiny_grid(1, n_bus=30, n_branch=40, n_pv=4), net]
    m = Plan.multi(nets, host_only=True)
    Rm = m.jacobian_row_order()
    off = nets[0].n_var
    assert np.array_equal(Rm[off:] - off, R) and np.all(Rm[:off] < off)


def test_refact_rejects_pattern_without_fill(ora):
    """A numeric LU's pattern can miss fill entries; pf_refact_create
    rejects such a T instead of refactorising incompletely."""
    import scipy.sparse.linalg as spla
    net = synth.tiny_grid(3)
    plan = Plan(net, host_only=True)
    M = _csr(ora, net, 1)
    n = plan.n
    trp, tci, tv, pivP, pivQ = host_lu(M.indptr, M.indices, M.data, n,
                                       row_order=plan.jacobian_row_order())
    # drop one fill entry (a T entry that is not in P M Q)
    A = M[pivP][:, pivQ].tocsr()
    A.sort_indices()
    for r in range(n):
        cols = set(A.indices[A.indptr[r]:A.indptr[r + 1]])
        fill = [e for e in range(trp[r], trp[r + 1]) if tci[e] not in cols]
        if fill:
            e = fill[0]
            break
    tci2, tv2 = np.delete(tci, e), np.delete(tv, e)
    trp2 = trp.copy()
    trp2[r + 1:] -= 1
    rc, msg, _ = _create(plan, M.data, trp2, tci2, tv2, pivP, pivQ)
    assert rc == capi.PF_EINVAL and "fill" in msg
    rc, msg, _ = _create(plan, M.data, trp, tci, tv, pivP, pivQ)
    assert rc == capi.PF_EINVAL and "host-only" in msg


def test_batch_lu_binding_refusals():
    """The binding refuses, before any device work, a panel-layout plan and
    an instance other than 0 of a single-instance plan."""
    from paper_2011_11880_amd.api import BatchLU
    net = synth.tiny_grid(4)
    panels = Plan(net, host_only=True, batch=dict(n_inst=3, layout="panels"))
    with pytest.raises(ValueError, match="row layout"):
        BatchLU(panels, None)
    single = Plan(net, host_only=True)
    with pytest.raises(ValueError, match="instance 0"):
        BatchLU(single, None, inst=1)
