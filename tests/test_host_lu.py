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
