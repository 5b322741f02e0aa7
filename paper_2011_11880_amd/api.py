"""Torch-facing wrapper of libpf: plans, evaluation, Newton, adjoint.

PyTorch only provides device memory and streams here; every evaluation is a
libpf HIP kernel launched on the caller's current stream.  Tensors passed in
must be contiguous float64 CUDA tensors of the documented shapes.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

from . import capi
from .capi import check

_KIND = {0: "single", 1: "batch", 2: "multi"}


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class _NetStruct:
    """pf_network over the arrays of a network object (keeps them alive)."""

    INT = ("br_from", "br_to", "br_status", "load_bus", "pv_bus", "slack_bus", "shunt_bus")
    DBL = ("br_r", "br_x", "br_b", "br_tap", "br_shift_deg", "load_p", "load_q", "pv_p",
           "pv_v", "slack_v", "slack_theta", "shunt_g", "shunt_b")

    def __init__(self, net):
        self.keep = {}
        kw = {}
        for k in self.INT:
            a = getattr(net, k, None)
            if a is None:
                kw[k] = None
                continue
            a = _i32(a)
            self.keep[k] = a
            kw[k] = a.ctypes.data_as(capi._pi32)
        for k in self.DBL:
            a = _f64(getattr(net, k))
            self.keep[k] = a
            kw[k] = a.ctypes.data_as(capi._pd)
        self.s = capi.pf_network(
            n_bus=int(net.n_bus), n_branch=len(self.keep["br_from"]),
            n_load=len(self.keep["load_bus"]), n_pv=len(self.keep["pv_bus"]),
            n_slack=len(self.keep["slack_bus"]), n_shunt=len(self.keep["shunt_bus"]), **kw)


def params_vector(nets):
    """Host vector [r, x, b, tap, shift_deg, load_p, load_q] of one network,
    or of several concatenated in grid order (the layout of pf_set_params)."""
    if not isinstance(nets, (list, tuple)):
        nets = [nets]
    cat = np.concatenate
    return cat([cat([_f64(getattr(n, k)) for n in nets])
                for k in ("br_r", "br_x", "br_b", "br_tap", "br_shift_deg", "load_p", "load_q")])


def host_lu(rowptr, colidx, values, n, permc_spec=None, row_order=None):
    """One sparse LU of the CSR matrix M on the host (SuperLU), in the form
    the device re-factorisations take: (T_rowptr, T_colidx, T_val, pivP,
    pivQ) with T = (L - I) + U in CSR (sorted columns, the full symbolic
    pattern) and M[pivP][:, pivQ] = L U.  With ``row_order`` (a Jacobian's
    pf_jacobian_row_order) the rows are reordered first and pivots are taken
    on the diagonal, so that they stay usable for every matrix of the same
    pattern; otherwise partial pivoting.  ``permc_spec`` None picks the
    ordering: minimum degree on A + A^T with diagonal pivots (a third of
    COLAMD's elimination levels on power-flow Jacobians), unless the matrix
    has more than 9 nonzeros per row (well-meshed grids, where SuperLU's
    minimum degree takes minutes), and COLAMD otherwise."""
    rowptr, colidx = _i32(rowptr), _i32(colidx)
    lu, pivP, pivQ = _superlu(rowptr, colidx, values, n, permc_spec, row_order)
    trp, tci = lu_pattern(rowptr, colidx, n, pivP, pivQ)
    return trp, tci, _t_values(lu, trp, tci, n), pivP, pivQ


def _t_values(lu, trp, tci, n):
    """SuperLU's L and U as T = (L - I) + U on the full symbolic pattern
    (trp, tci): SuperLU's factors leave out entries whose values vanish for
    this matrix, which stay 0."""
    import scipy.sparse as sp
    T = (lu.L - sp.identity(n, format="csc") + lu.U).tocsr()
    T.sum_duplicates()
    T.sort_indices()
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(trp))
    keys = rows * n + tci
    trow = np.repeat(np.arange(n, dtype=np.int64), np.diff(T.indptr))
    tkeys = trow * n + T.indices
    pos = np.searchsorted(keys, tkeys)
    if np.any(pos >= keys.size) or np.any(keys[np.minimum(pos, keys.size - 1)] != tkeys):
        raise RuntimeError("the numeric LU has entries outside the symbolic pattern")
    tv = np.zeros(tci.size)
    tv[pos] = T.data
    return tv


def host_lu_switchable(rowptr, colidx, values, n, order, qv, permc_spec=None):
    """host_lu with pivots that survive reactive-limit switches: SuperLU's
    column order under pf_jacobian_switch_order's rows, each Q_g column moved
    ahead of its voltage column (switch_safe_pivots), then SuperLU again on
    the matrix so permuted, in that order with diagonal pivots, for the
    values of T.  ``values`` must have every PV unit under voltage control
    (+1 on the voltage column of its control row).  Returns (T_rowptr,
    T_colidx, T_val, pivP, pivQ) as host_lu."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    rowptr, colidx = _i32(rowptr), _i32(colidx)
    _, _, q0 = _superlu(rowptr, colidx, values, n, permc_spec, order)
    P1, Q1 = switch_safe_pivots(q0, order, qv)
    M = sp.csr_matrix((_f64(values), colidx, rowptr), shape=(n, n))
    lu = spla.splu(M[P1][:, Q1].tocsc(), permc_spec="NATURAL", diag_pivot_thresh=0.0)
    if not np.array_equal(lu.perm_r, lu.perm_c):
        raise RuntimeError("SuperLU pivoted off the diagonal of the switch-proof order")
    # SuperLU may post-order the columns of its elimination tree
    pivP = P1[np.argsort(lu.perm_r)].astype(np.int32)
    pivQ = Q1[np.argsort(lu.perm_c)].astype(np.int32)
    at = np.argsort(pivQ)
    qv = np.asarray(qv).reshape(-1, 2)
    if not np.all(at[qv[:, 0]] < at[qv[:, 1]]):
        raise RuntimeError("the elimination order lost a Q_g column's place before its voltage column")
    trp, tci = lu_pattern(rowptr, colidx, n, pivP, pivQ)
    return trp, tci, _t_values(lu, trp, tci, n), pivP, pivQ


def _superlu(rowptr, colidx, values, n, permc_spec, row_order):
    """SuperLU of M (CSR) as host_lu describes; returns (lu, pivP, pivQ)
    with M[pivP][:, pivQ] = L U."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    M = sp.csr_matrix((_f64(values), _i32(colidx), _i32(rowptr)), shape=(n, n))
    R = np.arange(n) if row_order is None else np.asarray(row_order, dtype=np.int64)
    thresh = 1.0 if row_order is None else 0.0
    if permc_spec is None:
        dense = M.nnz > 9 * n
        permc_spec = "MMD_AT_PLUS_A" if (row_order is not None and not dense) else "COLAMD"
    lu = spla.splu(M[R].tocsc(), permc_spec=permc_spec, diag_pivot_thresh=thresh)
    # SuperLU: Pr A Pc = L U with (Pr A)[perm_r[i]] = A[i], (A Pc)[:, perm_c[j]] = A[:, j],
    # here A = M[R]
    pivP = R[np.argsort(lu.perm_r)].astype(np.int32)
    pivQ = np.argsort(lu.perm_c).astype(np.int32)
    return lu, pivP, pivQ


def lu_pattern(rowptr, colidx, n, pivP, pivQ):
    """(T_rowptr, T_colidx): the filled pattern of the LU of M[pivP][:, pivQ]
    without pivoting (pf_lu_symbolic), M's pattern being (rowptr, colidx)."""
    rowptr, colidx = _i32(rowptr), _i32(colidx)
    pivP, pivQ = _i32(pivP), _i32(pivQ)
    nz = ctypes.c_int64(0)
    L = capi.lib()
    args = (n, rowptr.ctypes.data_as(capi._pi32), colidx.ctypes.data_as(capi._pi32),
            pivP.ctypes.data_as(capi._pi32), pivQ.ctypes.data_as(capi._pi32))
    check(L.pf_lu_symbolic(*args, ctypes.byref(nz), None, None))
    trp = np.empty(n + 1, np.int32)
    tci = np.empty(nz.value, np.int32)
    check(L.pf_lu_symbolic(*args, ctypes.byref(nz), trp.ctypes.data_as(capi._pi32),
                           tci.ctypes.data_as(capi._pi32)))
    return trp, tci


def switch_safe_pivots(pivQ, order, qv):
    """Pivots that survive reactive-limit switches, from a column order
    ``pivQ`` taken with diagonal pivots under the row order ``order`` of
    pf_jacobian_switch_order (row order[c] pivots on column c): every PV
    unit's Q_g column qv[2k] is moved to just before its bus voltage column
    qv[2k + 1] where the order had it later, so that elimination has added
    the bus's Q row to a held unit's control row before its voltage pivot.
    Returns (pivP, pivQ)."""
    pivQ = np.asarray(pivQ, dtype=np.int64)
    order = np.asarray(order, dtype=np.int64)
    qv = np.asarray(qv, dtype=np.int64).reshape(-1, 2)
    at = np.empty(pivQ.size, np.int64)
    at[pivQ] = np.arange(pivQ.size)
    key = at.astype(np.float64)
    late = at[qv[:, 0]] > at[qv[:, 1]]
    key[qv[late, 0]] = at[qv[late, 1]] - 0.5
    q = np.argsort(key, kind="stable")
    return order[q].astype(np.int32), q.astype(np.int32)


_ORDERS = {"input": capi.PF_ORDER_INPUT, "locality": capi.PF_ORDER_LOCALITY}


def _opts(host_only=False, device=None, schedule=None, q_limits=False, bus_order="input"):
    o = capi.pf_setup_opts()
    o.host_only = 1 if host_only else 0
    o.q_limits = 1 if q_limits else 0
    o.bus_order = _ORDERS[bus_order]
    o.device = -1 if device is None else int(device)
    if schedule:
        for k, v in schedule.items():
            setattr(o.sched, k, int(v))
    return o


def _ptr(t, numel, name):
    """Device pointer of a contiguous float64 CUDA tensor with ``numel`` elements."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_cuda:
        raise ValueError(f"{name} must live on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() != numel:
        raise ValueError(f"{name} has {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """A setup-time plan over one network, a batch, or several grids.

    ``Plan(net)``                         single instance
    ``Plan(net, batch=dict(n_inst=..., load_scale=..., pv_scale=..., outage=...))``
    ``Plan.multi([net0, net1, ...])``     block-diagonal multi-grid plan

    ``bus_order="locality"`` renumbers each grid's buses breadth-first at
    setup; bus-indexed vectors (x, F, the pattern) are then in the plan's
    order: ``to_plan`` / ``from_plan`` convert states and residuals.
    """

    def __init__(self, net=None, *, batch=None, host_only=False, device=None, schedule=None,
                 q_limits=False, bus_order="input", _handle=None, _grid_buses=None):
        self._h = None
        L = capi.lib()
        if _handle is not None:
            self._h = _handle
        else:
            ns = _NetStruct(net)
            _grid_buses = [int(net.n_bus)]
            opts = _opts(host_only, device, schedule, q_limits, bus_order)
            h = capi._P()
            if batch is None:
                check(L.pf_setup(ctypes.byref(ns.s), ctypes.byref(opts), ctypes.byref(h)))
            else:
                n_inst = int(batch["n_inst"])
                layout = {"rows": capi.PF_LAYOUT_ROWS, "panels": capi.PF_LAYOUT_PANELS}[
                    batch.get("layout", "rows")]
                spec = capi.pf_batch_spec(n_inst=n_inst,
                                          inst_stride=int(batch.get("inst_stride", 0)),
                                          layout=layout)
                keep = []
                if batch.get("load_scale") is not None:
                    a = _f64(batch["load_scale"])
                    if a.shape != (n_inst, ns.s.n_load):
                        raise ValueError("load_scale must be (n_inst, n_load)")
                    keep.append(a)
                    spec.load_scale = a.ctypes.data_as(capi._pd)
                if batch.get("pv_scale") is not None:
                    a = _f64(batch["pv_scale"])
                    if a.shape != (n_inst, ns.s.n_pv):
                        raise ValueError("pv_scale must be (n_inst, n_pv)")
                    keep.append(a)
                    spec.pv_scale = a.ctypes.data_as(capi._pd)
                if batch.get("outage") is not None:
                    a = _i32(batch["outage"])
                    if a.shape != (n_inst,):
                        raise ValueError("outage must be (n_inst,)")
                    keep.append(a)
                    spec.outage = a.ctypes.data_as(capi._pi32)
                check(L.pf_setup_batch(ctypes.byref(ns.s), ctypes.byref(spec),
                                       ctypes.byref(opts), ctypes.byref(h)))
            self._h = h
        self._load_info()
        self.device = device
        self._grid_buses = _grid_buses
        self._perm = None

    @classmethod
    def multi(cls, nets, *, host_only=False, device=None, schedule=None, q_limits=False,
              bus_order="input"):
        structs = [_NetStruct(n) for n in nets]
        arr = (capi.pf_network * len(structs))(*[s.s for s in structs])
        opts = _opts(host_only, device, schedule, q_limits, bus_order)
        h = capi._P()
        check(capi.lib().pf_setup_multi(arr, len(structs), ctypes.byref(opts), ctypes.byref(h)))
        p = cls(_handle=h, device=device, _grid_buses=[int(n.n_bus) for n in nets])
        xo = np.empty(len(structs) + 1, np.int64)
        jo = np.empty(len(structs) + 1, np.int64)
        check(capi.lib().pf_info_multi(h, xo.ctypes.data_as(capi._pi64),
                                       jo.ctypes.data_as(capi._pi64)))
        p.x_off, p.j_off = xo, jo
        return p

    # bus order --------------------------------------------------------------
    def bus_order(self):
        """pf_bus_order: input bus (within its grid) of every plan bus."""
        order = np.empty(self.info["n_bus"], np.int32)
        check(capi.lib().pf_bus_order(self._h, order.ctypes.data_as(capi._pi32)))
        return order

    def state_perm(self):
        """Index vector p of length n with x_plan = y_input[p] (angle and
        voltage blocks of each grid permuted, generator entries in place)."""
        if self._perm is None:
            order = self.bus_order().astype(np.int64)
            xo = getattr(self, "x_off", np.array([0, self.n], np.int64))
            perm = np.arange(self.n, dtype=np.int64)
            b0 = 0
            for g, N in enumerate(self._grid_buses or [self.info["n_bus"]]):
                o = order[b0:b0 + N]
                perm[xo[g]:xo[g] + N] = xo[g] + o
                perm[xo[g] + N:xo[g] + 2 * N] = xo[g] + N + o
                b0 += N
            self._perm = perm
        return self._perm

    def to_plan(self, y):
        """State(s) or residual(s) in input numbering (last axis n) -> plan order."""
        return np.ascontiguousarray(np.asarray(y)[..., self.state_perm()])

    def from_plan(self, x):
        """Plan order (last axis n) -> input numbering."""
        x = np.asarray(x)
        out = np.empty_like(x)
        out[..., self.state_perm()] = x
        return out

    def _load_info(self):
        inf = capi.pf_info_t()
        check(capi.lib().pf_info_ex(self._h, ctypes.byref(inf)))
        self.info = {k: int(getattr(inf, k)) for k, _ in inf._fields_}
        self.info["kind"] = _KIND[self.info["kind"]]
        self.n = self.info["n"]
        self.nnz = self.info["nnz"]
        self.n_inst = self.info["n_inst"]
        self.ld = self.info["inst_stride"]
        self.panels = self.info["layout"] == capi.PF_LAYOUT_PANELS
        self.n_params = self.info["n_params"]

    # lifetime ---------------------------------------------------------------
    def close(self):
        fd = getattr(self, "_fd", None)
        if fd is not None:
            capi.lib().pf_fdlf_destroy(fd[0])
            for lu in fd[1]:
                if lu is not None:
                    lu.close()
            self._fd = None
        for ref in getattr(self, "_lus", ()):
            lu = ref()
            if lu is not None:
                lu.close()
        if self._h is not None and self._h.value:
            capi.lib().pf_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # structure --------------------------------------------------------------
    def pattern(self):
        rp = np.empty(self.n + 1, np.int32)
        ci = np.empty(self.nnz, np.int32)
        check(capi.lib().pf_pattern(self._h, rp.ctypes.data_as(capi._pi32),
                                    ci.ctypes.data_as(capi._pi32)))
        return rp, ci

    @property
    def schedule(self):
        s = capi.pf_schedule()
        check(capi.lib().pf_get_schedule(self._h, ctypes.byref(s)))
        return s.as_dict()

    @schedule.setter
    def schedule(self, d):
        s = capi.pf_schedule(**{k: int(v) for k, v in d.items()})
        check(capi.lib().pf_set_schedule(self._h, ctypes.byref(s)))
        self._load_info()

    # evaluation -------------------------------------------------------------
    def _dev(self, t):
        import torch
        return t.device if t is not None else torch.device("cuda", self.device or 0)

    def eval(self, x, F=None, J=None, want_F=True, want_J=True):
        """Fused residual + Jacobian values for one state (pf_eval)."""
        import torch
        dev = self._dev(x)
        if want_F and F is None:
            F = torch.empty(self.n, dtype=torch.float64, device=dev)
        if want_J and J is None:
            J = torch.empty(self.nnz, dtype=torch.float64, device=dev)
        check(capi.lib().pf_eval(self._h, _ptr(x, self.n, "x"), _ptr(F, self.n, "F"),
                                 _ptr(J, self.nnz, "J"), _stream(dev)))
        return F, J

    def eval_residual(self, x, F=None):
        import torch
        dev = self._dev(x)
        F = torch.empty(self.n, dtype=torch.float64, device=dev) if F is None else F
        check(capi.lib().pf_eval_residual(self._h, _ptr(x, self.n, "x"), _ptr(F, self.n, "F"),
                                          _stream(dev)))
        return F

    def eval_jacobian(self, x, J=None):
        import torch
        dev = self._dev(x)
        J = torch.empty(self.nnz, dtype=torch.float64, device=dev) if J is None else J
        check(capi.lib().pf_eval_jacobian(self._h, _ptr(x, self.n, "x"),
                                          _ptr(J, self.nnz, "J"), _stream(dev)))
        return J

    def batch_shape(self, rows):
        """Tensor shape of a batched array with ``rows`` rows (n or nnz):
        (rows, ld) for the row layout, (P, rows, 64) for panels."""
        if self.panels:
            return (-(-self.n_inst // 64), rows, 64)
        return (rows, self.ld)

    def eval_batch(self, X, F=None, J=None, want_F=True, want_J=True):
        """Batched evaluation in the plan's layout: X, F of batch_shape(n),
        J of batch_shape(nnz), contiguous.  In the row layout X may instead
        be an instance view, (n_inst, n) with strides (1, ld) (see
        ``instances``); F and J are then allocated and returned as instance
        views too, and given ones must be views of the same kind."""
        import torch
        dev = self._dev(X)
        views = self._is_instance_view(X, self.n)
        sx, sj = self.batch_shape(self.n), self.batch_shape(self.nnz)
        if want_F and F is None:
            F = torch.empty(sx, dtype=torch.float64, device=dev)
            F = self.instances(F) if views else F
        if want_J and J is None:
            J = torch.empty(sj, dtype=torch.float64, device=dev)
            J = self.instances(J) if views else J
        check(capi.lib().pf_eval_batch(self._h, self._batch_ptr(X, self.n, "X", views),
                                       self._batch_ptr(F, self.n, "F", views),
                                       self._batch_ptr(J, self.nnz, "J", views), _stream(dev)))
        return F, J

    def instances(self, A):
        """Zero-copy (n_inst, rows) view of a device array in the row layout
        (rows, ld): row i is instance i, with stride ld between its entries."""
        if self.panels:
            raise ValueError("instance views need the row layout")
        if tuple(A.shape) != (A.shape[0], self.ld) or not A.is_contiguous():
            raise ValueError(f"expected a contiguous (rows, {self.ld}) array")
        return A[:, :self.n_inst].T

    def _is_instance_view(self, A, rows):
        return (not self.panels and A is not None and A.dim() == 2 and
                tuple(A.shape) == (self.n_inst, rows) and tuple(A.stride()) == (1, self.ld))

    def _batch_ptr(self, A, rows, name, views):
        """Device pointer of a batched array: the contiguous layout, or with
        ``views`` an instance view over a (rows, ld) allocation."""
        import math

        import torch
        if A is None:
            return None
        if not views:
            return _ptr(A, math.prod(self.batch_shape(rows)), name)
        if not self._is_instance_view(A, rows):
            raise ValueError(f"{name} must be an instance view ({self.n_inst}, {rows}) with "
                             f"strides (1, {self.ld})")
        if A.dtype != torch.float64 or not A.is_cuda:
            raise TypeError(f"{name} must be a float64 CUDA tensor")
        base = A.untyped_storage()
        if (A.storage_offset() + rows * self.ld) * 8 > base.nbytes():
            raise ValueError(f"{name}: the view's storage is smaller than ({rows}, {self.ld})")
        return ctypes.c_void_p(A.data_ptr())

    def to_batch(self, Y):
        """Host array (n_inst, n) of states -> numpy array in the plan's
        batched layout (padding columns zero)."""
        Y = np.asarray(Y, dtype=np.float64)
        I, n = Y.shape
        if self.panels:
            P = -(-I // 64)
            out = np.zeros((P * 64, n))
            out[:I] = Y
            return np.ascontiguousarray(out.reshape(P, 64, n).transpose(0, 2, 1))
        out = np.zeros((n, self.ld))
        out[:, :I] = Y.T
        return out

    def from_batch(self, A):
        """Batched array (layout of this plan) -> (n_inst, rows) host array."""
        A = A.cpu().numpy() if hasattr(A, "cpu") else np.asarray(A)
        if self.panels:
            P, rows, _ = A.shape
            return A.transpose(0, 2, 1).reshape(P * 64, rows)[:self.n_inst]
        return A[:, :self.n_inst].T

    def set_params(self, params):
        """Replace [r, x, b, tap, shift_deg, load_p, load_q] (device vector)."""
        dev = self._dev(params)
        check(capi.lib().pf_set_params(self._h, _ptr(params, self.n_params, "params"),
                                       _stream(dev)))

    def vjp(self, x, W, gx=None, gparam=None, want_gx=True, want_gparam=True):
        """J^T W and (dF/dparams)^T W for W of shape (n, k), cotangent-fastest."""
        import torch
        dev = self._dev(x)
        if W.dim() != 2 or W.shape[0] != self.n:
            raise ValueError("W must be (n, k)")
        k = int(W.shape[1])
        if want_gx and gx is None:
            gx = torch.empty((self.n, k), dtype=torch.float64, device=dev)
        if want_gparam and gparam is None:
            gparam = torch.empty((self.n_params, k), dtype=torch.float64, device=dev)
        check(capi.lib().pf_vjp(self._h, _ptr(x, self.n, "x"), _ptr(W, self.n * k, "W"), k,
                                _ptr(gx, self.n * k, "gx"),
                                _ptr(gparam, self.n_params * k, "gparam"), _stream(dev)))
        return gx, gparam

    def autotune(self, x, F=None, J=None, reps=5, cache=None):
        """Time every candidate schedule on these buffers and keep the fastest
        (pf_autotune).  ``cache``: path of a tune-cache file
        (pf_autotune_cached; a hit applies the stored schedule without
        timing, a miss appends the result); None leaves the choice to the
        PF_TUNE_CACHE environment variable.  ``self.tune_hit`` records
        whether the schedule came from the cache."""
        dev = self._dev(x)
        best = capi.pf_schedule()
        if self.info["kind"] == "batch":
            import math
            sx, sj = self.batch_shape(self.n), self.batch_shape(self.nnz)
            xs = _ptr(x, math.prod(sx), "X")
            Fs = _ptr(F, math.prod(sx), "F")
            Js = _ptr(J, math.prod(sj), "J")
        else:
            xs, Fs, Js = _ptr(x, self.n, "x"), _ptr(F, self.n, "F"), _ptr(J, self.nnz, "J")
        hit = ctypes.c_int32(0)
        path = os.environ.get("PF_TUNE_CACHE", "") if cache is None else os.fspath(cache)
        check(capi.lib().pf_autotune_cached(self._h, xs, Fs, Js, int(reps), _stream(dev),
                                            path.encode() if path else None,
                                            ctypes.byref(best), ctypes.byref(hit)))
        self.tune_hit = bool(hit.value)
        self._load_info()
        return best.as_dict()

    def _newton_opts(self, tol, max_iter, q_min=None, q_max=None, check_below=1e-3,
                     switch_tol=1e-9):
        """pf_newton_opts, with the reactive limits when q_min/q_max are given
        (one entry per PV unit).  Returns (opts, arrays to keep alive)."""
        opts = capi.pf_newton_opts(tol=float(tol), max_iter=int(max_iter))
        if (q_min is None) != (q_max is None):
            raise ValueError("q_min and q_max go together")
        if q_min is None:
            return opts, ()
        lo, hi = _f64(q_min), _f64(q_max)
        if lo.shape != (self.info["n_pv"],) or hi.shape != lo.shape:
            raise ValueError("q_min and q_max need one entry per PV unit")
        opts.q_min = lo.ctypes.data_as(capi._pd)
        opts.q_max = hi.ctypes.data_as(capi._pd)
        opts.q_check_below = float(check_below)
        opts.q_switch_tol = float(switch_tol)
        return opts, (lo, hi)

    def newton(self, x, solve=None, tol=1e-10, max_iter=10, q_min=None, q_max=None,
               check_below=1e-3, switch_tol=1e-9):
        """Newton power flow with a host sparse solve (scipy SuperLU by default).
        ``x`` (device) is updated in place.  With ``q_min``/``q_max`` (one
        entry per PV unit) the reactive limits are checked inside the
        iterations, at every iterate whose mismatch is below ``check_below``
        (pf_newton's limit checks); the report then lists the units switched
        at each iterate.  Returns a dict report; raises PFError on failure
        except non-convergence (report['converged'] False)."""
        import scipy.sparse as sp
        import scipy.sparse.linalg as spla

        n = self.n
        errors = []

        def default_solve(rp, ci, jv, rhs):
            A = sp.csr_matrix((jv, ci, rp), shape=(n, n))
            return spla.spsolve(A.tocsc(), rhs)

        user_solve = solve or default_solve

        @capi.pf_linsolve_fn
        def cb(user, nn, rowptr, colidx, jv, rhs, dx):
            try:
                m = int(nn)
                rp = np.ctypeslib.as_array(rowptr, shape=(m + 1,))
                nz = int(rp[-1])
                ci = np.ctypeslib.as_array(colidx, shape=(nz,))
                J = np.ctypeslib.as_array(jv, shape=(nz,))
                b = np.ctypeslib.as_array(rhs, shape=(m,))
                out = np.ctypeslib.as_array(dx, shape=(m,))
                sol = np.asarray(user_solve(rp.copy(), ci.copy(), J.copy(), b.copy()))
                if sol.shape != (m,) or not np.all(np.isfinite(sol)):
                    return 1
                out[:] = sol
                return 0
            except Exception as ex:  # reported through PF_ESOLVE
                errors.append(ex)
                return 2

        opts, _keep = self._newton_opts(tol, max_iter, q_min, q_max, check_below, switch_tol)
        rep = capi.pf_newton_report()
        # pf_newton works on the null stream; whatever the caller's stream
        # still has to write into x must land first
        import torch
        torch.cuda.current_stream(self._dev(x)).synchronize()
        rc = capi.lib().pf_newton(self._h, _ptr(x, n, "x"), ctypes.byref(opts), cb, None,
                                  ctypes.byref(rep))
        if rc not in (capi.PF_OK, capi.PF_ENOCONV):
            check(rc)
        it = int(rep.iterations)
        return {"iterations": it, "converged": bool(rep.converged),
                "norms": [float(v) for v in rep.norm[:min(it + 1, 65)]],
                "switched": [int(v) for v in rep.switched[:min(it + 1, 65)]],
                "n_switches": int(rep.n_switches),
                "t_eval_s": rep.t_eval_s, "t_solve_s": rep.t_solve_s,
                "t_total_s": rep.t_total_s, "solver_errors": errors}

    # reactive limits ------------------------------------------------------
    def set_gen_modes(self, mode, q_target=None):
        """Hold PV units at reactive targets (mode 1) or return them to
        voltage control (mode 0); arrays over the plan's PV units."""
        m = _i32(mode)
        if m.shape != (self.info["n_pv"],):
            raise ValueError("mode must have one entry per PV unit")
        qt = None if q_target is None else _f64(q_target)
        if qt is not None and qt.shape != m.shape:
            raise ValueError("q_target must match mode")
        check(capi.lib().pf_set_gen_modes(self._h, m.ctypes.data_as(capi._pi32),
                                          None if qt is None else qt.ctypes.data_as(capi._pd)))

    def gen_modes(self):
        """(mode, q_target) of the plan's PV units."""
        k = self.info["n_pv"]
        m = np.zeros(k, np.int32)
        qt = np.zeros(k)
        check(capi.lib().pf_get_gen_modes(self._h, m.ctypes.data_as(capi._pi32),
                                          qt.ctypes.data_as(capi._pd)))
        return m, qt

    def q_limit_check(self, x, q_min, q_max, tol=1e-9):
        """One reactive-limit check at the state x (pf_q_limit_check); returns
        the number of PV units that switched."""
        lo, hi = _f64(q_min), _f64(q_max)
        ns = ctypes.c_int32(0)
        check(capi.lib().pf_q_limit_check(self._h, _ptr(x, self.n, "x"),
                                          lo.ctypes.data_as(capi._pd),
                                          hi.ctypes.data_as(capi._pd), float(tol),
                                          ctypes.byref(ns),
                                          None if x is None else _stream(self._dev(x))))
        return int(ns.value)

    def newton_qlim(self, x, q_min, q_max, device=False, tol=1e-10, max_iter=10,
                    max_outer=10, switch_tol=1e-9, inner=False, check_below=1e-3):
        """Newton power flow with reactive limits: solve, check the limits,
        and solve again from the last state until no unit switches.
        ``device``: False solves on the host; True runs every step on the
        device with this library's factorisation (the plan as one instance);
        "rocsolver" with rocSOLVER's re-factorisation.  After a switch a held
        row's nonzero moves from the V column to the Q_g column, so a device
        path takes a fresh host LU (new pivots) for the next solve.
        ``inner``: one Newton run that checks the limits inside its
        iterations instead (``max_iter`` bounds the whole run): on the host
        solve, or on the device (either factorisation) with pivots that
        survive a switch, so one host LU serves the whole run.  ``x`` is
        updated in place."""
        if device not in (False, True, "rocsolver"):
            raise ValueError("device must be False, True or 'rocsolver'")
        if inner:
            if device == "rocsolver":
                lu = DeviceLU(self, x, switchable=True)
                try:
                    rep = self.newton_device(x, lu, tol=tol, max_iter=max_iter, q_min=q_min,
                                             q_max=q_max, check_below=check_below,
                                             switch_tol=switch_tol)
                finally:
                    lu.close()
            elif device:
                lu = BatchLU(self, x, switchable=True)
                try:
                    rep = self.newton_batch(x, lu, tol=tol, max_iter=max_iter, q_min=q_min,
                                            q_max=q_max, check_below=check_below,
                                            switch_tol=switch_tol)
                finally:
                    lu.close()
                rep["converged"] = rep["n_converged"] == 1
            else:
                rep = self.newton(x, tol=tol, max_iter=max_iter, q_min=q_min, q_max=q_max,
                                  check_below=check_below, switch_tol=switch_tol)
            return {"converged": rep["converged"], "outer": 1, "rounds": [rep]}
        rounds = []
        lu = None
        for outer in range(1, max_outer + 1):
            if device == "rocsolver":
                if lu is None:
                    lu = DeviceLU(self, x)
                rep = self.newton_device(x, lu, tol=tol, max_iter=max_iter)
            elif device:
                if lu is None:
                    lu = BatchLU(self, x)
                rep = self.newton_batch(x, lu, tol=tol, max_iter=max_iter)
                rep["converged"] = rep["n_converged"] == 1
            else:
                rep = self.newton(x, tol=tol, max_iter=max_iter)
            rounds.append(rep)
            if not rep["converged"]:
                return {"converged": False, "outer": outer, "rounds": rounds}
            if self.q_limit_check(x, q_min, q_max, switch_tol) == 0:
                return {"converged": True, "outer": outer, "rounds": rounds}
            if lu is not None:
                lu.close()
                lu = None
        return {"converged": False, "outer": max_outer, "rounds": rounds}

    # fast decoupled method -------------------------------------------------
    def fdlf_matrices(self):
        """(B', B'', buses of B' rows, buses of B'' rows) as scipy CSR
        (pf_fdlf_matrices)."""
        import scipy.sparse as sp
        L = capi.lib()
        n1, n2 = ctypes.c_int64(0), ctypes.c_int64(0)
        check(L.pf_fdlf_matrices(self._h, ctypes.byref(n1), None, None, None, None,
                                 ctypes.byref(n2), None, None, None, None))
        N = self.info["n_bus"]
        m1 = N - self.info["n_slack"]
        m2 = N - self.info["n_pv"] - self.info["n_slack"]
        a = [np.zeros(m1 + 1, np.int32), np.zeros(n1.value, np.int32), np.zeros(n1.value),
             np.zeros(m1, np.int32)]
        b = [np.zeros(m2 + 1, np.int32), np.zeros(n2.value, np.int32), np.zeros(n2.value),
             np.zeros(m2, np.int32)]
        P = (capi._pi32, capi._pi32, capi._pd, capi._pi32)
        check(L.pf_fdlf_matrices(self._h, None, *[v.ctypes.data_as(t) for v, t in zip(a, P)],
                                 None, *[v.ctypes.data_as(t) for v, t in zip(b, P)]))
        Bp = sp.csr_matrix((a[2], a[1], a[0]), shape=(m1, m1))
        Bpp = sp.csr_matrix((b[2], b[1], b[0]), shape=(m2, m2))
        return Bp, Bpp, a[3], b[3]

    def fdlf(self, x, tol=1e-10, max_iter=50):
        """Fast decoupled power flow (XB) with every iteration on the device
        (pf_fdlf_solve).  B' and B'' are factorised once per plan (host LU,
        then constant device factors).  ``x`` is updated in place."""
        import time
        t_setup = 0.0
        if getattr(self, "_fd", None) is None:
            t0 = time.perf_counter()
            Bp, Bpp, _, _ = self.fdlf_matrices()
            dev = self.device if self.device is not None else -1
            lus = [DeviceSparseLU(M, dev) if M.shape[0] else None for M in (Bp, Bpp)]
            h = capi._vp()
            check(capi.lib().pf_fdlf_create(self._h, lus[0] and lus[0]._h,
                                            lus[1] and lus[1]._h, ctypes.byref(h)))
            self._fd = (h, lus)
            t_setup = time.perf_counter() - t0
        opts = capi.pf_newton_opts(tol=float(tol), max_iter=int(max_iter))
        rep = capi.pf_newton_report()
        rc = capi.lib().pf_fdlf_solve(self._fd[0], _ptr(x, self.n, "x"), ctypes.byref(opts),
                                      ctypes.byref(rep), _stream(self._dev(x)))
        if rc not in (capi.PF_OK, capi.PF_ENOCONV):
            check(rc)
        it = int(rep.iterations)
        conv = rc == capi.PF_OK
        return {"iterations": it, "converged": conv,
                "norms": [float(v) for v in rep.norm[:min(it + 2 if conv else it + 1, 65)]],
                "t_eval_s": rep.t_eval_s, "t_solve_s": rep.t_solve_s,
                "t_total_s": rep.t_total_s, "t_setup_s": t_setup}

    # batched Newton ---------------------------------------------------------
    def batch_lu(self, X, inst=0, permc_spec=None):
        """A BatchLU for this plan: pattern and pivots from one host LU of
        instance ``inst``'s Jacobian at the batched state X.  A single-instance
        or multi-grid plan is one instance (X of shape (n,)); its newton_batch
        is then a device-resident Newton on this library's own factorisation."""
        return BatchLU(self, X, inst=inst, permc_spec=permc_spec)

    def _lu_shape(self, rows):
        return self.batch_shape(rows) if self.info["kind"] == "batch" else (rows,)

    def newton_batch(self, X, lu=None, tol=1e-10, max_iter=10, q_min=None, q_max=None,
                     check_below=1e-3, switch_tol=1e-9):
        """Newton power flow for every instance of this plan at once
        (pf_newton_batch).  X (batch_shape(n), or (n,) for a plan of one
        instance) is updated in place.  With ``q_min``/``q_max`` (plan of one
        instance set up with q_limits) the reactive limits are checked inside
        the iterations as in ``newton``; ``lu`` must then be a BatchLU made
        with switchable=True (made so when not given).  Returns a dict report
        with per-instance step counts and last norms."""
        opts, _keep = self._newton_opts(tol, max_iter, q_min, q_max, check_below, switch_tol)
        if lu is None:
            lu = BatchLU(self, X, switchable=q_min is not None)
        I = self.n_inst
        its = np.zeros(I, np.int32)
        nrm = np.zeros(I)
        rep = capi.pf_newton_report()
        import math
        rc = capi.lib().pf_newton_batch(self._h, lu._h,
                                        _ptr(X, math.prod(self._lu_shape(self.n)), "X"),
                                        ctypes.byref(opts), its.ctypes.data_as(capi._pi32),
                                        nrm.ctypes.data_as(capi._pd), ctypes.byref(rep),
                                        _stream(self._dev(X)))
        if rc not in (capi.PF_OK, capi.PF_ENOCONV):
            check(rc)
        it = int(rep.iterations)
        return {"iterations": it, "n_converged": int(rep.converged),
                "inst_iterations": its, "inst_norm": nrm,
                "norms": [float(v) for v in rep.norm[:min(it + 1, 65)]],
                "switched": [int(v) for v in rep.switched[:min(it + 1, 65)]],
                "n_switches": int(rep.n_switches),
                "t_eval_s": rep.t_eval_s, "t_solve_s": rep.t_solve_s,
                "t_total_s": rep.t_total_s, "nnz_lu": lu.nnzT}

    def jacobian_row_order(self):
        """pf_jacobian_row_order: the row order under which the Jacobian's
        diagonal pivots survive outages and later iterates."""
        order = np.empty(self.n, np.int32)
        check(capi.lib().pf_jacobian_row_order(self._h, order.ctypes.data_as(capi._pi32)))
        return order

    def jacobian_switch_order(self):
        """pf_jacobian_switch_order: (order [n], qv [n_pv, 2]) -- the row
        order that pairs every PV unit's bus Q row with its Q_g column and its
        control row with the bus voltage column, whatever the unit's mode,
        and each unit's (Q_g column, voltage column)."""
        order = np.empty(self.n, np.int32)
        qv = np.empty((self.info["n_pv"], 2), np.int32)
        check(capi.lib().pf_jacobian_switch_order(self._h, order.ctypes.data_as(capi._pi32),
                                                  qv.ctypes.data_as(capi._pi32)))
        return order, qv

    def device_lu(self, x, permc_spec=None):
        """A DeviceLU for this plan, its pattern and pivots taken from one host
        LU of the Jacobian at ``x`` (device [n])."""
        return DeviceLU(self, x, permc_spec=permc_spec)

    def newton_device(self, x, lu=None, tol=1e-10, max_iter=10, q_min=None, q_max=None,
                      check_below=1e-3, switch_tol=1e-9):
        """Newton power flow with every step on the device (pf_newton_device).
        ``lu`` (a DeviceLU of this plan) is created at ``x`` when not given.
        With ``q_min``/``q_max`` the reactive limits are checked inside the
        iterations as in ``newton``; ``lu`` must then be a DeviceLU made with
        switchable=True (made so when not given).  ``x`` is updated in place.
        Returns a dict report (as ``newton``, plus the time of the host LU if
        one was made)."""
        import time
        opts, _keep = self._newton_opts(tol, max_iter, q_min, q_max, check_below, switch_tol)
        t_lu = 0.0
        if lu is None:
            t0 = time.perf_counter()
            lu = DeviceLU(self, x, switchable=q_min is not None)
            t_lu = time.perf_counter() - t0
        rep = capi.pf_newton_report()
        rc = capi.lib().pf_newton_device(self._h, lu._h, _ptr(x, self.n, "x"),
                                         ctypes.byref(opts), ctypes.byref(rep),
                                         _stream(self._dev(x)))
        if rc not in (capi.PF_OK, capi.PF_ENOCONV):
            check(rc)
        it = int(rep.iterations)
        return {"iterations": it, "converged": bool(rep.converged),
                "norms": [float(v) for v in rep.norm[:min(it + 1, 65)]],
                "switched": [int(v) for v in rep.switched[:min(it + 1, 65)]],
                "n_switches": int(rep.n_switches),
                "t_eval_s": rep.t_eval_s, "t_solve_s": rep.t_solve_s,
                "t_total_s": rep.t_total_s, "t_host_lu_s": t_lu, "nnz_lu": lu.nnzT}


class DeviceLU:
    """Device re-factorisation (pf_refact_*) bound to one non-batched plan:
    pattern and pivots from one host LU of the plan's Jacobian at ``x``,
    every later factorisation and solve on the GPU (rocSOLVER csrrf)."""

    def __init__(self, plan, x, permc_spec=None, switchable=False):
        """``switchable``: pivots that stay usable when PV units switch mode
        (pf_jacobian_switch_order; plan set up with q_limits), which
        newton_device needs to check reactive limits inside its
        iterations."""
        import weakref
        self.plan = plan
        self._h = None
        J = plan.eval_jacobian(x)
        Jh = J.cpu().numpy()
        rp, ci = plan.pattern()
        if switchable:
            order, qv, Jh = _voltage_control_values(plan, Jh)
            trp, tci, tv, pivP, pivQ = host_lu_switchable(rp, ci, Jh, plan.n, order, qv,
                                                          permc_spec)
        else:
            trp, tci, tv, pivP, pivQ = host_lu(rp, ci, Jh, plan.n, permc_spec,
                                               row_order=plan.jacobian_row_order())
        self.switchable = bool(switchable)
        self.nnzT = int(trp[-1])
        h = capi._vp()
        check(capi.lib().pf_refact_create(
            plan._h, Jh.ctypes.data_as(capi._pd), self.nnzT, trp.ctypes.data_as(capi._pi32),
            tci.ctypes.data_as(capi._pi32), tv.ctypes.data_as(capi._pd),
            pivP.ctypes.data_as(capi._pi32), pivQ.ctypes.data_as(capi._pi32), ctypes.byref(h)))
        self._h = h
        if not hasattr(plan, "_lus"):
            plan._lus = []
        plan._lus.append(weakref.ref(self))

    def solve(self, J, b):
        """Refactorise with the Jacobian values J (device [nnz]) and solve
        J y = b in place (b: device [n]); returns b."""
        n, nnz = self.plan.n, self.plan.nnz
        check(capi.lib().pf_refact_solve(self._h, _ptr(J, nnz, "J"), _ptr(b, n, "b"),
                                         _stream(b.device)))
        return b

    def close(self):
        if self._h is not None and self._h.value:
            capi.lib().pf_refact_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class DeviceSparseLU:
    """Constant device factorisation of a host CSR matrix (pf_lu_*): one host
    LU (SuperLU) fixes the factors, solves run on the GPU."""

    def __init__(self, M, device=-1, permc_spec=None):
        M = M.tocsr()
        M.sort_indices()
        n = M.shape[0]
        rp, ci, v = M.indptr.astype(np.int32), M.indices.astype(np.int32), _f64(M.data)
        trp, tci, tv, pivP, pivQ = host_lu(rp, ci, v, n, permc_spec)
        self.n = n
        self._h = None
        h = capi._vp()
        check(capi.lib().pf_lu_create(
            int(device), n, int(M.nnz), rp.ctypes.data_as(capi._pi32),
            ci.ctypes.data_as(capi._pi32), v.ctypes.data_as(capi._pd), int(trp[-1]),
            trp.ctypes.data_as(capi._pi32), tci.ctypes.data_as(capi._pi32),
            tv.ctypes.data_as(capi._pd), pivP.ctypes.data_as(capi._pi32),
            pivQ.ctypes.data_as(capi._pi32), ctypes.byref(h)))
        self._h = h

    def solve(self, b, noalloc=False):
        """Solve M y = b in place (b: device [n]); returns b.  ``noalloc``:
        pf_lu_solve_noalloc, the working vector in the library's static
        device array."""
        fn = capi.lib().pf_lu_solve_noalloc if noalloc else capi.lib().pf_lu_solve
        check(fn(self._h, _ptr(b, self.n, "b"), _stream(b.device)))
        return b

    def close(self):
        if self._h is not None and self._h.value:
            capi.lib().pf_lu_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _voltage_control_values(plan, Jh):
    """(order, qv, values): pf_jacobian_switch_order's row order and pairs,
    and a copy of the Jacobian values Jh with every PV unit's control row
    as under voltage control (+1 on the voltage column, 0 on Q_g), on which
    SuperLU's diagonal pivots in that order are nonzero."""
    rp, ci = plan.pattern()
    order, qv = plan.jacobian_switch_order()
    rows = qv[:, 0].astype(np.int64)
    if not (np.array_equal(ci[rp[rows]], qv[:, 1]) and np.array_equal(ci[rp[rows] + 1], qv[:, 0])):
        raise RuntimeError("unexpected control-row pattern")
    v = np.array(Jh, dtype=np.float64)
    v[rp[rows]] = 1.0
    v[rp[rows] + 1] = 0.0
    return order, qv, v


class BatchLU:
    """Batched factorisation (pf_batch_lu_*) of every instance of a plan
    along the pattern and pivots of one host LU of one instance's Jacobian
    (a single-instance or multi-grid plan is one instance)."""

    def __init__(self, plan, X, inst=0, permc_spec=None, switchable=False):
        """``switchable``: pivots that stay usable when PV units switch mode
        (pf_jacobian_switch_order; plan of one instance set up with
        q_limits), which newton_batch needs to check reactive limits inside
        its iterations."""
        import weakref
        if plan.panels:
            raise ValueError("the batched factorisation needs the row layout")
        self.plan = plan
        self._h = None
        if plan.info["kind"] == "batch":
            if switchable:
                raise ValueError("reactive-limit switches need a plan of one instance")
            _, J = plan.eval_batch(X, want_F=False)
            Jh = plan.from_batch(J)[inst]
        else:
            if inst != 0:
                raise ValueError("a single-instance plan has instance 0 only")
            _, J = plan.eval(X, want_F=False)
            Jh = J.cpu().numpy()
        rp, ci = plan.pattern()
        if switchable:
            order, qv, Jh = _voltage_control_values(plan, Jh)
            # only SuperLU's column order is kept
            _, _, q0 = _superlu(rp, ci, Jh, plan.n, permc_spec, order)
            pivP, pivQ = switch_safe_pivots(q0, order, qv)
            trp, tci = lu_pattern(rp, ci, plan.n, pivP, pivQ)
        else:
            trp, tci, _, pivP, pivQ = host_lu(rp, ci, Jh, plan.n, permc_spec,
                                              row_order=plan.jacobian_row_order())
        self.switchable = bool(switchable)
        self.nnzT = int(trp[-1])
        h = capi._vp()
        check(capi.lib().pf_batch_lu_create(
            plan._h, self.nnzT, trp.ctypes.data_as(capi._pi32), tci.ctypes.data_as(capi._pi32),
            pivP.ctypes.data_as(capi._pi32), pivQ.ctypes.data_as(capi._pi32), ctypes.byref(h)))
        self._h = h
        if not hasattr(plan, "_lus"):
            plan._lus = []
        plan._lus.append(weakref.ref(self))

    def factor(self, J):
        """Factorise every instance from the batched Jacobian J."""
        import math
        p = self.plan
        check(capi.lib().pf_batch_lu_factor(self._h, _ptr(J, math.prod(p._lu_shape(p.nnz)), "J"),
                                            _stream(J.device)))

    def solve(self, B, out=None):
        """Per-instance solves J_i x = B[:, i] after factor(); returns out."""
        import math

        import torch
        p = self.plan
        sh = p._lu_shape(p.n)
        if out is None:
            out = torch.empty(sh, dtype=torch.float64, device=B.device)
        check(capi.lib().pf_batch_lu_solve(self._h, _ptr(B, math.prod(sh), "B"),
                                           _ptr(out, math.prod(sh), "out"), _stream(B.device)))
        return out

    def close(self):
        if self._h is not None and self._h.value:
            capi.lib().pf_batch_lu_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
