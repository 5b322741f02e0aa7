"""Python side of the CPU oracle (TEST INFRASTRUCTURE).

Loads ``liboracle.so`` (plain C, FP64, built from ``pf_oracle.c``) and adds
the steps that are library primitives: summing Jacobian triplets into CSR
(Section III: triplets assembled into a sparse matrix), the explicit
transposed-Jacobian product, and a Newton loop whose linear solve is
scipy's sparse LU (tasks 1-4 of Section I).

Only tests, the package smoke check and the benchmark's CPU baseline may use
this module.  It shares no code with the HIP library: it reads networks as
the plain arrays of :class:`paper_2011_11880_amd.synth.Network`.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pf_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

_i = ctypes.c_int
_pi = ctypes.POINTER(ctypes.c_int)
_pd = ctypes.POINTER(ctypes.c_double)


class _Topo(ctypes.Structure):
    _fields_ = [("n_bus", _i), ("n_branch", _i), ("n_load", _i), ("n_pv", _i),
                ("n_slack", _i), ("n_shunt", _i),
                ("br_from", _pi), ("br_to", _pi), ("br_status", _pi),
                ("load_bus", _pi), ("pv_bus", _pi), ("slack_bus", _pi),
                ("shunt_bus", _pi), ("pv_mode", _pi)]


class _Data(ctypes.Structure):
    _fields_ = [(k, _pd) for k in (
        "br_r", "br_x", "br_b", "br_tap", "br_shift_deg", "load_p", "load_q",
        "pv_p", "pv_v", "slack_v", "slack_theta", "shunt_g", "shunt_b", "pv_qtarget")]


PARAM_FIELDS = ("br_r", "br_x", "br_b", "br_tap", "br_shift_deg", "load_p",
                "load_q", "pv_p", "pv_v", "slack_v", "slack_theta",
                "shunt_g", "shunt_b")


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (no contraction of a*b+c into FMA)."""
    if force or not os.path.exists(_LIB) or \
            os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                         os.path.getmtime(os.path.join(_HERE, "ora_core.inc"))):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c99",
                               "-fPIC", "-shared", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load(path):
    L = ctypes.CDLL(path)
    L.ora_residual.argtypes = [ctypes.POINTER(_Topo), ctypes.POINTER(_Data),
                               _pd, _pd, _pd]
    L.ora_residual_cs.argtypes = [ctypes.POINTER(_Topo)] + [_pd] * 16
    L.ora_branch_flows.argtypes = [ctypes.c_double] * 9 + [_pd]
    L.ora_jacobian_size.argtypes = [ctypes.POINTER(_Topo)]
    L.ora_jacobian_size.restype = ctypes.c_long
    L.ora_jacobian.argtypes = [ctypes.POINTER(_Topo), ctypes.POINTER(_Data),
                               _pd, _pi, _pi, _pd, _pd]
    L.ora_jacobian.restype = ctypes.c_long
    L.ora_vjp_params.argtypes = [ctypes.POINTER(_Topo), ctypes.POINTER(_Data),
                                 _pd, _pd] + [_pd] * 7
    L.ora_vjp_params_scale.argtypes = [ctypes.POINTER(_Topo), ctypes.POINTER(_Data),
                                       _pd, _pd] + [_pd] * 5
    return L


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = _load(_LIB)
    return _lib


def use_library(path):
    """Point this module at another build of the oracle (mutation tests load
    deliberately broken copies); ``None`` restores the real one.  Returns the
    previous handle."""
    global _lib
    prev = _lib
    _lib = None if path is None else _load(path)
    return prev


def _ip(a):
    return a.ctypes.data_as(_pi)


def _dp(a):
    return a.ctypes.data_as(_pd)


class _Bound:
    """Keeps the numpy arrays behind the ctypes structures alive."""

    def __init__(self, net, data=None, modes=None):
        self.arrs = {}
        keep = self.arrs

        def I(name):
            a = np.ascontiguousarray(getattr(net, name), dtype=np.int32)
            keep[name] = a
            return _ip(a)

        def D(name, src):
            a = np.ascontiguousarray(src, dtype=np.float64)
            keep[name] = a
            return _dp(a)

        # modes = (pv_mode, pv_qtarget): per PV generator 0 = voltage
        # control, 1 = reactive output held at pv_qtarget
        if modes is None:
            mode = np.zeros(net.n_pv, np.int32)
            qt = np.zeros(net.n_pv)
        else:
            mode = np.asarray(modes[0], dtype=np.int32)
            qt = np.asarray(modes[1], dtype=np.float64)
            assert mode.shape == (net.n_pv,) and qt.shape == (net.n_pv,)
        mode = np.ascontiguousarray(mode)
        keep["pv_mode"] = mode
        self.topo = _Topo(net.n_bus, net.n_branch, net.n_load, net.n_pv,
                          net.n_slack, net.n_shunt, I("br_from"), I("br_to"),
                          I("br_status"), I("load_bus"), I("pv_bus"),
                          I("slack_bus"), I("shunt_bus"), _ip(mode))
        data = data or {}
        self.data = _Data(*[D(k, data.get(k, getattr(net, k))) for k in PARAM_FIELDS],
                          D("pv_qtarget", qt))


def n_var(net) -> int:
    return 2 * net.n_bus + net.n_pv + 2 * net.n_slack


def residual(net, y, data=None, modes=None):
    """F(y) and the per-row sum of |terms| S (eq. 2).  ``modes`` =
    (pv_mode, pv_qtarget) switches PV generators to a held reactive output."""
    b = _Bound(net, data, modes)
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = n_var(net)
    assert y.shape == (n,)
    F = np.empty(n)
    S = np.empty(n)
    lib().ora_residual(ctypes.byref(b.topo), ctypes.byref(b.data), _dp(y), _dp(F), _dp(S))
    return F, S


def residual_complex(net, y, data=None, modes=None):
    """F in complex arithmetic: ``y`` and any entry of ``data`` may be complex."""
    b = _Bound(net, None, modes)
    data = data or {}
    keep = []

    def Z(a):
        z = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
        keep.append(z)
        return z.view(np.float64).ctypes.data_as(_pd)

    args = [Z(data.get(k, getattr(net, k))) for k in PARAM_FIELDS]
    args.append(Z(np.zeros(net.n_pv) if modes is None else modes[1]))
    yz = Z(y)
    F = np.zeros(n_var(net), dtype=np.complex128)
    lib().ora_residual_cs(ctypes.byref(b.topo), *args, yz,
                          F.view(np.float64).ctypes.data_as(_pd))
    return F


def branch_flows(r, x, bc, tap, shift_deg, vf, vt, thf, tht):
    out = np.empty(4)
    lib().ora_branch_flows(r, x, bc, tap, shift_deg, vf, vt, thf, tht, _dp(out))
    return out


def jacobian_coo(net, y, data=None, modes=None, scales=False):
    """Jacobian triplets (rows, cols, values) model by model; with
    ``scales`` also each triplet's sum of |products| (a tolerance scale)."""
    b = _Bound(net, data, modes)
    y = np.ascontiguousarray(y, dtype=np.float64)
    m = lib().ora_jacobian_size(ctypes.byref(b.topo))
    rows = np.empty(m, np.int32)
    cols = np.empty(m, np.int32)
    vals = np.empty(m)
    sc = np.empty(m)
    k = lib().ora_jacobian(ctypes.byref(b.topo), ctypes.byref(b.data), _dp(y),
                           _ip(rows), _ip(cols), _dp(vals), _dp(sc))
    if scales:
        return rows[:k], cols[:k], vals[:k], sc[:k]
    return rows[:k], cols[:k], vals[:k]


def jacobian(net, y, data=None, modes=None):
    """(J, scale) as scipy CSR: triplets summed into a sparse matrix; the
    second matrix sums the triplets' sums of |products| (used for
    tolerances: a bound on the rounding of either side's sum)."""
    n = n_var(net)
    r, c, v, m = jacobian_coo(net, y, data, modes, scales=True)
    J = sp.csr_matrix((v, (r, c)), shape=(n, n))
    A = sp.csr_matrix((m, (r, c)), shape=(n, n))
    J.sort_indices()
    A.sort_indices()
    return J, A


def vjp(net, y, w, data=None, modes=None):
    """(g_state, g_params) for the loss w.F: g_state = J^T w with the explicit
    Jacobian; g_params is a dict keyed by parameter name."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    J, _ = jacobian(net, y, data, modes)
    gx = J.T @ w
    return gx, vjp_params(net, y, w, data)


def vjp_params(net, y, w, data=None):
    """The parameter half of vjp(): gradients of w.F with respect to every
    branch's r, x, b, tap and shift (per degree) and every load's P and Q,
    from the pi-model partials."""
    b = _Bound(net, data)
    y = np.ascontiguousarray(y, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    B, L = net.n_branch, net.n_load
    out = {k: np.empty(B) for k in ("br_r", "br_x", "br_b", "br_tap", "br_shift_deg")}
    out["load_p"] = np.empty(L)
    out["load_q"] = np.empty(L)
    lib().ora_vjp_params(ctypes.byref(b.topo), ctypes.byref(b.data), _dp(y), _dp(w),
                         _dp(out["br_r"]), _dp(out["br_x"]), _dp(out["br_b"]),
                         _dp(out["br_tap"]), _dp(out["br_shift_deg"]),
                         _dp(out["load_p"]), _dp(out["load_q"]))
    return out


def vjp_params_scale(net, y, w, data=None):
    """Per-parameter sum of |terms| behind vjp()'s parameter gradients (a
    tolerance scale for comparisons under cancellation)."""
    b = _Bound(net, data)
    y = np.ascontiguousarray(y, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    B = net.n_branch
    out = {k: np.empty(B) for k in ("br_r", "br_x", "br_b", "br_tap", "br_shift_deg")}
    lib().ora_vjp_params_scale(ctypes.byref(b.topo), ctypes.byref(b.data), _dp(y), _dp(w),
                               _dp(out["br_r"]), _dp(out["br_x"]), _dp(out["br_b"]),
                               _dp(out["br_tap"]), _dp(out["br_shift_deg"]))
    return out


def newton(net, y0, tol=1e-10, max_iter=10, data=None, modes=None):
    """Full-step Newton (tasks 1-4): returns (y, list of ||F||_inf per
    iteration, list of iterates).  The list of norms starts at y0."""
    y = np.array(y0, dtype=np.float64)
    norms, iters = [], [y.copy()]
    for it in range(max_iter + 1):
        F, _ = residual(net, y, data, modes)
        nf = float(np.max(np.abs(F))) if F.size else 0.0
        norms.append(nf)
        if nf < tol or it == max_iter:
            break
        J, _ = jacobian(net, y, data, modes)
        dx = spla.spsolve(J.tocsc(), F)
        y = y - dx
        iters.append(y.copy())
    return y, norms, iters


def q_limit_switch(net, y, mode, qt, qmin, qmax, tol=1e-9):
    """One check of the PV generators' reactive limits (Section II-A: the
    formulation lets the limits be checked during the iterations, and a PV
    generator that reaches one becomes a PQ injection under the same
    equations).  A generator under voltage control whose Q_g has left
    [qmin, qmax] by more than tol is held at the violated limit.  A held
    generator returns to voltage control when its bus voltage has crossed
    the set point to the side where less reactive output would hold it:
    above V_set when held at qmax, below V_set when held at qmin.
    Returns (mode, qt, number of switches) as new arrays."""
    N = net.n_bus
    mode = np.array(mode, dtype=np.int32)
    qt = np.array(qt, dtype=np.float64)
    switched = 0
    for k in range(net.n_pv):
        q = y[2 * N + k]
        v = y[N + net.pv_bus[k]]
        if mode[k] == 0:
            if q > qmax[k] + tol:
                mode[k], qt[k] = 1, qmax[k]
                switched += 1
            elif q < qmin[k] - tol:
                mode[k], qt[k] = 1, qmin[k]
                switched += 1
        else:
            at_max = qt[k] == qmax[k]
            if (at_max and v > net.pv_v[k] + tol) or (not at_max and v < net.pv_v[k] - tol):
                mode[k], qt[k] = 0, 0.0
                switched += 1
    return mode, qt, switched


def newton_qlim_inner(net, y0, qmin, qmax, tol=1e-10, max_iter=20, check_below=1e-3,
                      switch_tol=1e-9):
    """Newton power flow with the reactive limits checked during the
    iterations (Section II-A: in the extended formulation one set of equations
    covers a PV unit both under voltage control and held at a reactive
    target, so the limits can be checked at any iterate).  At every iterate whose mismatch is below ``check_below`` the
    switching rule (q_limit_switch) is applied; after a switch the residual
    is taken again under the new modes before the step.  Converged when
    ||F||_inf < tol under modes that the check at that iterate left
    unchanged.  Returns (y, mode, qt, list of ||F||_inf, list of the
    iterations at which a switch happened, converged)."""
    y = np.array(y0, dtype=np.float64)
    mode = np.zeros(net.n_pv, np.int32)
    qt = np.zeros(net.n_pv)
    norms, switched_at = [], []
    for it in range(max_iter + 1):
        F, _ = residual(net, y, modes=(mode, qt))
        nf = float(np.max(np.abs(F)))
        if nf < check_below:
            mode, qt, ns = q_limit_switch(net, y, mode, qt, qmin, qmax, switch_tol)
            if ns:
                switched_at.append(it)
                F, _ = residual(net, y, modes=(mode, qt))
                nf = float(np.max(np.abs(F)))
        norms.append(nf)
        if nf < tol:
            return y, mode, qt, norms, switched_at, True
        if it == max_iter:
            break
        J, _ = jacobian(net, y, modes=(mode, qt))
        y = y - spla.spsolve(J.tocsc(), F)
    return y, mode, qt, norms, switched_at, False


def newton_qlim(net, y0, qmin, qmax, tol=1e-10, max_iter=10, max_outer=10):
    """Newton power flow with reactive limits (Section II-A: one set of
    equations covers a PV unit both under voltage control and held at a
    reactive target): solve, check the limits, switch, and solve again from the
    last state until no generator switches.  Returns (y, mode, qt, outer
    rounds, converged)."""
    y = np.array(y0, dtype=np.float64)
    mode = np.zeros(net.n_pv, np.int32)
    qt = np.zeros(net.n_pv)
    for outer in range(1, max_outer + 1):
        y, norms, _ = newton(net, y, tol, max_iter, modes=(mode, qt))
        if not norms[-1] < tol:
            return y, mode, qt, outer, False
        mode, qt, ns = q_limit_switch(net, y, mode, qt, qmin, qmax)
        if ns == 0:
            return y, mode, qt, outer, True
    return y, mode, qt, max_outer, False


def fdlf_matrices(net):
    """Constant matrices of the fast decoupled method, XB variant (the
    method Section V names as another user of the same residual
    evaluation).  B' (angle step) over the buses without a slack:
    per in-service branch the weight 1/x only (resistance, taps, shifts and
    charging left out), so B' is the weighted Laplacian of the network with
    the slack rows and columns removed.  B'' (voltage step) over the buses
    with no voltage controller: -Im(Y_bus) of the full pi-models with taps,
    charging and bus shunts, phase shifts left out.  Returns
    (Bp, Bpp, buses of B' rows, buses of B'' rows) with CSR matrices."""
    N = net.n_bus
    ctrl = np.zeros(N, bool)
    ctrl[net.pv_bus] = True
    ctrl[net.slack_bus] = True
    slack = np.zeros(N, bool)
    slack[net.slack_bus] = True
    rows_p = np.nonzero(~slack)[0]
    rows_q = np.nonzero(~ctrl)[0]
    ip = -np.ones(N, np.int64)
    ip[rows_p] = np.arange(rows_p.size)
    iq = -np.ones(N, np.int64)
    iq[rows_q] = np.arange(rows_q.size)
    P = {}
    Q = {}

    def add(D, idx, i, j, v):
        a, b = idx[i], idx[j]
        if a >= 0 and b >= 0:
            D[(a, b)] = D.get((a, b), 0.0) + v

    for e in range(net.n_branch):
        if net.br_status is not None and not net.br_status[e]:
            continue
        f, t = int(net.br_from[e]), int(net.br_to[e])
        w = 1.0 / net.br_x[e]
        add(P, ip, f, f, w)
        add(P, ip, t, t, w)
        add(P, ip, f, t, -w)
        add(P, ip, t, f, -w)
        r, x, bc, tap = net.br_r[e], net.br_x[e], net.br_b[e], net.br_tap[e]
        b = -x / (r * r + x * x)          # Im of the series admittance
        add(Q, iq, f, f, -(b + bc / 2) / (tap * tap))
        add(Q, iq, t, t, -(b + bc / 2))
        add(Q, iq, f, t, b / tap)
        add(Q, iq, t, f, b / tap)
    for k in range(net.n_shunt):
        i = int(net.shunt_bus[k])
        add(Q, iq, i, i, -net.shunt_b[k])

    def csr(D, m):
        if not D:
            return sp.csr_matrix((m, m))
        keys = np.array(list(D.keys()))
        M = sp.csr_matrix((np.array(list(D.values())), (keys[:, 0], keys[:, 1])), shape=(m, m))
        M.sort_indices()
        return M

    return csr(P, rows_p.size), csr(Q, rows_q.size), rows_p, rows_q


def fdlf(net, y0, tol=1e-10, max_iter=50):
    """Fast decoupled power flow (XB): per iteration an angle half-step
    theta <- theta - B'^-1 (F_p / V) over the non-slack buses, then a voltage
    half-step V <- V - B''^-1 (F_q / V) over the buses without a voltage
    controller, each from a fresh residual.  The generator variables are
    not stepped: once the bus mismatches are below tol, Q_g and P_s take the
    values that zero their buses' rows.  Controlled voltages and slack
    angles are never stepped, so they start at their set points.  Returns
    (y, norms, iterates) with norms[k] the largest mismatch of the stepped
    rows before iteration k and the last entry ||F||_inf after the
    generator update."""
    N, NPV, NG = net.n_bus, net.n_pv, net.n_gen
    Bp, Bpp, rp, rq = fdlf_matrices(net)
    lup = spla.splu(Bp.tocsc()) if rp.size else None
    luq = spla.splu(Bpp.tocsc()) if rq.size else None
    y = np.array(y0, dtype=np.float64)
    y[N + net.pv_bus] = net.pv_v
    y[N + net.slack_bus] = net.slack_v
    y[net.slack_bus] = net.slack_theta
    norms, iters = [], [y.copy()]
    for it in range(max_iter + 1):
        F, _ = residual(net, y)
        m = max(np.max(np.abs(F[rp]), initial=0.0), np.max(np.abs(F[N + rq]), initial=0.0))
        norms.append(float(m))
        if m < tol or it == max_iter:
            break
        if lup is not None:
            y[rp] -= lup.solve(F[rp] / y[N + rp])
        F, _ = residual(net, y)
        if luq is not None:
            y[N + rq] -= luq.solve(F[N + rq] / y[N + rq])
        iters.append(y.copy())
    F, _ = residual(net, y)
    y[2 * N:2 * N + NPV] += F[N + net.pv_bus]
    y[2 * N + NPV:2 * N + NG] += F[N + net.slack_bus]
    y[2 * N + NG:] += F[net.slack_bus]
    F, _ = residual(net, y)
    norms.append(float(np.max(np.abs(F))))
    return y, norms, iters
