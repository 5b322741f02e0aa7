"""ctypes declarations of libpf's C ABI (include/pf.h).

Argument marshalling only: every step of the evaluation runs in libpf's HIP
kernels.  Loading fails loudly when the library has not been built; there is
no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libpf.so")

PF_OK = 0
PF_EINVAL = -1
PF_ETOPO = -2
PF_EDEVICE = -3
PF_ENOMEM = -4
PF_ESOLVE = -5
PF_ENOCONV = -6

PF_LAYOUT_ROWS = 0
PF_LAYOUT_PANELS = 1

PF_ORDER_INPUT = 0
PF_ORDER_LOCALITY = 1

_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_d = ctypes.c_double
_pi32 = ctypes.POINTER(ctypes.c_int32)
_pi64 = ctypes.POINTER(ctypes.c_int64)
_pd = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p


class pf_network(ctypes.Structure):
    _fields_ = [
        ("n_bus", _i32), ("n_branch", _i32), ("n_load", _i32), ("n_pv", _i32),
        ("n_slack", _i32), ("n_shunt", _i32),
        ("br_from", _pi32), ("br_to", _pi32),
        ("br_r", _pd), ("br_x", _pd), ("br_b", _pd), ("br_tap", _pd), ("br_shift_deg", _pd),
        ("br_status", _pi32),
        ("load_bus", _pi32), ("load_p", _pd), ("load_q", _pd),
        ("pv_bus", _pi32), ("pv_p", _pd), ("pv_v", _pd),
        ("slack_bus", _pi32), ("slack_v", _pd), ("slack_theta", _pd),
        ("shunt_bus", _pi32), ("shunt_g", _pd), ("shunt_b", _pd),
    ]


class pf_schedule(ctypes.Structure):
    _fields_ = [("tile_entries", _i32), ("waves_per_block", _i32), ("grid_blocks", _i32),
                ("batch_buses", _i32), ("batch_order", _i32), ("xcd_remap", _i32),
                ("batch_group", _i32)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


class pf_setup_opts(ctypes.Structure):
    _fields_ = [("host_only", _i32), ("device", _i32), ("sched", pf_schedule),
                ("q_limits", _i32), ("bus_order", _i32)]


class pf_batch_spec(ctypes.Structure):
    _fields_ = [("n_inst", _i32), ("load_scale", _pd), ("pv_scale", _pd), ("outage", _pi32),
                ("inst_stride", _i32), ("layout", _i32)]


class pf_info_t(ctypes.Structure):
    _fields_ = [("n", _i64), ("nnz", _i64), ("n_params", _i64), ("n_entries", _i64),
                ("n_bus", _i32), ("n_branch", _i32), ("n_load", _i32), ("n_pv", _i32),
                ("n_slack", _i32), ("n_shunt", _i32), ("n_inst", _i32), ("inst_stride", _i32),
                ("layout", _i32), ("n_grids", _i32),
                ("n_tiles", _i32), ("kind", _i32)]


class pf_newton_opts(ctypes.Structure):
    _fields_ = [("tol", _d), ("max_iter", _i32), ("q_min", _pd), ("q_max", _pd),
                ("q_check_below", _d), ("q_switch_tol", _d)]


class pf_newton_report(ctypes.Structure):
    _fields_ = [("iterations", _i32), ("converged", _i32), ("norm", _d * 65),
                ("t_eval_s", _d), ("t_solve_s", _d), ("t_total_s", _d),
                ("switched", _i32 * 65), ("n_switches", _i32)]


pf_linsolve_fn = ctypes.CFUNCTYPE(ctypes.c_int, _vp, _i64, _pi32, _pi32, _pd, _pd, _pd)

_P = ctypes.c_void_p  # pf_plan*

SIGNATURES = {
    "pf_setup": (ctypes.c_int, [ctypes.POINTER(pf_network), ctypes.POINTER(pf_setup_opts),
                                ctypes.POINTER(_P)]),
    "pf_setup_batch": (ctypes.c_int, [ctypes.POINTER(pf_network), ctypes.POINTER(pf_batch_spec),
                                      ctypes.POINTER(pf_setup_opts), ctypes.POINTER(_P)]),
    "pf_setup_multi": (ctypes.c_int, [ctypes.POINTER(pf_network), _i32,
                                      ctypes.POINTER(pf_setup_opts), ctypes.POINTER(_P)]),
    "pf_info": (ctypes.c_int, [_P, _pi64, _pi64]),
    "pf_info_ex": (ctypes.c_int, [_P, ctypes.POINTER(pf_info_t)]),
    "pf_info_multi": (ctypes.c_int, [_P, _pi64, _pi64]),
    "pf_pattern": (ctypes.c_int, [_P, _pi32, _pi32]),
    "pf_bus_order": (ctypes.c_int, [_P, _pi32]),
    "pf_jacobian_row_order": (ctypes.c_int, [_P, _pi32]),
    "pf_jacobian_switch_order": (ctypes.c_int, [_P, _pi32, _pi32]),
    "pf_eval_residual": (ctypes.c_int, [_P, _vp, _vp, _vp]),
    "pf_eval_jacobian": (ctypes.c_int, [_P, _vp, _vp, _vp]),
    "pf_eval": (ctypes.c_int, [_P, _vp, _vp, _vp, _vp]),
    "pf_eval_batch": (ctypes.c_int, [_P, _vp, _vp, _vp, _vp]),
    "pf_set_params": (ctypes.c_int, [_P, _vp, _vp]),
    "pf_vjp": (ctypes.c_int, [_P, _vp, _vp, _i32, _vp, _vp, _vp]),
    "pf_get_schedule": (ctypes.c_int, [_P, ctypes.POINTER(pf_schedule)]),
    "pf_set_schedule": (ctypes.c_int, [_P, ctypes.POINTER(pf_schedule)]),
    "pf_autotune": (ctypes.c_int, [_P, _vp, _vp, _vp, _i32, _vp, ctypes.POINTER(pf_schedule)]),
    "pf_autotune_cached": (ctypes.c_int, [_P, _vp, _vp, _vp, _i32, _vp, ctypes.c_char_p,
                                          ctypes.POINTER(pf_schedule), _pi32]),
    "pf_newton": (ctypes.c_int, [_P, _vp, ctypes.POINTER(pf_newton_opts), pf_linsolve_fn, _vp,
                                 ctypes.POINTER(pf_newton_report)]),
    "pf_set_gen_modes": (ctypes.c_int, [_P, _pi32, _pd]),
    "pf_get_gen_modes": (ctypes.c_int, [_P, _pi32, _pd]),
    "pf_q_limit_check": (ctypes.c_int, [_P, _vp, _pd, _pd, ctypes.c_double, _pi32, _vp]),
    "pf_refact_create": (ctypes.c_int, [_P, _pd, _i64, _pi32, _pi32, _pd, _pi32, _pi32,
                                        ctypes.POINTER(_vp)]),
    "pf_refact_solve": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "pf_newton_device": (ctypes.c_int, [_P, _vp, _vp, ctypes.POINTER(pf_newton_opts),
                                        ctypes.POINTER(pf_newton_report), _vp]),
    "pf_refact_destroy": (None, [_vp]),
    "pf_fdlf_matrices": (ctypes.c_int, [_P, _pi64, _pi32, _pi32, _pd, _pi32, _pi64, _pi32,
                                        _pi32, _pd, _pi32]),
    "pf_lu_symbolic": (ctypes.c_int, [_i64, _pi32, _pi32, _pi32, _pi32, _pi64, _pi32, _pi32]),
    "pf_lu_create": (ctypes.c_int, [_i32, _i64, _i64, _pi32, _pi32, _pd, _i64, _pi32, _pi32,
                                    _pd, _pi32, _pi32, ctypes.POINTER(_vp)]),
    "pf_lu_solve": (ctypes.c_int, [_vp, _vp, _vp]),
    "pf_lu_solve_noalloc": (ctypes.c_int, [_vp, _vp, _vp]),
    "pf_lu_destroy": (None, [_vp]),
    "pf_fdlf_create": (ctypes.c_int, [_P, _vp, _vp, ctypes.POINTER(_vp)]),
    "pf_fdlf_solve": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(pf_newton_opts),
                                     ctypes.POINTER(pf_newton_report), _vp]),
    "pf_fdlf_destroy": (None, [_vp]),
    "pf_batch_lu_create": (ctypes.c_int, [_P, _i64, _pi32, _pi32, _pi32, _pi32,
                                          ctypes.POINTER(_vp)]),
    "pf_batch_lu_factor": (ctypes.c_int, [_vp, _vp, _vp]),
    "pf_batch_lu_solve": (ctypes.c_int, [_vp, _vp, _vp, _vp]),
    "pf_newton_batch": (ctypes.c_int, [_P, _vp, _vp, ctypes.POINTER(pf_newton_opts), _pi32, _pd,
                                       ctypes.POINTER(pf_newton_report), _vp]),
    "pf_batch_lu_destroy": (None, [_vp]),
    "pf_destroy": (None, [_P]),
    "pf_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """The loaded libpf (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                "libpf.so is missing: build it with `python -m paper_2011_11880_amd.build`; "
                "there is no fallback path")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class PFError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"[{code}] {msg}")
        self.code = code


def check(rc):
    if rc != PF_OK:
        msg = lib().pf_last_error()
        raise PFError(rc, msg.decode() if msg else "")
    return rc
