"""Plant plausible mistakes in copies of the CPU oracle and check that the
pins in test_oracle_pins.py catch every one of them.

Each mutant is a one-site textual change (a dropped term, a flipped sign, a
wrong index or a transposed operand) to ``oracle/pf_oracle.c`` or
``oracle/ora_core.inc``, compiled with gcc into a temporary directory, or to
the reactive-limit logic of ``oracle/oracle.py``, executed as a separate
module.  The real oracle is restored after every mutant.  Runs on the CPU
only.
"""

import os
import shutil
import subprocess
import types

import pytest

import test_oracle_pins as P
import test_oracle_qlim as Q

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORA = os.path.join(ROOT, "oracle")

# (id, file, original text, mutated text)
MUTANTS = [
    ("P_f sin sign", "ora_core.inc", "out[0] = vf * vf * (g + gsh) / t2 - u * (g * c + b * s);",
     "out[0] = vf * vf * (g + gsh) / t2 - u * (g * c - b * s);"),
    ("Q_f charging dropped", "ora_core.inc", "out[1] = -vf * vf * (b + bsh) / t2",
     "out[1] = -vf * vf * (b) / t2"),
    ("P_f tap squared -> tap", "ora_core.inc", "out[0] = vf * vf * (g + gsh) / t2",
     "out[0] = vf * vf * (g + gsh) / tap"),
    ("shift sign", "ora_core.inc", "thf - tht - phi;", "thf - tht + phi;"),
    ("Q_t sign of B2", "ora_core.inc", "out[3] = -vt * vt * (b + bsh) + u * (g * s + b * c);",
     "out[3] = -vt * vt * (b + bsh) - u * (g * s + b * c);"),
    ("P_t uses V_f", "ora_core.inc", "out[2] = vt * vt * (g + gsh)", "out[2] = vf * vf * (g + gsh)"),
    ("susceptance sign", "ora_core.inc", "const ORA_T b = -x / d;", "const ORA_T b = x / d;"),
    ("shunt Q sign", "ora_core.inc", "Fq[i] -= shunt_b[k] * V[i] * V[i];",
     "Fq[i] += shunt_b[k] * V[i] * V[i];"),
    ("slack P sign", "ora_core.inc", "Fp[i] -= Ps[k];", "Fp[i] += Ps[k];"),
    ("load Q uses P", "ora_core.inc", "Fq[i] += load_q[k];", "Fq[i] += load_p[k];"),
    ("PV Q_g index", "ora_core.inc", "Fq[i] -= Qg[k];", "Fq[i] -= Qg[NPV - 1 - k];"),
    ("to-bus row gets from flow", "ora_core.inc", "Fp[t] += fl[2];", "Fp[t] += fl[0];"),
    ("J dPf/dth_t sign", "pf_oracle.c", "PUT(f, t, -B1, mB);", "PUT(f, t, B1, mB);"),
    ("J dQf/dV_t column", "pf_oracle.c", "PUT(N + f, N + t, -(vf / tap) * (g * S - b * C),",
     "PUT(N + f, t, -(vf / tap) * (g * S - b * C),"),
    ("J dPt/dV_t factor 2 dropped", "pf_oracle.c",
     "PUT(t, N + t, 2.0 * vt * g - (vf / tap) * (g * C - b * S),",
     "PUT(t, N + t, vt * g - (vf / tap) * (g * C - b * S),"),
    ("J transposed dQt/dth", "pf_oracle.c", "PUT(N + t, f, A2, mA);", "PUT(f, N + t, A2, mA);"),
    ("J shunt Q sign", "pf_oracle.c", "vb = -2.0 * dd->shunt_b[e] * V[i];",
     "vb = 2.0 * dd->shunt_b[e] * V[i];"),
    ("J slack theta row", "pf_oracle.c", "PUT(2 * N + NG + e, i, 1.0, 1.0);",
     "PUT(2 * N + NG + e, N + i, 1.0, 1.0);"),
    ("vjp dg/dx sign", "pf_oracle.c", "dg_dx = -2.0 * r * x / D2;", "dg_dx = 2.0 * r * x / D2;"),
    ("vjp tap term", "pf_oracle.c", "wpt * (A2 / tap) + wqt * (-B2 / tap);",
     "wpt * (A2 / tap) + wqt * (B2 / tap);"),
    ("vjp shift unit", "pf_oracle.c", "g_shift[e] = -(wpf * B1 + wqf * (-A1) + wpt * B2 + wqt * A2) *\n                     (ORA_PI / 180.0);",
     "g_shift[e] = -(wpf * B1 + wqf * (-A1) + wpt * B2 + wqt * A2);"),
    ("vjp load index", "pf_oracle.c", "g_lq[e] = w[N + tp->load_bus[e]];", "g_lq[e] = w[tp->load_bus[e]];"),
    ("held PV row uses V", "ora_core.inc", "FV[k] = Qg[k] - pv_qt[k];", "FV[k] = V[i] - pv_qt[k];"),
    ("scale s_x = s_r", "pf_oracle.c",
     "s_x[e] = (sg * fabs(2.0 * r * x) + sb * (x * x + r * r)) / D2;", "s_x[e] = s_r[e];"),
    ("scale difference counted once", "pf_oracle.c", "s_r[e] = (sg * (x * x + r * r)",
     "s_r[e] = (sg * fabs(x * x - r * r)"),
    ("scale tap charging dropped", "pf_oracle.c", "(ab + fabs(bc) / 2.0)", "(ab)"),
    ("J held PV column", "pf_oracle.c", "PUT(2 * N + e, 2 * N + e, 1.0, 1.0);",
     "PUT(2 * N + e, N + i, 1.0, 1.0);"),
    ("flow scale drops u b S", "pf_oracle.c", "out[0] = fabs(vf * vf * g / t2) + ugc + ubs;",
     "out[0] = fabs(vf * vf * g / t2) + ugc;"),
    ("flow scale charging dropped", "pf_oracle.c",
     "out[3] = fabs(vt * vt * b) + fabs(vt * vt * bc / 2.0) + ugs + ubc;",
     "out[3] = fabs(vt * vt * b) + ugs + ubc;"),
    ("flow scale to-side uses V_f", "pf_oracle.c", "out[2] = fabs(vt * vt * g) + ugc + ubs;",
     "out[2] = fabs(vf * vf * g) + ugc + ubs;"),
    ("J scale of B1 taken as |B1|", "pf_oracle.c", "mB = fabs(u * g * S) + fabs(u * b * C);",
     "mB = fabs(u * (g * S - b * C));"),
    ("J scale dQf/dV_f charging dropped", "pf_oracle.c",
     "fabs(2.0 * vf * b / t2) + fabs(vf * bc / t2) + fabs(at * g * S)",
     "fabs(2.0 * vf * b / t2) + fabs(at * g * S)"),
    ("J scale shunt dropped", "pf_oracle.c", "PUT(i, N + i, vg, fabs(vg));",
     "PUT(i, N + i, vg, 0.0);"),
]

PINS = [
    P.test_eq4_printed_case,
    P.test_two_bus_hand_cases,
    P.test_branch_losses_closed_form,
    lambda o: P.test_against_complex_ybus(o, "everything"),
    P.test_outaged_branch_is_absent,
    P.test_power_balance,
    P.test_common_angle_shift_invariance,
    P.test_voltage_homogeneity,
    P.test_flat_start_laplacian,
    lambda o: P.test_jacobian_complex_step(o, "everything"),
    P.test_sizes_and_pattern,
    P.test_vjp_state_is_transpose_product,
    P.test_vjp_params_complex_step,
    P.test_vjp_params_scale_is_sum_of_abs_terms,
    P.test_residual_scale_is_sum_of_abs_products,
    P.test_jacobian_scale_is_sum_of_abs_products,
    Q.test_held_output_equals_pq_injection,
    lambda o: Q.test_jacobian_complex_step_with_held_outputs(o, "tiny"),
]


@pytest.mark.parametrize("mid,fname,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(ora, tmp_path, mid, fname, old, new):
    for f in ("pf_oracle.c", "ora_core.inc"):
        shutil.copy(os.path.join(ORA, f), tmp_path / f)
    src = (tmp_path / fname).read_text()
    assert src.count(old) == 1, "mutation site must be unique: " + mid
    (tmp_path / fname).write_text(src.replace(old, new))
    so = str(tmp_path / "libmut.so")
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-fPIC",
                           "-shared", str(tmp_path / "pf_oracle.c"), "-o", so, "-lm"])
    prev = ora.use_library(so)
    caught = []
    try:
        for pin in PINS:
            try:
                pin(ora)
            except AssertionError:
                caught.append(getattr(pin, "__name__", "pin"))
    finally:
        ora.use_library(None)
        del prev
    assert caught, "no pin caught mutant: " + mid


# (id, original text, mutated text) in oracle/oracle.py: the switching rule
# and the Newton loops with limits
PY_MUTANTS = [
    ("release at qmax on the wrong side", "(at_max and v > net.pv_v[k] + tol)",
     "(at_max and v < net.pv_v[k] - tol)"),
    ("held at the wrong limit", "mode[k], qt[k] = 1, qmax[k]", "mode[k], qt[k] = 1, qmin[k]"),
    ("lower limit never checked", "elif q < qmin[k] - tol:", "elif q < qmin[k] - tol - 1e9:"),
    ("in-iteration check never switches", "mode, qt, ns = q_limit_switch(net, y, mode, qt, qmin, qmax, switch_tol)",
     "ns = 0"),
]

PY_PINS = [
    Q.test_switching_rule_cases,
    Q.test_newton_with_limits_ends_feasible,
    Q.test_newton_with_limits_checked_in_the_iterations_ends_feasible,
]


@pytest.mark.parametrize("mid,old,new", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_python_mutant_is_caught(ora, mid, old, new):
    path = os.path.join(ORA, "oracle.py")
    with open(path) as fh:
        src = fh.read()
    assert src.count(old) == 1, "mutation site must be unique: " + mid
    mod = types.ModuleType("oracle_mutant")
    mod.__file__ = path
    exec(compile(src.replace(old, new), path, "exec"), mod.__dict__)
    caught = []
    for pin in PY_PINS:
        try:
            pin(mod)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, "no pin caught mutant: " + mid
