"""Property-based pins of the oracle (CPU): the same mathematical facts as
the fixed-network pins, on networks that hypothesis draws from the seeded
fuzz generator (2 to 89 buses, transformers with taps and phase shifts,
parallel and out-of-service branches, shunts, extra loads, held PV units).
Each property is fixed by the mathematics, not by the oracle: the textbook
bus-admittance product (Section II-A's bus rows are the sums of the device
injections), invariance under a common angle shift, degree-2 homogeneity of
the network injections in V, the Jacobian as the derivative of the
residual (complex step), the adjoint as the transposed product, and a held
unit's control row."""

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

from fuzz_nets import random_net
from paper_2011_11880_amd import synth
from test_oracle_pins import _model_terms, _ybus

CASES = settings(max_examples=25, deadline=None, derandomize=True,
                 suppress_health_check=[HealthCheck.too_slow,
                                        HealthCheck.function_scoped_fixture])
net_seeds = st.integers(min_value=0, max_value=100_000)
state_seeds = st.integers(min_value=0, max_value=1_000)


def _case(net_seed, state_seed):
    net = random_net(net_seed)
    return net, synth.random_states(net, seed=state_seed)


@CASES
@given(net_seeds, state_seeds)
def test_bus_rows_are_the_admittance_product(ora, net_seed, state_seed):
    net, yv = _case(net_seed, state_seed)
    N = net.n_bus
    F, S = ora.residual(net, yv)
    V = yv[N:2 * N] * np.exp(1j * yv[:N])
    Sbus = V * np.conj(_ybus(net) @ V)
    p, q = _model_terms(net, yv)
    assert np.all(np.abs(F[:N] - (Sbus.real + p)) <= 1e-12 * S[:N] + 1e-14)
    assert np.all(np.abs(F[N:2 * N] - (Sbus.imag + q)) <= 1e-12 * S[N:2 * N] + 1e-14)


@CASES
@given(net_seeds, state_seeds, st.floats(min_value=-3.0, max_value=3.0))
def test_common_angle_shift(ora, net_seed, state_seed, shift):
    net, yv = _case(net_seed, state_seed)
    N = net.n_bus
    F0, S = ora.residual(net, yv)
    y1 = yv.copy()
    y1[:N] += shift
    F1, S1 = ora.residual(net, y1)
    tol = 1e-12 * (S[:2 * N] + S1[:2 * N]) + 1e-14
    assert np.all(np.abs(F1[:2 * N] - F0[:2 * N]) <= tol)
    J, A = ora.jacobian(net, yv)
    rs = np.asarray(J[:2 * N, :N].sum(axis=1)).ravel()
    sc = np.asarray(A[:2 * N, :N].sum(axis=1)).ravel()
    assert np.all(np.abs(rs) <= 1e-12 * sc + 1e-14)


@CASES
@given(net_seeds, state_seeds)
def test_network_injections_homogeneous_in_v(ora, net_seed, state_seed):
    net, yv = _case(net_seed, state_seed)
    N = net.n_bus
    F, S = ora.residual(net, yv)
    p, q = _model_terms(net, yv)
    Fnet = np.concatenate([F[:N] - p, F[N:2 * N] - q])
    J, A = ora.jacobian(net, yv)
    lhs = J[:2 * N, N:2 * N] @ yv[N:2 * N]
    sc = A[:2 * N, N:2 * N] @ yv[N:2 * N]
    assert np.all(np.abs(lhs - 2 * Fnet) <= 1e-12 * (sc + 2 * S[:2 * N]) + 1e-14)


@CASES
@given(net_seeds, state_seeds)
def test_jacobian_is_the_complex_step_derivative(ora, net_seed, state_seed):
    net, yv = _case(net_seed, state_seed)
    J, A = ora.jacobian(net, yv)
    Jd, Ad = J.toarray(), A.toarray()
    h = 1e-30
    rng = np.random.default_rng(state_seed)
    cols = rng.choice(yv.size, min(yv.size, 24), replace=False)
    for j in cols:
        yz = yv.astype(complex)
        yz[j] += 1j * h
        col = ora.residual_complex(net, yz).imag / h
        assert np.all(np.abs(col - Jd[:, j]) <= 1e-13 * (Ad[:, j] + 1)), j


@CASES
@given(net_seeds, state_seeds)
def test_adjoint_is_the_transposed_product(ora, net_seed, state_seed):
    net, yv = _case(net_seed, state_seed)
    w = np.random.default_rng(state_seed + 1).standard_normal(yv.size)
    gx, _ = ora.vjp(net, yv, w)
    J, A = ora.jacobian(net, yv)
    ref = J.T @ w
    sc = abs(A).T @ np.abs(w)
    assert np.all(np.abs(gx - ref) <= 1e-12 * sc + 1e-14)


@CASES
@given(net_seeds, state_seeds, st.integers(min_value=0, max_value=2 ** 31 - 1))
def test_held_unit_rows(ora, net_seed, state_seed, pick):
    """A held PV unit's control row is Q_g - Q_target with a single +1 on its
    own Q_g column; every other row keeps its voltage-control value."""
    net, yv = _case(net_seed, state_seed)
    if net.n_pv == 0:
        return
    N, NPV = net.n_bus, net.n_pv
    rng = np.random.default_rng(pick)
    mode = (rng.random(NPV) < 0.5).astype(np.int32)
    qt = rng.normal(size=NPV)
    F0, _ = ora.residual(net, yv)
    F1, _ = ora.residual(net, yv, modes=(mode, qt))
    J1, _ = ora.jacobian(net, yv, modes=(mode, qt))
    J0, _ = ora.jacobian(net, yv)
    rows = 2 * N + np.arange(NPV)
    held = rows[mode == 1]
    np.testing.assert_array_equal(F1[held], yv[held] - qt[mode == 1])
    keep = np.setdiff1d(np.arange(yv.size), held)
    np.testing.assert_array_equal(F1[keep], F0[keep])
    for r in held:
        row = J1.getrow(r).toarray().ravel()
        e = np.zeros(yv.size)
        e[r] = 1.0
        np.testing.assert_array_equal(row, e)
    d = (J1 - J0)[keep]
    assert abs(d).sum() == 0.0
