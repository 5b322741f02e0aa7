"""Pins of the oracle's fast decoupled method (CPU only): B' against the
weighted Laplacian built from the branch-bus incidence matrix, B'' against
the textbook bus admittance matrix, and the iteration's fixed point against
Newton's solution."""

import numpy as np
import scipy.sparse as sp

from paper_2011_11880_amd import synth
from test_oracle_pins import _net_with_everything, _ybus, manufactured


def test_bprime_is_reduced_weighted_laplacian(ora):
    net = _net_with_everything()
    Bp, _, rp, _ = ora.fdlf_matrices(net)
    on = net.br_status.astype(bool)
    f, t, x = net.br_from[on], net.br_to[on], net.br_x[on]
    m = f.size
    A = sp.csr_matrix((np.concatenate([np.ones(m), -np.ones(m)]),
                       (np.concatenate([np.arange(m)] * 2), np.concatenate([f, t]))),
                      shape=(m, net.n_bus))
    L = (A.T @ sp.diags(1.0 / x) @ A).toarray()
    np.testing.assert_allclose(Bp.toarray(), L[np.ix_(rp, rp)], rtol=1e-14, atol=1e-12)
    assert not np.isin(net.slack_bus, rp).any() and rp.size == net.n_bus - net.n_slack


def test_bdoubleprime_is_minus_imag_ybus(ora):
    net = _net_with_everything()
    _, Bpp, _, rq = ora.fdlf_matrices(net)
    flat = net.copy()
    flat.br_shift_deg = np.zeros(net.n_branch)
    Y = _ybus(flat).toarray()
    np.testing.assert_allclose(Bpp.toarray(), -Y.imag[np.ix_(rq, rq)], rtol=1e-13, atol=1e-12)
    ctrl = np.concatenate([net.pv_bus, net.slack_bus])
    assert not np.isin(ctrl, rq).any() and rq.size == net.n_bus - ctrl.size


def test_fixed_point_is_newton_solution(ora):
    net0 = synth.fill_zero_injection_buses(synth.grid_meshed(200, 5))
    N = net0.n_bus
    ystar = synth.random_states(net0, seed=40)
    ystar[:N] *= 0.3
    net, ystar = manufactured(ora, net0, ystar)
    assert np.max(np.abs(ora.residual(net, ystar)[0])) < 1e-12
    rng = np.random.default_rng(1)
    y0 = ystar + np.concatenate([rng.normal(0, 0.02, 2 * N), rng.normal(0, 0.05, net.n_var - 2 * N)])
    y, norms, iters = ora.fdlf(net, y0, tol=1e-11, max_iter=60)
    assert norms[-1] < 1e-10
    # linear convergence: the stepped-row mismatch falls by a steady factor
    ratio = np.array(norms[2:-1]) / np.array(norms[1:-2])
    assert np.all(ratio < 0.8)
    yn, nn, _ = ora.newton(net, y0, tol=1e-12)
    assert nn[-1] < 1e-12
    np.testing.assert_allclose(y, yn, rtol=0, atol=1e-10)
    np.testing.assert_allclose(y, ystar, rtol=0, atol=1e-10)
    F, _ = ora.residual(net, y)
    assert np.max(np.abs(F)) < 1e-10
