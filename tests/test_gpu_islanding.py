"""Branch outages that split the network (a bridge taken out) make the
Jacobian singular: an island without the slack has no angle reference.
Newton with host solves reports PF_ESOLVE; batched Newton leaves only the
islanded instances unconverged (non-finite where the singularity is exact),
and every other instance ends bit for bit where it ends in a batch without
them.  No kernel faults: a zero pivot gives IEEE infinities and NaNs in its
own instance only."""

import numpy as np
import pytest

from paper_2011_11880_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _with_pendant_pair(net, k):
    """Two new PQ buses a, b joined by a branch, and a bridge k -> a."""
    N = net.n_bus
    a, b = N, N + 1
    n = net.copy()
    n.n_bus = N + 2
    n.br_from = np.concatenate([net.br_from, [k, a]]).astype(np.int32)
    n.br_to = np.concatenate([net.br_to, [a, b]]).astype(np.int32)
    n.br_r = np.concatenate([net.br_r, [0.01, 0.02]])
    n.br_x = np.concatenate([net.br_x, [0.1, 0.15]])
    n.br_b = np.concatenate([net.br_b, [0.01, 0.02]])
    n.br_tap = np.concatenate([net.br_tap, [1.0, 1.0]])
    n.br_shift_deg = np.concatenate([net.br_shift_deg, [0.0, 0.0]])
    n.br_status = np.concatenate([net.br_status, [1, 1]]).astype(np.int32)
    n.load_bus = np.concatenate([net.load_bus, [a, b]]).astype(np.int32)
    n.load_p = np.concatenate([net.load_p, [0.1, 0.2]])
    n.load_q = np.concatenate([net.load_q, [0.03, 0.06]])
    n.coords = None
    return n, net.n_branch   # index of the bridge


def test_newton_host_solve_reports_singular_island(cuda):
    """Newton (pf_newton, SuperLU on the host) on a network whose bridge to
    a two-bus island is out of service: the first solve meets a singular
    Jacobian and the call ends with PF_ESOLVE; x holds the start."""
    from paper_2011_11880_amd.api import Plan
    from paper_2011_11880_amd.capi import PF_ESOLVE, PFError
    net0, bridge = _with_pendant_pair(synth.tiny_grid(10), 5)
    net = net0.without_branch(bridge)
    p = Plan(net)
    y0 = synth.random_states(net, seed=4)
    x = torch.from_numpy(y0).to(cuda)
    with pytest.warns(Warning):   # SuperLU: the matrix is exactly singular
        with pytest.raises(PFError) as ei:
            p.newton(x, max_iter=5)
    assert ei.value.code == PF_ESOLVE
    torch.cuda.synchronize()
    assert np.array_equal(x.cpu().numpy(), y0)


def test_newton_batch_islanding_outages_stay_in_their_instance(ora, cuda):
    """N-1 batch on the 200-bus grid (with a pendant two-bus feeder) from a
    perturbed start.  Taking out the only branch of a load bus zeroes that
    bus's angle column exactly: the factorisation meets a zero pivot and the
    instance ends non-finite.  Taking out the bridge to the two-bus feeder
    leaves the feeder without an angle reference: its pivots are rounding
    residue, the steps diverge and the instance does not converge.  Every
    other instance matches the oracle's Newton and ends bit for bit as in the
    same batch with those two outages replaced by the base case."""
    from paper_2011_11880_amd.api import Plan
    import test_gpu_newton_device as D
    net1, bridge = _with_pendant_pair(synth.tiny_grid(10), 5)
    net, ystar, y0 = D._manufactured(ora, net1, 10)
    nonb = set(synth.non_bridge_branches(net).tolist())
    bridges = [e for e in range(net.n_branch) if e not in nonb and net.br_status[e]]
    assert bridge in bridges
    # the only branch of a bus without a generator
    deg = np.bincount(np.concatenate([net.br_from, net.br_to]), minlength=net.n_bus)
    gen = set(net.pv_bus.tolist()) | set(net.slack_bus.tolist())
    leaf = next(e for e in bridges
                for u in (int(net.br_from[e]), int(net.br_to[e])) if deg[u] == 1 and u not in gen)
    I = 70
    out = np.full(I, -1, np.int32)
    out[1:] = synth.contingencies(net, I - 1, seed=21)
    isl = [5, 40]
    out_a = out.copy()
    out_a[isl[0]] = leaf
    out_a[isl[1]] = bridge
    out_b = out.copy()
    out_b[isl] = -1
    res = []
    for o in (out_a, out_b):
        p = Plan(net, batch=dict(n_inst=I, outage=o))
        X = torch.from_numpy(p.to_batch(np.tile(y0, (I, 1)))).to(cuda)
        rep = p.newton_batch(X, tol=1e-10, max_iter=10)
        torch.cuda.synchronize()
        res.append((rep, p.from_batch(X)))
    (rep_a, Xa), (rep_b, Xb) = res
    for i in isl:
        assert not rep_a["inst_norm"][i] < 1e-10, i   # NaN or above tol
    assert not np.all(np.isfinite(Xa[isl[0]]))
    assert not np.isfinite(rep_a["inst_norm"][isl[0]])
    others = [i for i in range(I) if i not in isl]
    assert np.array_equal(Xa[others], Xb[others])
    assert np.array_equal(rep_a["inst_iterations"][others], rep_b["inst_iterations"][others])
    assert rep_a["n_converged"] == rep_b["n_converged"] - len(isl)
    for i in others[::7]:
        v = net if out[i] < 0 else net.without_branch(int(out[i]))
        y, norms, _ = ora.newton(v, y0, tol=1e-10, max_iter=10)
        assert (norms[-1] < 1e-10) == (rep_a["inst_norm"][i] < 1e-10), i
        if norms[-1] < 1e-10:
            np.testing.assert_allclose(Xa[i], y, rtol=0, atol=1e-9)
