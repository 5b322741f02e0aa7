"""GPU parity of the single-instance kernel (pf_eval / pf_eval_residual /
pf_eval_jacobian) against the CPU oracle, through the C ABI.

Cases: the 200-bus tiny grid, a grid with shunts, transformers and parallel
branches, a hub bus whose admittance row spans many 64-entry chunks, a
one-bus network, the 70,000-bus grid, bit-reproducibility across runs and
across every schedule."""

import sys

import numpy as np
import pytest

from paper_2011_11880_amd import synth
from parity import check_close, check_jacobian

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _plan(net, **kw):
    from paper_2011_11880_amd.api import Plan
    return Plan(net, **kw)


def _eval(plan, y, cuda):
    x = torch.from_numpy(y).to(cuda)
    F, J = plan.eval(x)
    torch.cuda.synchronize()
    return F.cpu().numpy(), J.cpu().numpy()


def _check_state(ora, plan, net, y, cuda, what):
    F, J = _eval(plan, y, cuda)
    Fo, So = ora.residual(net, y)
    Jo, Ao = ora.jacobian(net, y)
    rp, ci = plan.pattern()
    nf = check_close(F, Fo, So, what + " F")
    nj = check_jacobian(rp, ci, J, Jo, Ao, what + " J")
    return nf, nj


def _hub_grid(n_leaf=300, seed=5):
    """Bus 0 joined to every other bus (row of n_leaf + 1 entries), plus a
    ring among the leaves."""
    rng = np.random.default_rng(seed)
    N = n_leaf + 1
    f = [0] * n_leaf + list(range(1, N))
    t = list(range(1, N)) + list(range(2, N)) + [1]
    B = len(f)
    r, x, b, tap, sh = synth._branch_params(rng, B)
    loads = np.arange(2, N)
    return synth.Network(n_bus=N, br_from=f, br_to=t, br_r=r, br_x=x, br_b=b, br_tap=tap,
                         br_shift_deg=sh, br_status=np.ones(B), load_bus=loads,
                         load_p=rng.uniform(0, 1, loads.size), load_q=rng.uniform(0, .3, loads.size),
                         pv_bus=[1], pv_p=[1.0], pv_v=[1.02], slack_bus=[0], slack_v=[1.0],
                         slack_theta=[0.0], shunt_bus=[0, 3, 3], shunt_g=[0.01, 0.0, 0.002],
                         shunt_b=[0.1, 0.2, -0.05])


def test_tiny_grid_parity(ora, cuda):
    net = synth.tiny_grid(0)
    p = _plan(net)
    for s in range(4):
        _say("tiny grid state", s)
        _check_state(ora, p, net, synth.random_states(net, seed=s), cuda, f"tiny s{s}")


def test_everything_grid_parity(ora, cuda):
    net = synth.with_parallel_branches(synth.tiny_grid(3, n_bus=120, n_branch=170, n_pv=20,
                                                       n_shunt=15), 12, 9)
    net.br_status[5] = 0  # an out-of-service branch stays out of the model
    if len(set(map(int, net.br_from[net.br_status == 1])) |
           set(map(int, net.br_to[net.br_status == 1]))) < net.n_bus:
        net.br_status[5] = 1
    p = _plan(net)
    for s in range(3):
        _check_state(ora, p, net, synth.random_states(net, seed=10 + s), cuda, f"everything s{s}")


def test_hub_row_spans_chunks(ora, cuda):
    net = _hub_grid()
    for te in (64, 128, 512):
        p = _plan(net, schedule=dict(tile_entries=te))
        _say("hub grid tile_entries", te)
        _check_state(ora, p, net, synth.random_states(net, seed=te), cuda, f"hub te{te}")


def test_single_bus(ora, cuda):
    net = synth.Network(n_bus=1, br_from=[], br_to=[], br_r=[], br_x=[], br_b=[], br_tap=[],
                        br_shift_deg=[], br_status=[], load_bus=[0], load_p=[0.3], load_q=[0.1],
                        pv_bus=[], pv_p=[], pv_v=[], slack_bus=[0], slack_v=[1.0],
                        slack_theta=[0.1], shunt_bus=[0], shunt_g=[0.1], shunt_b=[0.2])
    p = _plan(net)
    y = np.array([0.05, 1.02, 0.3, 0.7])
    _check_state(ora, p, net, y, cuda, "one bus")


def test_entry_points_agree_bitwise(cuda):
    net = synth.tiny_grid(1, n_shunt=4)
    p = _plan(net)
    x = torch.from_numpy(synth.random_states(net, seed=3)).to(cuda)
    F, J = p.eval(x)
    F2 = p.eval_residual(x)
    J2 = p.eval_jacobian(x)
    torch.cuda.synchronize()
    assert torch.equal(F, F2) and torch.equal(J, J2)


SCHEDULES = [
    dict(tile_entries=64, waves_per_block=1, grid_blocks=-1, xcd_remap=2),
    dict(tile_entries=128, waves_per_block=4, grid_blocks=-1, xcd_remap=1),
    dict(tile_entries=256, waves_per_block=8, grid_blocks=3, xcd_remap=1),
    dict(tile_entries=1024, waves_per_block=2, grid_blocks=64, xcd_remap=2),
    dict(tile_entries=4096, waves_per_block=4, grid_blocks=9, xcd_remap=1),
]


def test_bitwise_across_runs_and_schedules(cuda):
    net = synth.grid_10k()
    p = _plan(net)
    x = torch.from_numpy(synth.random_states(net, seed=7)).to(cuda)
    F0, J0 = p.eval(x)
    for s in SCHEDULES:
        p.schedule = dict(p.schedule, **s)
        for _ in range(2):
            F, J = p.eval(x)
            torch.cuda.synchronize()
            assert torch.equal(F, F0) and torch.equal(J, J0), s


def test_70k_grid_parity(ora, cuda):
    net = synth.grid_70k()
    p = _plan(net)
    assert p.n == 150002
    counts = []
    for s in range(2):
        _say("70k state", s)
        counts.append(_check_state(ora, p, net, synth.random_states(net, seed=100 + s), cuda,
                                   f"70k s{s}"))
    _say("fallback counts (F, J):", counts)


def test_nan_state_propagates(cuda):
    net = synth.tiny_grid(0)
    p = _plan(net)
    y = synth.random_states(net, seed=1)
    y[net.n_bus + 5] = np.nan
    F, J = _eval(p, y, cuda)
    assert np.isnan(F[5]) and np.isnan(F[net.n_bus + 5])
    touched = {5} | set(net.br_to[net.br_from == 5].tolist()) | set(net.br_from[net.br_to == 5].tolist())
    far = [i for i in range(net.n_bus) if i not in touched]
    assert np.all(np.isfinite(F[far]))


def test_single_instance_graph_replay(cuda):
    """Launches of the single-instance kernel captured in a graph (as the
    benchmark's plain leg runs them) replay to the eager results."""
    from paper_2011_11880_amd.api import Plan
    net = synth.grid_10k()
    p = Plan(net)
    Y = synth.random_states(net, 3, seed=5)
    X = torch.from_numpy(Y).to(cuda)
    F0 = torch.stack([p.eval(X[s])[0] for s in range(3)])
    J0 = torch.stack([p.eval(X[s])[1] for s in range(3)])
    F = torch.zeros_like(F0)
    J = torch.zeros_like(J0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            for s in range(3):
                p.eval(X[s], F[s], J[s])
    torch.cuda.synchronize()
    for r in range(3):
        F.fill_(-1.0)
        J.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(F, F0) and torch.equal(J, J0), r
