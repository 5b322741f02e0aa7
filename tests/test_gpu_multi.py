"""GPU parity of the multi-grid plan (pf_setup_multi + pf_eval): grids of
uneven size evaluated in one launch, each checked against the oracle and
bit-identical to its own single-grid plan."""

import numpy as np
import pytest

from paper_2011_11880_amd import synth
from parity import check_close, check_jacobian

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def _one_bus():
    return synth.Network(n_bus=1, br_from=[], br_to=[], br_r=[], br_x=[], br_b=[], br_tap=[],
                         br_shift_deg=[], br_status=[], load_bus=[0], load_p=[0.2], load_q=[0.1],
                         pv_bus=[], pv_p=[], pv_v=[], slack_bus=[0], slack_v=[1.0],
                         slack_theta=[0.0], shunt_bus=[], shunt_g=[], shunt_b=[])


def _check_multi(ora, nets, idx, cuda, schedule=None):
    from paper_2011_11880_amd.api import Plan
    mp = Plan.multi(nets, schedule=schedule)
    ys = [synth.random_states(n, seed=40 + g) for g, n in enumerate(nets)]
    x = torch.from_numpy(np.concatenate(ys)).to(cuda)
    F, J = mp.eval(x)
    torch.cuda.synchronize()
    F, J = F.cpu().numpy(), J.cpu().numpy()
    for g in idx:
        net = nets[g]
        x0, x1 = mp.x_off[g], mp.x_off[g + 1]
        j0, j1 = mp.j_off[g], mp.j_off[g + 1]
        Fo, So = ora.residual(net, ys[g])
        Jo, Ao = ora.jacobian(net, ys[g])
        check_close(F[x0:x1], Fo, So, f"grid {g} F")
        sp = Plan(net)
        rp, ci = sp.pattern()
        check_jacobian(rp, ci, J[j0:j1], Jo, Ao, f"grid {g} J")
        Fs, Js = sp.eval(torch.from_numpy(ys[g]).to(cuda))
        torch.cuda.synchronize()
        assert np.array_equal(Fs.cpu().numpy(), F[x0:x1])
        assert np.array_equal(Js.cpu().numpy(), J[j0:j1])
    return mp


def test_small_uneven_grids(ora, cuda):
    nets = [synth.tiny_grid(1, n_bus=30, n_branch=40, n_pv=4, n_shunt=2), _one_bus(),
            synth.tiny_grid(2, n_bus=300, n_branch=420, n_pv=30, n_shunt=10),
            synth.with_parallel_branches(synth.tiny_grid(3, n_bus=80, n_branch=100, n_pv=9), 5, 1),
            synth.geometric_grid(2000, 2500, 286, 1143, 100, seed=77)]
    for sched in (None, dict(tile_entries=64, grid_blocks=3), dict(tile_entries=2048)):
        _check_multi(ora, nets, range(len(nets)), cuda, sched)


def test_256_uneven_grids(ora, cuda):
    """The 256-grid launch: every grid against the oracle and bit-identical
    to its own single-grid plan."""
    nets = synth.uneven_grids(256, seed=3000)
    mp = _check_multi(ora, nets, range(len(nets)), cuda)
    assert mp.info["n_grids"] == 256
