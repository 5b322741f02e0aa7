"""The autotuner (pf_autotune / pf_autotune_cached) on small batched,
multi-grid and single-instance plans: the schedule it picks gives outputs
bit-identical to the default schedule's and equal to the oracle's; the tune
cache returns the stored schedule without timing on a hit, keys plans of
another shape apart, and accepts the schedule the search wrote."""

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


def _net():
    net = synth.tiny_grid(4, n_bus=150, n_branch=210, n_pv=25, n_shunt=12)
    return synth.with_parallel_branches(net, 8, 3)


def _batched(net, I):
    from paper_2011_11880_amd.api import Plan
    ls, ps = synth.batch_scenarios(net, I, seed=7)
    out = np.full(I, -1, np.int32)
    out[::3] = synth.contingencies(net, len(out[::3]), seed=7)
    spec = dict(n_inst=I, load_scale=ls, pv_scale=ps, outage=out)
    return Plan(net, batch=spec), spec


def _lines(path):
    with open(path) as fh:
        return [ln for ln in fh.read().splitlines() if ln.strip()]


def test_batched_autotune_and_cache(ora, cuda, tmp_path):
    import test_gpu_batch as TB
    net = _net()
    I = 130
    bp, spec = _batched(net, I)
    default = dict(bp.schedule)
    Y = synth.random_states(net, I, seed=8)
    X = torch.from_numpy(bp.to_batch(Y)).to(cuda)
    F0, J0 = bp.eval_batch(X)
    cache = tmp_path / "tune.txt"
    F = torch.empty_like(F0)
    J = torch.empty_like(J0)
    best = bp.autotune(X, F, J, reps=3, cache=cache)
    assert not bp.tune_hit and bp.schedule == best
    assert len(_lines(cache)) == 1
    F1, J1 = bp.eval_batch(X)
    torch.cuda.synchronize()
    assert torch.equal(F1, F0) and torch.equal(J1, J0), (best, default)
    rp, ci = bp.pattern()
    Fh, Jh = bp.from_batch(F1), bp.from_batch(J1)
    for k in (0, 1, 64, I - 1):
        nk = TB._instance_net(net, spec, k)
        Fo, So = ora.residual(nk, Y[k])
        Jo, Ao = ora.jacobian(nk, Y[k])
        check_close(Fh[k], Fo, So, f"tuned inst {k} F")
        check_jacobian(rp, ci, Jh[k], Jo, Ao, f"tuned inst {k} J")
    # a second plan of the same shape takes the stored schedule, untimed
    bp2, _ = _batched(net, I)
    got = bp2.autotune(X, F, J, reps=3, cache=cache)
    assert bp2.tune_hit and got == best and bp2.schedule == best
    assert len(_lines(cache)) == 1
    # another instance count is another key
    bp3, _ = _batched(net, 70)
    X3 = torch.from_numpy(bp3.to_batch(Y[:70])).to(cuda)
    bp3.autotune(X3, None, torch.empty((bp3.nnz, 70), dtype=torch.float64, device=cuda),
                 reps=2, cache=cache)
    assert not bp3.tune_hit and len(_lines(cache)) == 2
    # the residual-only launch is keyed apart from the fused one
    bp4, _ = _batched(net, I)
    bp4.autotune(X, F, None, reps=2, cache=cache)
    assert not bp4.tune_hit and len(_lines(cache)) == 3


def test_multi_grid_autotune(ora, cuda, tmp_path):
    from paper_2011_11880_amd.api import Plan
    import test_gpu_multi as TM
    nets = [synth.tiny_grid(1, n_bus=30, n_branch=40, n_pv=4, n_shunt=2), TM._one_bus(),
            synth.tiny_grid(2, n_bus=300, n_branch=420, n_pv=30, n_shunt=10),
            synth.geometric_grid(2000, 2500, 286, 1143, 100, seed=77)]
    mp = Plan.multi(nets)
    ys = [synth.random_states(n, seed=50 + g) for g, n in enumerate(nets)]
    x = torch.from_numpy(np.concatenate(ys)).to(cuda)
    F0, J0 = mp.eval(x)
    F = torch.empty_like(F0)
    J = torch.empty_like(J0)
    cache = tmp_path / "tune.txt"
    best = mp.autotune(x, F, J, reps=3, cache=cache)
    F1, J1 = mp.eval(x)
    torch.cuda.synchronize()
    assert torch.equal(F1, F0) and torch.equal(J1, J0), best
    F1, J1 = F1.cpu().numpy(), J1.cpu().numpy()
    for g, net in enumerate(nets):
        x0, x1 = mp.x_off[g], mp.x_off[g + 1]
        j0, j1 = mp.j_off[g], mp.j_off[g + 1]
        Fo, So = ora.residual(net, ys[g])
        Jo, Ao = ora.jacobian(net, ys[g])
        check_close(F1[x0:x1], Fo, So, f"tuned grid {g} F")
        rp, ci = Plan(net, host_only=True).pattern()
        check_jacobian(rp, ci, J1[j0:j1], Jo, Ao, f"tuned grid {g} J")
    mp2 = Plan.multi(nets)
    assert mp2.autotune(x, F, J, reps=3, cache=cache) == best and mp2.tune_hit
    F2, J2 = mp2.eval(x)
    torch.cuda.synchronize()
    assert torch.equal(F2, F0) and torch.equal(J2, J0)


def test_single_instance_autotune_retiles(cuda, tmp_path):
    """The single-instance search changes the tile size (the tile tables are
    rebuilt); whatever it picks, and a cached tile size applied to a fresh
    plan, leave the outputs unchanged."""
    from paper_2011_11880_amd.api import Plan
    import test_gpu_eval as E
    net = E._hub_grid()
    p = Plan(net)
    x = torch.from_numpy(synth.random_states(net, seed=3)).to(cuda)
    F0, J0 = p.eval(x)
    cache = tmp_path / "tune.txt"
    best = p.autotune(x, torch.empty_like(F0), torch.empty_like(J0), reps=3, cache=cache)
    F1, J1 = p.eval(x)
    torch.cuda.synchronize()
    assert torch.equal(F1, F0) and torch.equal(J1, J0), best
    # a hand-written cache line with another tile size is taken as given
    key = _lines(cache)[0].split(" ")[0]
    other = 512 if best["tile_entries"] != 512 else 128
    with open(cache, "a") as fh:
        fh.write(f"{key} {other} 2 -1 1 1 1 64 0.0\n")
    p2 = Plan(net)
    got = p2.autotune(x, torch.empty_like(F0), torch.empty_like(J0), reps=3, cache=cache)
    assert p2.tune_hit and got["tile_entries"] == other and p2.info["n_tiles"] != 0
    F2, J2 = p2.eval(x)
    torch.cuda.synchronize()
    assert torch.equal(F2, F0) and torch.equal(J2, J0)
