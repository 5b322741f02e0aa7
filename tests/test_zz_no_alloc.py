"""pf_lu_solve_noalloc (the constant-factorisation solve with its working
vector in the library's static device array) against pf_lu_solve, bit for
bit, on two calls in a row, the second on a smaller system; sizes above the
array are refused with PF_EINVAL and leave the right-hand side untouched; a
captured solve replays from a HIP graph to the eager result."""

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2011_11880_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def cuda():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def test_noalloc_solve_equals_solve(cuda):
    from paper_2011_11880_amd.api import DeviceSparseLU, Plan
    Bp, _, _, _ = Plan(synth.grid_meshed(10000, 2100), host_only=True).fdlf_matrices()
    _, Bpp, _, _ = Plan(synth.grid_meshed(300, 3), host_only=True).fdlf_matrices()
    assert Bpp.shape[0] < Bp.shape[0]
    rng = np.random.default_rng(1)
    for M in (Bp, Bpp):
        lu = DeviceSparseLU(M)
        b = rng.normal(size=M.shape[0])
        ref = torch.from_numpy(b).to(cuda)
        lu.solve(ref)
        y = torch.from_numpy(b).to(cuda)
        lu.solve(y, noalloc=True)
        torch.cuda.synchronize()
        assert torch.equal(y, ref)
        yh = y.cpu().numpy()
        assert np.max(np.abs(M @ yh - b)) <= 1e-11 * (abs(M).max() * np.max(np.abs(yh)) + 1)
        lu.close()


def test_noalloc_refuses_more_than_the_array(cuda):
    from paper_2011_11880_amd.api import DeviceSparseLU
    from paper_2011_11880_amd.capi import PF_EINVAL, PFError
    n = (1 << 20) + 1
    d = np.random.default_rng(2).uniform(1.0, 2.0, n)
    lu = DeviceSparseLU(sp.diags(d).tocsr())
    b = torch.ones(n, dtype=torch.float64, device=cuda)
    with pytest.raises(PFError) as ei:
        lu.solve(b, noalloc=True)
    assert ei.value.code == PF_EINVAL
    assert torch.all(b == 1.0)
    lu.solve(b)
    torch.cuda.synchronize()
    assert np.allclose(b.cpu().numpy(), 1.0 / d, rtol=1e-15, atol=0)
    lu.close()


def test_noalloc_solve_replays_from_a_graph(cuda):
    """The callers the no-allocation entry point is for include code under
    graph capture: a solve captured into a HIP graph replays, three times with
    eager solves of other right-hand sides between the replays, to the eager
    result bit for bit each time."""
    from paper_2011_11880_amd.api import DeviceSparseLU, Plan
    Bp, _, _, _ = Plan(synth.grid_meshed(2000, 2200), host_only=True).fdlf_matrices()
    lu = DeviceSparseLU(Bp)
    rng = np.random.default_rng(3)
    b0 = torch.from_numpy(rng.normal(size=Bp.shape[0])).to(cuda)
    ref = b0.clone()
    lu.solve(ref, noalloc=True)
    y = b0.clone()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):          # warm-up on the capture stream
        y.copy_(b0)
        lu.solve(y, noalloc=True)
    torch.cuda.current_stream().wait_stream(st)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        y.copy_(b0)
        lu.solve(y, noalloc=True)
    for k in range(3):
        other = torch.from_numpy(rng.normal(size=Bp.shape[0])).to(cuda)
        lu.solve(other, noalloc=True)    # the shared array holds another solve's data
        torch.cuda.synchronize()
        y.fill_(7.0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, ref), k
    del g
    lu.close()
