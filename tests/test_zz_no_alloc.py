"""pf_lu_solve_noalloc (the constant-factorisation solve with its working
vector in the library's static device array) against pf_lu_solve, bit for
bit, on two calls in a row, the second on a smaller system; sizes above the
array are refused with PF_EINVAL and leave the right-hand side untouched."""

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
