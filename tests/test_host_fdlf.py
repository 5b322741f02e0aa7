"""The library's fast-decoupled matrices (host side, no GPU) against the
oracle's, and the FDLF entry points' argument checks."""

import numpy as np
import pytest

from paper_2011_11880_amd import capi, synth
from paper_2011_11880_amd.api import Plan
from paper_2011_11880_amd.capi import PFError
from test_oracle_pins import _net_with_everything


@pytest.mark.parametrize("which", ["everything", "meshed", "10k"])
def test_matrices_match_oracle(ora, which):
    net = {"everything": _net_with_everything, "meshed": lambda: synth.grid_meshed(300, 3),
           "10k": synth.grid_10k}[which]()
    p = Plan(net, host_only=True)
    Bp, Bpp, bus_p, bus_q = p.fdlf_matrices()
    Op, Opp, rp, rq = ora.fdlf_matrices(net)
    assert np.array_equal(bus_p, rp) and np.array_equal(bus_q, rq)
    for A, B in ((Bp, Op), (Bpp, Opp)):
        assert np.array_equal(A.indptr, B.indptr) and np.array_equal(A.indices, B.indices)
        np.testing.assert_allclose(A.data, B.data, rtol=1e-15, atol=0)


def test_argument_checks():
    L = capi.lib()
    nets = [synth.tiny_grid(1, n_bus=30, n_branch=40, n_pv=4), synth.tiny_grid(2)]
    with pytest.raises(PFError):   # multi-grid plans are not supported
        Plan.multi(nets, host_only=True).fdlf_matrices()
    assert L.pf_fdlf_matrices(None, None, None, None, None, None, None, None, None, None,
                              None) == capi.PF_EINVAL
    p = Plan(synth.tiny_grid(3), host_only=True)
    h = capi._vp()
    assert L.pf_fdlf_create(p._h, None, None, h) == capi.PF_EINVAL   # host-only plan
    assert L.pf_fdlf_solve(None, None, None, None, None) == capi.PF_EINVAL
    assert L.pf_lu_solve(None, None, None) == capi.PF_EINVAL
    L.pf_fdlf_destroy(None)
    L.pf_lu_destroy(None)
