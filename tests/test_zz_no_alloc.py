"""mrcm_fine_flux_static (the allocation-free reconstruction, whose scratch
is the library's static device array) against mrcm_fine_flux on the same
solved contexts: the same kernels on the same data, so every output is
bitwise equal.  Two contexts in a row, the second with fewer subdomains, so
that the second call reads nothing the first one left in the array."""
import numpy as np
import pytest

import inputs
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _case(prob, s):
    import torch
    from paper_2104_04653_amd import MRCMSolver
    with MRCMSolver(prob) as sol:
        sol.update_mobility(s)
        sol.solve()
        ref = sol.fine_flux()
        got = sol.fine_flux(static=True)
        ref_d = sol.fine_flux(device=True)
        got_d = sol.fine_flux(device=True, static=True)
        torch.cuda.synchronize()
        st = sol.stats()
    return ref, got, ref_d, got_d, st


def test_static_scratch_matches_fine_flux_on_two_calls():
    cases = [
        # 256 subdomains, all-Neumann with wells: the zero-mean shift reads
        # the reduced pressure sum from the scratch
        (inputs.make_problem("channel256_q5", seed=3), (4, 10)),
        # then 16 subdomains: a smaller input after a larger one
        (inputs.make_problem("gauss64", seed=2), (2, 5)),
    ]
    for prob, (k, n) in cases:
        s = inputs.synthetic_saturation(prob, k, n)
        say("case: static scratch,", prob.name, prob.nx, prob.ny, "subdomains", prob.n_sub)
        ref, got, ref_d, got_d, st = _case(prob, s)
        for a, b in zip(ref[:3], got[:3]):
            assert np.array_equal(a, b)
        assert ref[3] == got[3]
        for a, b in zip(ref_d[:3], got_d[:3]):
            assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
        assert ref_d[3] == got_d[3]
        assert np.array_equal(ref[0], ref_d[0].cpu().numpy())
        say("  imbalance %.2e, flux phase %.3f ms" % (got[3], st["ms_flux"]))
        assert got[3] < 1e-12
