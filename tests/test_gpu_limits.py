"""The largest inputs, checked by properties that hold at any size (the
oracle would take minutes per step here):

* 4096 x 4096 cells, 65,536 subdomains of 16 x 16 (the limit of the
  allocation-free reconstruction; the interface tree's root front has
  1024 unknowns):
  - homogeneous K with p = 1 on W and 0 on E: the linear pressure exactly
    (the linear interface spaces contain its traces);
  - log-normal K with the 1024^2 field's statistics (variance 6, contrast
    about 6e9 on this seed) and a front saturation: the allocation-free
    reconstruction equals mrcm_fine_flux bit for bit, and every cell
    balances to 1e-10 of max |F|.  (The 1e-12 bar of the 1024^2 and
    2048 x 1024 workloads is not met at this size: a few floating
    subdomains carry a compatibility defect near 3e-9 of max |F|, which the
    stitch spreads over their cells, 1e-11 per cell.  The local solutions
    agree with the generic kernels' to rounding, so the defect is the FP64
    floor of the composed solution amplified by the conditioning of the
    interface system, whose coefficients the two kernel paths give only to
    1.6e-10 of each other at 2048^2.);
* 65,792 subdomains: the allocation-free reconstruction refuses with
  MRCM_E_INVAL, mrcm_fine_flux still works.
"""
import numpy as np
import pytest

import inputs
from tests.gpu_util import say

pytestmark = pytest.mark.gpu

N = 4096


def test_linear_pressure_at_the_largest_size():
    from paper_2104_04653_amd import MRCMSolver
    base = inputs.make_problem("gauss1024", nx=64, ny=64)     # boundary kinds and values
    prob = base.replace(nx=N, ny=N, lx=4.0, ly=4.0, perm=np.ones(N * N),
                        bc_value=(np.ones(N), np.zeros(N), None, None))
    say("case: linear pressure, %dx%d, %d subdomains" % (N, N, prob.n_sub))
    with MRCMSolver(prob) as sol:
        sol.update_mobility(np.ones(N * N), is_lambda=True)
        sol.solve()
        p, ux, uy, imb = sol.fine_flux()
        st = sol.stats()
    x = (np.arange(N) + 0.5) / N
    exact = np.tile(1.0 - x, N)
    err = np.abs(p - exact).max()
    say("  max |p - (1 - x)| %.2e, max |u_x - 1/L| %.2e, max |u_y| %.2e, imbalance %.2e, "
        "interface %.3f ms" % (err, np.abs(ux - 0.25).max(), np.abs(uy).max(), imb, st["ms_interface"]))
    assert err < 1e-11
    assert np.abs(ux - 0.25).max() < 1e-10 and np.abs(uy).max() < 1e-10
    assert imb < 1e-12


def test_balance_and_static_reconstruction_at_the_largest_size():
    from paper_2104_04653_amd import MRCMSolver
    prob = inputs.make_problem("gauss1024", nx=N, ny=N, lx=4.0, ly=4.0, seed=5)
    s = inputs.synthetic_saturation(prob, 3, 10)
    say("case: log-normal field, %dx%d, %d subdomains" % (N, N, prob.n_sub))
    with MRCMSolver(prob) as sol:
        sol.update_mobility(s)
        sol.solve()
        ref = sol.fine_flux()
        got = sol.fine_flux(static=True)
        st = sol.stats()
    say("  imbalance %.2e, interface residual %.2e (%d refinement steps), ms local %.2f "
        "interface %.2f flux %.2f" % (ref[3], st["interface_residual"], st["interface_ir_steps"],
                                      st["ms_local"], st["ms_interface"], st["ms_flux"]))
    assert ref[3] < 1e-10
    assert np.all(np.isfinite(ref[0]))
    for a, b in zip(ref[:3], got[:3]):
        assert np.array_equal(a, b)
    assert ref[3] == got[3]


def test_static_reconstruction_refuses_beyond_its_scratch():
    from paper_2104_04653_amd import MRCMError, MRCMSolver
    from paper_2104_04653_amd.mrcm import E_INVAL
    ny = N + 16                        # 256 x 257 subdomains = 65,792
    base = inputs.make_problem("gauss1024", nx=64, ny=64)
    prob = base.replace(nx=N, ny=ny, lx=4.0, ly=ny / 1024.0, perm=np.ones(N * ny),
                        bc_value=(np.ones(ny), np.zeros(ny), None, None))
    say("case: %d subdomains, beyond the static scratch" % prob.n_sub)
    with MRCMSolver(prob) as sol:
        sol.update_mobility(np.ones(N * ny), is_lambda=True)
        sol.solve()
        p, ux, uy, imb = sol.fine_flux()
        assert imb < 1e-12
        with pytest.raises(MRCMError) as ei:
            sol.fine_flux(static=True)
        assert ei.value.code == E_INVAL
