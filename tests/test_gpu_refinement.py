"""Stopping rules of the two iterative refinements, driven to their
fallback and failure paths from the host (GPU, through the C ABI).

* FP32 + FP64 refinement of the local solves: with no refinement step
  allowed, every subdomain ends above the tolerance and is re-solved by the
  FP64 kernels (the listed re-solve); the basis functions and interface
  blocks are then those of the FP64 form, bit for bit.
* Refinement of the FP64 interface solve: a failure bound it cannot reach
  makes the solve fail with MRCM_E_NO_CONV and leaves no solution behind.

These are ordinary numerical outcomes forced by settings; every kernel runs
to completion.
"""
import numpy as np
import pytest

import inputs
from oracle.discretization import total_mobility
from tests.gpu_util import rel, run_oracle, say

pytestmark = pytest.mark.gpu


def solve(prob, lam, precision, refinement=None, interface=None):
    from paper_2104_04653_amd import MRCMSolver
    with MRCMSolver(prob, precision=precision) as sol:
        if refinement is not None:
            sol.set_refinement(*refinement)
        if interface is not None:
            sol.set_interface_refinement(*interface)
        sol.update_mobility(lam, is_lambda=True)
        sol.solve()
        p, ux, uy, imb = sol.fine_flux()
        return dict(p=p, ux=ux, uy=uy, imb=imb, stats=sol.stats(), basis=sol.basis(),
                    blocks=sol.local_blocks())


@pytest.mark.parametrize("workload,kw", [
    ("gauss64", dict(seed=2)),                                                   # 16 x 16 kernels
    ("channel2048x1024", dict(nx=256, ny=128, lx=0.25, ly=0.125, seed=2)),       # 32 x 32 kernels
])
def test_fp32_every_subdomain_falls_back(workload, kw):
    prob = inputs.make_problem(workload, **kw)
    lam = total_mobility(inputs.synthetic_saturation(prob, 2, 5), prob.mu_w, prob.mu_o)
    say("case: FP32 refinement with no step allowed,", workload, prob.nx, prob.ny, "sub", prob.sub_nx)
    a = solve(prob, lam, "fp32_ir", refinement=(0, 1e-9))
    b = solve(prob, lam, "fp64")
    st = a["stats"]
    say("  fallbacks %d of %d, refinement steps %d; interface refinement %d / %d"
        % (st["fallbacks"], st["n_sub"], st["ir_iters_max"], st["interface_ir_steps"],
           b["stats"]["interface_ir_steps"]))
    assert st["fallbacks"] == st["n_sub"] and st["ir_iters_max"] == 0
    assert np.array_equal(a["basis"], b["basis"])
    assert np.array_equal(a["blocks"], b["blocks"])
    if st["interface_ir_steps"] == b["stats"]["interface_ir_steps"]:
        for k in ("p", "ux", "uy"):
            assert np.array_equal(a[k], b[k])
    else:   # the two forms refine the interface solve to different tolerances
        assert rel(a["p"], b["p"]) < 1e-11
    assert a["imb"] < 1e-12


def test_fp32_partial_fallback_stays_within_tolerance():
    """One refinement step at most: the subdomains it does not converge go to
    the FP64 re-solve, the rest keep their FP32 + one-step solution; the
    result stays within the form's 1e-8 of the oracle."""
    prob = inputs.make_problem("gauss64", seed=3)
    lam = total_mobility(inputs.synthetic_saturation(prob, 4, 8), prob.mu_w, prob.mu_o)
    say("case: FP32 refinement with one step")
    a = solve(prob, lam, "fp32_ir", refinement=(1, 1e-9))
    ref = run_oracle(prob, lam=lam)
    st = a["stats"]
    ep, ef = rel(a["p"], ref.p), rel(np.r_[a["ux"], a["uy"]], np.r_[ref.ux, ref.uy])
    say("  fallbacks %d of %d; p %.2e flux %.2e imbalance %.2e" % (st["fallbacks"], st["n_sub"],
                                                                     ep, ef, a["imb"]))
    assert st["ir_iters_max"] <= 1
    assert ep < 1e-8 and ef < 1e-8 and a["imb"] < 1e-12


def test_interface_refinement_failure_is_reported():
    from paper_2104_04653_amd import MRCMError, MRCMSolver
    from paper_2104_04653_amd.mrcm import E_INVAL, E_NO_CONV, E_STATE
    prob = inputs.make_problem("gauss64", seed=1)
    s = inputs.synthetic_saturation(prob, 2, 5)
    say("case: interface refinement out of reach")
    with MRCMSolver(prob) as sol:
        good = None
        sol.update_mobility(s)
        sol.solve()
        good = sol.fine_flux()
        for max_steps in (0, 2):
            sol.set_interface_refinement(max_steps, 1e-300, 1e-300)
            with pytest.raises(MRCMError) as ei:
                sol.solve()
            assert ei.value.code == E_NO_CONV
            assert sol.stats()["interface_ir_steps"] == max_steps
            with pytest.raises(MRCMError) as ei:
                sol.fine_flux()
            assert ei.value.code == E_STATE
            with pytest.raises(MRCMError) as ei:
                sol.step(s)
            assert ei.value.code == E_NO_CONV
        with pytest.raises(MRCMError) as ei:
            sol.set_interface_refinement(3, 1e-14, 0.0)
        assert ei.value.code == E_INVAL
        with pytest.raises(MRCMError) as ei:
            sol.set_refinement(3, 1e-9)        # not an FP32_IR context
        assert ei.value.code == E_STATE
        sol.set_interface_refinement(3, 1e-14, 1e-10)
        sol.solve()
        again = sol.fine_flux()
    for x, y in zip(good[:3], again[:3]):
        assert np.array_equal(x, y)
