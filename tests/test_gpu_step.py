"""mrcm_step (mobility update, solve and fine-scale reconstruction in one
call with one synchronisation) against the three separate calls: the same
kernels on the same inputs, so the outputs are bitwise equal, also where the
interface solve is refined (the reconstruction is then redone; the
refinement is forced by a stopping tolerance below the FP64 floor)."""
import numpy as np
import pytest

import inputs
from oracle.discretization import total_mobility
from tests.gpu_util import rel, run_oracle, say

pytestmark = pytest.mark.gpu


def separate_calls(prob, s, precision="fp64", refine=False):
    from paper_2104_04653_amd import MRCMSolver
    with MRCMSolver(prob, precision=precision) as sol:
        if refine:
            sol.set_interface_refinement(2, 1e-17, 1e-10)
        sol.update_mobility(s)
        sol.solve()
        p, ux, uy, imb = sol.fine_flux()
        return p, ux, uy, imb, sol.stats()


def one_step(prob, s, precision="fp64", refine=False):
    from paper_2104_04653_amd import MRCMSolver
    with MRCMSolver(prob, precision=precision) as sol:
        if refine:
            sol.set_interface_refinement(2, 1e-17, 1e-10)
        p, ux, uy, imb = sol.step(s)
        return p, ux, uy, imb, sol.stats()


@pytest.mark.parametrize("workload,kw,step,refine", [
    ("gauss64", {"seed": 2}, (3, 10), False),
    ("channel256_q5", {}, (7, 20), True),   # with interface refinement
])
def test_step_equals_separate_calls(workload, kw, step, refine):
    prob = inputs.make_problem(workload, **kw)
    s = inputs.synthetic_saturation(prob, *step)
    say("case: step vs separate calls,", workload)
    a = separate_calls(prob, s, refine=refine)
    b = one_step(prob, s, refine=refine)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    assert a[3] == b[3]
    sa, sb = a[4], b[4]
    say("  interface refinement steps %d / %d, residual %.2e" % (
        sa["interface_ir_steps"], sb["interface_ir_steps"], sb["interface_residual"]))
    assert sa["interface_ir_steps"] == sb["interface_ir_steps"]
    assert sa["interface_residual"] == sb["interface_residual"]
    # phase times from the kernels' clock stamps: positive and plausible
    for st in (sa, sb):
        say("  phases ms: local %.3f interface %.3f flux %.3f" % (
            st["ms_local"], st["ms_interface"], st["ms_flux"]))
        for k in ("ms_local", "ms_interface", "ms_flux"):
            assert 0.0 < st[k] < 1e3
    if refine:
        assert sb["interface_ir_steps"] > 0
    # and against the oracle, as the separate calls are
    ref = run_oracle(prob, s=s)
    assert rel(b[0], ref.p) < 1e-10
    assert rel(np.r_[b[1], b[2]], np.r_[ref.ux, ref.uy]) < 1e-10


def test_step_device_arrays_and_repeated_steps():
    """Device saturation and device outputs written in place, three steps in
    a row on one context (the mobility changes every step), each equal to a
    fresh context's separate calls."""
    import torch
    from paper_2104_04653_amd import MRCMSolver
    prob = inputs.make_problem("gauss64", seed=4)
    say("case: step with device arrays, three steps")
    n = prob.nx * prob.ny
    out = (torch.empty(n, dtype=torch.float64, device="cuda"),
           torch.empty((prob.nx + 1) * prob.ny, dtype=torch.float64, device="cuda"),
           torch.empty(prob.nx * (prob.ny + 1), dtype=torch.float64, device="cuda"))
    with MRCMSolver(prob) as sol:
        for k in (2, 5, 9):
            s = inputs.synthetic_saturation(prob, k)
            p, ux, uy, imb = sol.step(torch.from_numpy(s).cuda(), out=out)
            torch.cuda.synchronize()
            ref = separate_calls(prob, s)
            assert np.array_equal(p.cpu().numpy(), ref[0])
            assert np.array_equal(ux.cpu().numpy(), ref[1])
            assert np.array_equal(uy.cpu().numpy(), ref[2])
            assert imb == ref[3]


def test_step_keeps_mobility_and_reports_errors():
    from paper_2104_04653_amd import MRCMSolver, MRCMError
    from paper_2104_04653_amd.mrcm import E_INVAL
    prob = inputs.make_problem("gauss64", seed=5)
    s = inputs.synthetic_saturation(prob, 4)
    say("case: step without new mobility; step with a bad mobility")
    with MRCMSolver(prob) as sol:
        sol.update_mobility(s)
        a = sol.step()            # values None: the mobility set before
        b = separate_calls(prob, s)
        assert np.array_equal(a[0], b[0])
        lam = total_mobility(s, prob.mu_w, prob.mu_o)
        lam[17] = -1.0
        with pytest.raises(MRCMError) as ei:
            sol.step(lam, is_lambda=True)
        assert ei.value.code == E_INVAL
        # the context stays usable
        c = sol.step(s)
        assert np.array_equal(c[0], b[0])
