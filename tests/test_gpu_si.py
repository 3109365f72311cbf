"""Sequential implicit and sequential fully implicit runs on the GPU
(mrcm_step, mrcm_si_step, mrcm_sfi_step: Darcy and transport device-resident)
against the oracle's runs of the same steps (section 4; section 5.4 for SFI).

Both sides start from the same saturation and use the same time step
(20 dt_CFL of the initial field, dt_CFL = h / (max f' max |u|)); the
saturation of every step is compared in the max norm.  Differences are the
accumulated rounding-level differences of the Darcy solves (1e-10 parity)
and of the transport solves, so the bar is 1e-7 after 20 steps.
"""
import numpy as np
import pytest

import inputs
from oracle import transport as ot
from oracle.discretization import total_mobility
from oracle.mrcm import solve_mrcm
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def run_si_gpu(prob, s0, dt, n_steps):
    import torch
    from paper_2104_04653_amd import MRCMSolver
    nx, ny = prob.nx, prob.ny
    out, stats = [], []
    with MRCMSolver(prob) as sol:
        s = _dev(s0)
        ux = torch.empty((nx + 1) * ny, dtype=torch.float64, device="cuda")
        uy = torch.empty(nx * (ny + 1), dtype=torch.float64, device="cuda")
        p = torch.empty(nx * ny, dtype=torch.float64, device="cuda")
        sol.step(s, out=(p, ux, uy))                # u^0
        for _ in range(n_steps):
            s_new = torch.empty_like(s)
            stats.append(sol.si_step(s, s_new, p, ux, uy, dt))
            s = s_new
            out.append(s.cpu().numpy())
    return out, stats


def _dt(prob, s0, mult=20.0):
    r = solve_mrcm(prob, lam=total_mobility(s0, prob.mu_w, prob.mu_o))
    return mult * ot.cfl_time_step(prob, r.ux, r.uy)


@pytest.mark.parametrize("workload,kw,steps,tol", [
    ("channel256_q5", dict(nx=64, ny=64), 6, 1e-8),
    ("channel256_q5", {}, 20, 1e-7),          # the 256^2 workload: 20 steps at 20 CFL
])
def test_si_run_matches_oracle(workload, kw, steps, tol):
    prob = inputs.make_problem(workload, **kw)
    s0 = np.zeros(prob.nx * prob.ny)
    dt = _dt(prob, s0)
    say("case: SI run %s %dx%d, %d steps, dt %.3e" % (workload, prob.nx, prob.ny, steps, dt))
    gpu, stats = run_si_gpu(prob, s0, dt, steps)
    traj, iters = ot.si_run(prob, s0, steps, dt)
    worst = 0.0
    for k in range(steps):
        err = np.abs(gpu[k] - traj[k + 1]).max()
        worst = max(worst, err)
        say("  step %2d: Newton %d (oracle %d), max |ds| %.2e, water %.4f" % (
            k + 1, stats[k]["newton_iters"], iters[k], err, traj[k + 1].mean()))
    assert worst < tol


def test_si_two_steps_of_the_1024_workload():
    """The 1024^2 workload (inflow through W at p = 1, log-normal field):
    two SI steps at 20 CFL from the synthetic front, per-step error against
    the oracle."""
    prob = inputs.make_problem("gauss1024")
    s0 = inputs.synthetic_saturation(prob, 0)
    dt = _dt(prob, s0)
    say("case: SI run gauss1024, 2 steps, dt %.3e" % dt)
    gpu, stats = run_si_gpu(prob, s0, dt, 2)
    traj, iters = ot.si_run(prob, s0, 2, dt)
    for k in range(2):
        err = np.abs(gpu[k] - traj[k + 1]).max()
        say("  step %d: Newton %d (oracle %d), BiCGSTAB %d, max |ds| %.2e, %.1f ms transport" % (
            k + 1, stats[k]["newton_iters"], iters[k], stats[k]["linear_iters"], err, stats[k]["ms"]))
        assert err < 1e-8


def test_sfi_step_matches_oracle():
    import torch
    from paper_2104_04653_amd import MRCMSolver
    prob = inputs.make_problem("channel256_q5", nx=64, ny=64)
    s0 = np.zeros(prob.nx * prob.ny)
    dt = _dt(prob, s0)
    say("case: SFI step 64x64, dt %.3e" % dt)
    ref = ot.sfi_step(prob, s0, dt)
    nx, ny = prob.nx, prob.ny
    with MRCMSolver(prob) as sol:
        so = _dev(s0)
        sn = torch.empty_like(so)
        ux = torch.empty((nx + 1) * ny, dtype=torch.float64, device="cuda")
        uy = torch.empty(nx * (ny + 1), dtype=torch.float64, device="cuda")
        st = sol.sfi_step(so, sn, None, ux, uy, dt)
        s = sn.cpu().numpy()
    err = np.abs(s - ref.s).max()
    say("  outer %d (oracle %d), Newton %d, last change %.2e, max |ds| %.2e"
        % (st["outer_iters"], ref.outer, st["newton_iters"], st["last_change"], err))
    assert st["converged"] and st["outer_iters"] == ref.outer
    assert err < 1e-8
