"""Physics-based interface spaces and the adaptive Robin parameter on the GPU
(MRCM_SPACE_PHYSICS, mrcm_set_adaptive_alpha; section 3.1) against the
oracle's spaces (4 + 4 dof slots per interface, the unused ones fixed to
zero), on the matrix-core kernels (two windows of 4 dofs per side) at
16 x 16 and 32 x 32 subdomains.

* the local solutions X, column by column, in the slots of each
  interface's functions (which also checks the library's construction of
  the functions and of the Robin data from them);
* p and the stitched fluxes at 1e-10, per-cell balance 1e-12, at 16x16 and
  32x32 subdomains, with and without the adaptive alpha;
* the barrier case on which these spaces are exact (the fine solution);
* the matrix-core kernels against the generic kernels on the same input
  (another elimination order: equal to rounding), blocks included.
"""
import numpy as np
import pytest

import inputs
from oracle.discretization import Geometry
from oracle.fine import solve_fine
from oracle.mrcm import solve_mrcm
from tests.gpu_util import rel, run_gpu, say
from tests.test_oracle_physics_spaces import barrier_problem

pytestmark = pytest.mark.gpu

SLOTS = 4


def physics_problem(workload, adaptive=None, **kw):
    base = inputs.make_problem(workload, **kw)
    return base.replace(space="physics", p_dofs=SLOTS, u_dofs=SLOTS, adaptive_alpha=adaptive)


def slot_columns(prob, ref):
    """For every subdomain: (oracle columns, library columns) of its local
    solutions, interface functions mapped to their slots."""
    g = Geometry(prob)
    out = []
    for sd in range(g.n_sub):
        oc, lc = [0], [0]
        col = 1
        for side in range(4):
            e = g.sub_iface[sd, side]
            if e < 0:
                continue
            n_p, n_u = int(ref.n_p[e]), int(ref.n_u[e])
            for k in range(n_p):
                oc.append(col + k)
                lc.append(1 + side * 2 * SLOTS + k)
            for k in range(n_u):
                oc.append(col + n_p + k)
                lc.append(1 + side * 2 * SLOTS + SLOTS + k)
            col += n_p + n_u
        out.append((np.array(oc), np.array(lc)))
    return out


def compare(prob, s, label):
    from oracle.discretization import total_mobility
    lam = total_mobility(s, prob.mu_w, prob.mu_o)
    ref = solve_mrcm(prob, lam=lam)
    got = run_gpu(prob, s=s)
    g = Geometry(prob)
    m = prob.sub_nx
    eX = 0.0
    for sd, (oc, lc) in enumerate(slot_columns(prob, ref)):
        I, J = sd % g.SX, sd // g.SX
        li, lj = np.meshgrid(np.arange(m), np.arange(m))
        cells = ((J * m + lj) * g.nx + I * m + li).reshape(-1)
        Xo = ref.X[cells][:, oc]
        Xg = got["basis"][sd][:, lc]
        eX = max(eX, np.abs(Xg - Xo).max() / max(np.abs(Xo).max(), 1e-300))
        # the unused slots hold nothing
        unused = np.setdiff1d(np.arange(got["basis"].shape[2]), lc)
        assert np.abs(got["basis"][sd][:, unused]).max(initial=0.0) == 0.0
    ep = rel(got["p"], ref.p)
    ef = rel(np.r_[got["ux"], got["uy"]], np.r_[ref.ux, ref.uy])
    sizes = (int(max(ref.n_p)), int(max(ref.n_u)))
    say("  %s: X %.2e, rel L2 p %.2e flux %.2e, imbalance %.2e; largest spaces %d + %d"
        % (label, eX, ep, ef, got["imbalance"], *sizes))
    assert eX < 1e-10 and ep < 1e-10 and ef < 1e-10
    assert got["imbalance"] < 1e-12
    assert max(sizes) > 2           # the physics functions are in use
    return got, ref


@pytest.mark.parametrize("adaptive", [None, (1e-2, 1e2)])
def test_physics_spaces_16x16(adaptive):
    prob = physics_problem("channel256_q5", adaptive=adaptive, nx=64, ny=64, seed=3)
    say("case: physics spaces 64x64 sub 16, adaptive alpha", adaptive)
    compare(prob, inputs.synthetic_saturation(prob, 4, 20), "q5 64")


def test_physics_spaces_32x32():
    prob = physics_problem("channel2048x1024", adaptive=(1e-2, 1e2), nx=256, ny=128, lx=0.25,
                           ly=0.125, seed=2)
    say("case: physics spaces 256x128 sub 32")
    compare(prob, inputs.synthetic_saturation(prob, 2, 5), "channel m32")


def test_physics_spaces_256_wells():
    prob = physics_problem("channel256_q5", adaptive=(1e-2, 1e2), seed=1)
    say("case: physics spaces 256x256 quarter-five-spot")
    compare(prob, inputs.synthetic_saturation(prob, 8, 20), "q5 256")


def test_adaptive_alpha_with_linear_spaces():
    """The adaptive alpha alone (linear spaces, the matrix-core kernels)."""
    base = inputs.make_problem("channel256_q5", nx=64, ny=64, seed=2)
    prob = base.replace(adaptive_alpha=(1e-2, 1e2))
    say("case: adaptive alpha, linear spaces")
    s = inputs.synthetic_saturation(prob, 4, 20)
    from oracle.discretization import total_mobility
    ref = solve_mrcm(prob, lam=total_mobility(s, prob.mu_w, prob.mu_o))
    got = run_gpu(prob, s=s, extras=False)
    ep = rel(got["p"], ref.p)
    ef = rel(np.r_[got["ux"], got["uy"]], np.r_[ref.ux, ref.uy])
    say("  rel L2 p %.2e flux %.2e imbalance %.2e" % (ep, ef, got["imbalance"]))
    assert ep < 1e-10 and ef < 1e-10 and got["imbalance"] < 1e-12


def test_barrier_case_is_exact_on_gpu():
    prob = barrier_problem("physics")
    say("case: physics spaces, barrier bands")
    ref = solve_fine(prob)
    got = run_gpu(prob, extras=False)
    ep = rel(got["p"], ref["p"])
    ef = rel(np.r_[got["ux"], got["uy"]], np.r_[ref["ux"], ref["uy"]])
    say("  against the fine solution: p %.2e flux %.2e" % (ep, ef))
    assert ep < 1e-11 and ef < 1e-10


def test_physics_spaces_errors():
    from paper_2104_04653_amd import MRCMError, MRCMSolver
    from paper_2104_04653_amd.mrcm import E_INVAL, E_UNSUPPORTED
    prob = physics_problem("channel256_q5", nx=64, ny=64)
    say("case: physics spaces, unsupported forms and bad alpha")
    for precision in ("fp32_ir", "surrogate"):
        with pytest.raises(MRCMError) as ei:
            MRCMSolver(prob, precision=precision)
        assert ei.value.code == E_UNSUPPORTED
    with pytest.raises(MRCMError) as ei:
        MRCMSolver(prob.replace(p_dofs=2, u_dofs=2))
    assert ei.value.code == E_INVAL
    with MRCMSolver(prob) as sol:
        with pytest.raises(MRCMError) as ei:
            sol.set_adaptive_alpha(0.0, 1.0)
        assert ei.value.code == E_INVAL


@pytest.mark.parametrize("m", [16, 32])
def test_physics_matrix_core_kernels_match_generic_kernels(m):
    """8 dofs per side on the matrix-core kernels (each window of 4 dofs per
    side solved by a work-group of its own, the blocks' columns written by
    their window) against the generic kernels (MRCM_GENERIC_KERNELS selects
    them) on the same input, with 16 x 16 and 32 x 32 subdomains."""
    import os
    if m == 16:
        prob = physics_problem("channel256_q5", adaptive=(1e-2, 1e2), nx=128, ny=96, lx=0.5, ly=0.375, seed=4)
    else:
        prob = physics_problem("channel2048x1024", adaptive=(1e-2, 1e2), nx=192, ny=128, lx=0.1875,
                               ly=0.125, seed=4)
    assert prob.sub_nx == m
    s = inputs.synthetic_saturation(prob, 5, 20)
    say("case: physics spaces, matrix-core vs generic kernels %dx%d sub %d" % (prob.nx, prob.ny, m))
    os.environ["MRCM_GENERIC_KERNELS"] = "1"
    try:
        gen = run_gpu(prob, s=s)
    finally:
        del os.environ["MRCM_GENERIC_KERNELS"]
    mc = run_gpu(prob, s=s)
    eb = np.abs(mc["basis"] - gen["basis"]).max() / np.abs(gen["basis"]).max()
    ebl = np.abs(mc["blocks"] - gen["blocks"]).max() / np.abs(gen["blocks"]).max()
    ep = rel(mc["p"], gen["p"])
    ef = rel(np.r_[mc["ux"], mc["uy"]], np.r_[gen["ux"], gen["uy"]])
    for name, r in (("generic", gen), ("matrix-core", mc)):
        st = r["stats"]
        say("  %s: ms local %.3f interface %.3f flux %.3f imbalance %.2e"
            % (name, st["ms_local"], st["ms_interface"], st["ms_flux"], r["imbalance"]))
    say("  max rel difference: basis %.2e blocks %.2e; rel L2 p %.2e flux %.2e" % (eb, ebl, ep, ef))
    # the unused slots hold exact zeros on both paths
    assert np.array_equal(mc["basis"] == 0.0, gen["basis"] == 0.0)
    assert np.array_equal(mc["blocks"] == 0.0, gen["blocks"] == 0.0)
    assert eb < 1e-11 and ebl < 1e-11 and ep < 1e-11 and ef < 1e-10
    assert mc["imbalance"] < 1e-12
