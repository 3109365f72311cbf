"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Every case runs the same seeded inputs through both and compares element by
element: local basis functions and interface blocks (steps a1-a5), the
interface solution (a6-a7), the composed pressure and the stitched fluxes
(a8-a9).  Floating-point tolerance: relative L2 1e-10 in pressure and flux
(FP64 path); local basis functions per column and interface blocks at 1e-10;
every cell of the stitched flux balances to 1e-12 of the largest face flux.
"""
import numpy as np
import pytest

import inputs
from oracle.discretization import total_mobility
from oracle.fine import solve_fine
from tests.gpu_util import (oracle_basis_padded, oracle_blocks_padded, rel, run_gpu, run_oracle,
                            say)
from tests.test_oracle_pins import box, linear_dirichlet

pytestmark = pytest.mark.gpu

TOL = 1e-10
IMB_TOL = 1e-12   # max over cells |net outflow - q |V|| / max |F|


def check_end_to_end(prob, s=None, lam=None, local=True, tol=TOL, label="", coef_tol=TOL):
    """Parity of one case.  The pressure and flux bar is `tol`; the interface
    coefficients are held to `coef_tol`, which cases with an ill-conditioned
    interface system (high contrast with non-polynomial spaces) relax: there
    rounding-level differences of the local blocks are amplified by the
    system's condition number while p and the fluxes stay at `tol`."""
    say("case:", label or prob.name, prob.nx, prob.ny, "sub", prob.sub_nx, "space", prob.space)
    if s is not None:
        lam = total_mobility(s, prob.mu_w, prob.mu_o)
    g = run_gpu(prob, lam=lam, extras=True if local else "coef")
    ref = run_oracle(prob, lam=lam)
    ep = rel(g["p"], ref.p)
    ef = rel(np.r_[g["ux"], g["uy"]], np.r_[ref.ux, ref.uy])
    ec = rel(g["coef"], ref.coeffs) if ref.coeffs.size else 0.0
    say("  rel L2: p %.2e  flux %.2e  interface coeffs %.2e  imbalance gpu %.2e oracle %.2e"
        "  iface res %.2e (%d refinement steps)" % (ep, ef, ec, g["imbalance"], ref.imbalance,
                                                   g["stats"]["interface_residual"],
                                                   g["stats"]["interface_ir_steps"]))
    if local:
        B = oracle_basis_padded(prob, ref)
        X = g["basis"]
        num = np.linalg.norm(X - B, axis=1)
        den = np.maximum(np.linalg.norm(B, axis=1), 1e-300)
        used = np.linalg.norm(B, axis=1) > 0
        eb = float((num[used] / den[used]).max())
        Bl = oracle_blocks_padded(prob, ref)
        scale = np.abs(Bl).max(axis=(1, 2), keepdims=True)
        ebl = float((np.abs(g["blocks"] - Bl) / scale).max())
        say("  basis max col rel %.2e  blocks %.2e" % (eb, ebl))
        assert eb < tol and ebl < tol
    assert ep < tol and ef < tol and ec < coef_tol
    # every cell of the stitched field balances (section 2, div u = q) to
    # 1e-12 of the largest face flux, on the GPU and in the oracle
    assert g["imbalance"] < IMB_TOL and ref.imbalance < IMB_TOL
    return g, ref


def test_gauss64_single_phase():
    check_end_to_end(inputs.make_problem("gauss64"))


def test_gauss64_two_phase_saturation():
    prob = inputs.make_problem("gauss64", seed=2)
    check_end_to_end(prob, s=inputs.synthetic_saturation(prob, 3, 10))


def test_sub8_rectangular_grid():
    prob = inputs.make_problem("gauss64", nx=64, ny=40, ly=0.5, sub=8, alpha=0.3, seed=3)
    check_end_to_end(prob)


def test_channel_quarter_five_spot_small():
    """All-Neumann boundary with wells: gauge path."""
    prob = inputs.make_problem("channel256_q5", nx=64, ny=64)
    check_end_to_end(prob, s=inputs.synthetic_saturation(prob, 5, 20))


def test_channel_quarter_five_spot_256():
    """The 256^2 channelized quarter-five-spot workload, one step."""
    prob = inputs.make_problem("channel256_q5")
    check_end_to_end(prob, s=inputs.synthetic_saturation(prob, 7, 20), local=False)


def test_linear_pressure_exact_on_gpu():
    """T-LIN through the GPU path."""
    prob, exact = linear_dirichlet(32, 16, 8, 0.5, 2.0, -1.5, alpha=0.4)
    say("case: linear pressure 32x16 sub 8")
    g = run_gpu(prob, extras=False)
    assert np.abs(g["p"] - exact).max() < 1e-12
    assert np.allclose(g["ux"], -3.0 * 2.0, rtol=1e-11)
    assert np.allclose(g["uy"], 3.0 * 1.5, rtol=1e-11)


def test_full_spaces_recover_fine_on_gpu():
    """T-FULL through the GPU path (4x4 subdomains, every fine-edge indicator)."""
    prob = inputs.make_problem("gauss64", nx=32, ny=32, sub=4, space="full", alpha=2.0)
    say("case: full spaces 32x32 sub 4")
    g = run_gpu(prob, extras=False)
    f = solve_fine(prob)
    assert rel(g["p"], f["p"]) < 1e-10
    assert rel(np.r_[g["ux"], g["uy"]], np.r_[f["ux"], f["uy"]]) < 1e-10


def test_one_subdomain_is_fine_on_gpu():
    """T-ONE through the GPU path: no skeleton, the local problem is the fine one."""
    prob = inputs.make_problem("gauss64", nx=16, ny=16, sub=16)
    say("case: one subdomain 16x16")
    g = run_gpu(prob, extras=False)
    f = solve_fine(prob)
    assert rel(g["p"], f["p"]) < 1e-12
    assert rel(np.r_[g["ux"], g["uy"]], np.r_[f["ux"], f["uy"]]) < 1e-11
    # no interface system: the local phase is timed by events, the interface
    # phase is empty, the flux phase by the kernels' clock stamps
    st = g["stats"]
    assert st["n_dof"] == 0
    assert 0.0 < st["ms_local"] < 1e3 and st["ms_interface"] == 0.0
    assert 0.0 < st["ms_flux"] < 1e3


def test_gauss1024_full_size_step():
    """The 1024^2 two-phase workload (4096 subdomains), one step, against the
    full oracle solve."""
    prob = inputs.make_problem("gauss1024")
    check_end_to_end(prob, s=inputs.synthetic_saturation(prob, 3), local=False)


@pytest.mark.parametrize("grid", [(10, 10), (16, 16), (24, 24), (32, 16)])
def test_interface_front_sizes(grid):
    """Subdomain grids whose tree levels take every register tile of the
    small-front elimination (largest front per level from 28 to 64
    unknowns, 64 on the 10 x 10 grid) and blocked levels of several shapes
    (fronts of 72 to 160 unknowns)."""
    sx, sy = grid
    prob = inputs.make_problem("gauss1024", nx=16 * sx, ny=16 * sy, lx=sx / 64, ly=sy / 64,
                               seed=sx + sy)
    check_end_to_end(prob, s=inputs.synthetic_saturation(prob, 2, 7), local=False,
                     label="front sizes %dx%d subdomains" % grid)


def test_bad_mobility_rejected():
    from paper_2104_04653_amd import MRCMSolver, MRCMError
    from paper_2104_04653_amd.mrcm import E_INVAL, E_STATE
    prob = inputs.make_problem("gauss64")
    say("case: error paths")
    with MRCMSolver(prob) as sol:
        with pytest.raises(MRCMError) as ei:
            sol.fine_flux()
        assert ei.value.code == E_STATE
        lam = np.ones(prob.nx * prob.ny)
        lam[100] = np.nan
        sol.update_mobility(lam, is_lambda=True)
        with pytest.raises(MRCMError) as ei:
            sol.solve()
        assert ei.value.code == E_INVAL
        lam[100] = -1.0
        sol.update_mobility(lam, is_lambda=True)
        with pytest.raises(MRCMError) as ei:
            sol.solve()
        assert ei.value.code == E_INVAL
        # a good mobility afterwards works again
        sol.update_mobility(np.ones(prob.nx * prob.ny), is_lambda=True)
        sol.solve()
        p, ux, uy, imb = sol.fine_flux()
        assert np.isfinite(p).all() and imb < 1e-10


def test_device_inputs_and_outputs():
    """Mobility from a device tensor, outputs into device tensors."""
    import torch
    from paper_2104_04653_amd import MRCMSolver
    prob = inputs.make_problem("gauss64", seed=4)
    s = inputs.synthetic_saturation(prob, 1, 4)
    say("case: device pointers")
    ref = run_gpu(prob, s=s, extras=False)
    with MRCMSolver(prob) as sol:
        sol.update_mobility(torch.from_numpy(s).cuda())
        sol.solve()
        p, ux, uy, imb = sol.fine_flux(device=True)
        torch.cuda.synchronize()
    assert np.array_equal(p.cpu().numpy(), ref["p"])
    assert np.array_equal(ux.cpu().numpy(), ref["ux"])
    assert np.array_equal(uy.cpu().numpy(), ref["uy"])


def test_repeat_solves_are_bitwise_identical():
    """Deterministic gathers, no atomics in the arithmetic: two solves of the
    same input give identical bits, and a different mobility in between does
    not leak into the next step."""
    from paper_2104_04653_amd import MRCMSolver
    prob = inputs.make_problem("channel256_q5", nx=64, ny=64)
    s1 = inputs.synthetic_saturation(prob, 2, 10)
    s2 = inputs.synthetic_saturation(prob, 6, 10)
    say("case: repeat solves")
    with MRCMSolver(prob) as sol:
        outs = []
        for s in (s1, s2, s1):
            sol.update_mobility(s)
            sol.solve()
            outs.append(sol.fine_flux())
    for a, b in zip(outs[0][:3], outs[2][:3]):
        assert np.array_equal(a, b)


def test_neumann_data_sources_and_alpha_per_interface():
    """Non-zero Neumann data on three sides (inflow through W, a varying
    outflow through S, none through N), Dirichlet on E, two wells, and a
    Robin parameter that differs per interface (eq. (beta)), on the 16 x 16
    register-tile kernels and on the 8 x 8 generic kernels."""
    from oracle.discretization import Geometry
    from inputs.problems import DIRICHLET, NEUMANN
    for sub in (16, 8):
        prob = inputs.make_problem("gauss64", seed=5, sub=sub)
        ny, nx = prob.ny, prob.nx
        yc = (np.arange(ny) + 0.5) / ny
        xc = (np.arange(nx) + 0.5) / nx
        src = np.zeros(nx * ny)
        src[5 * nx + 9] = 300.0
        src[40 * nx + 50] = -120.0
        prob = prob.replace(bc_kind=(NEUMANN, DIRICHLET, NEUMANN, NEUMANN),
                            bc_value=(-1.0 - 0.5 * np.sin(3 * yc), np.zeros(ny),
                                      0.3 * xc ** 2, None),
                            source=src)
        n_if = Geometry(prob).n_iface
        prob = prob.replace(alpha_per_interface=10.0 ** np.random.default_rng(sub).uniform(-1, 1, n_if))
        check_end_to_end(prob, s=inputs.synthetic_saturation(prob, 2, 6),
                         label="Neumann data, wells, alpha per interface, sub %d" % sub)


def test_layered_closed_form_on_gpu():
    """The 1-D closed form of the data terms (mass balance and series
    resistances; tests/test_oracle_pins_data.py) reproduced by the GPU path:
    one row of 16 x 16 (and 8 x 8) subdomains across a layered medium with
    prescribed inflow through W, a line source, and Dirichlet data on E."""
    from tests.test_oracle_pins_data import _kx, layered_column, x_layered
    for sub in (16, 8):
        nx, ny, lx = 8 * sub, sub, 2.0
        ly = lx * ny / nx
        k = _kx(nx, 4 + sub)
        west, east, qc, q = ("neumann", -2.0), ("dirichlet", 0.25), 3 * sub + 5, 40.0
        prob = x_layered(nx, ny, sub, k, lx, ly, west, east, qc, q, alpha=0.8)
        p_row, F_row = layered_column(k, lx / nx, ly / ny, west, east, qc, q)
        say("case: layered closed form, sub %d" % sub)
        g = run_gpu(prob, extras=False)
        P = g["p"].reshape(ny, nx)
        FX = (g["ux"] * prob.hy).reshape(ny, nx + 1)
        ep = np.abs(P - p_row[None, :]).max() / np.abs(p_row).max()
        ef = np.abs(FX - F_row[None, :]).max() / np.abs(F_row).max()
        say("  max rel error p %.2e flux %.2e imbalance %.2e" % (ep, ef, g["imbalance"]))
        assert ep < 1e-11 and ef < 1e-11
        assert np.abs(g["uy"]).max() * prob.hx < 1e-11 * np.abs(F_row).max()
        assert g["imbalance"] < IMB_TOL
