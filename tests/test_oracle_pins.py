"""Pins of the CPU oracle against facts fixed by the paper and the mathematics.

None of these compares the oracle with itself: each checks a closed form, an
invariant, a special case that reduces to a simpler solver, or an
independent formulation of the same equations.  They run on the CPU only.
"""
import numpy as np
import pytest

from inputs import Problem, make_problem
from inputs.problems import DIRICHLET, NEUMANN
from oracle.discretization import (Geometry, edge_solution_space, fractional_flow, harmonic_mean,
                                   total_mobility)
from oracle.fine import solve_fine
from oracle.mrcm import solve_mrcm, solve_mrcm_monolithic


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def box(nx, ny, sub, perm, lx=1.0, ly=1.0, kind=(DIRICHLET, DIRICHLET, NEUMANN, NEUMANN),
        val=None, **kw):
    if val is None:
        val = (np.ones(ny), np.zeros(ny), None, None)
    return Problem(name="box", nx=nx, ny=ny, lx=lx, ly=ly, perm=np.asarray(perm, float),
                   sub_nx=sub, sub_ny=sub, bc_kind=kind, bc_value=val, **kw)


def linear_dirichlet(nx, ny, sub, a, b, c, kval=3.0, **kw):
    """Uniform kappa, p = a + b x + c y prescribed on every boundary face."""
    hx, hy = 1.0 / nx, 1.0 / ny
    xc = (np.arange(nx) + 0.5) * hx
    yc = (np.arange(ny) + 0.5) * hy
    val = (a + c * yc, a + b + c * yc, a + b * xc, a + b * xc + c)
    prob = box(nx, ny, sub, np.full(nx * ny, kval), kind=(DIRICHLET,) * 4, val=val, **kw)
    X, Y = np.meshgrid(xc, yc)
    return prob, (a + b * X + c * Y).reshape(-1)


# --------------------------------------------------------------------------
# the fine-grid solver (reference of several pins) against closed forms
# --------------------------------------------------------------------------

def test_fine_two_cells_closed_form():
    """Two cells in series between p=1 and p=0 (section 2 face laws):
    F = 1/(1/k1 + 1/k2), p1 = 1 - F/(2 k1), p2 = F/(2 k2) for h = 1."""
    k1, k2 = 3.0, 0.25
    prob = box(2, 1, 1, [k1, k2], lx=2.0, ly=1.0)
    r = solve_fine(prob)
    F = 1.0 / (1.0 / k1 + 1.0 / k2)
    assert np.allclose(r["p"], [1 - F / (2 * k1), F / (2 * k2)], rtol=1e-14, atol=1e-15)
    assert np.allclose(r["Fx"], [F, F, F], rtol=1e-14)


def test_fine_layered_closed_form():
    """kappa varying in x only, p=1/p=0 on W/E, no flow N/S: the flux through
    every column of faces is 1 / (sum of the series resistances)."""
    nx, ny = 12, 5
    rng = np.random.default_rng(0)
    kx = np.exp(rng.normal(size=nx) * 2)
    prob = box(nx, ny, 1, np.tile(kx, ny))
    r = solve_fine(prob)
    h = 1.0 / nx
    # resistance of a row of cells for a face of length 1/ny
    res = (h / (1.0 / ny)) * (1.0 / kx).sum()
    F = 1.0 / res
    assert np.allclose(r["Fx"].reshape(ny, nx + 1), F, rtol=1e-12)
    assert np.allclose(r["Fy"], 0.0, atol=1e-12 * F)


def test_fine_linear_exact():
    prob, exact = linear_dirichlet(10, 7, 1, 0.3, -1.2, 0.7)
    r = solve_fine(prob)
    assert np.abs(r["p"] - exact).max() < 1e-13
    assert np.allclose(r["ux"], 3.0 * 1.2, rtol=1e-12)
    assert np.allclose(r["uy"], -3.0 * 0.7, rtol=1e-12)


# --------------------------------------------------------------------------
# MRCM pins
# --------------------------------------------------------------------------

def test_tiny_mrcm_closed_form():
    """T-TINY: two cells, one cell per subdomain, constant spaces (= full
    spaces).  Reduces to the two-cell series formula for every alpha."""
    k1, k2 = 3.0, 0.25
    F = 1.0 / (1.0 / k1 + 1.0 / k2)
    for alpha in (1e-3, 1.0, 1e3):
        prob = box(2, 1, 1, [k1, k2], lx=2.0, ly=1.0, space="full", p_dofs=1, u_dofs=1,
                   alpha=alpha)
        r = solve_mrcm(prob)
        assert np.allclose(r.p, [1 - F / (2 * k1), F / (2 * k2)], rtol=1e-13)
        assert np.allclose(r.Fx, [F, F, F], rtol=1e-13)
        # interface unknowns: P_H is the face pressure, U_H the face velocity
        assert np.allclose(r.coeffs, [1 - F / k1, F], rtol=1e-12)


@pytest.mark.parametrize("alpha", [1e-2, 1.0, 1e2])
def test_linear_pressure_reproduced(alpha):
    """T-LIN: uniform kappa and linear Dirichlet data; linear interface
    spaces contain the exact traces, so the MRCM is exact at every cell."""
    prob, exact = linear_dirichlet(16, 12, 4, 0.5, 2.0, -1.5, alpha=alpha)
    r = solve_mrcm(prob)
    assert np.abs(r.p - exact).max() < 1e-13
    assert np.allclose(r.ux, -3.0 * 2.0, rtol=1e-12)
    assert np.allclose(r.uy, 3.0 * 1.5, rtol=1e-12)
    assert np.allclose(r.Fx_raw / prob.hy, -3.0 * 2.0, rtol=1e-12)


def test_one_subdomain_is_fine():
    """T-ONE: a single subdomain has no skeleton; the local problem is the
    fine problem."""
    prob = make_problem("gauss64", nx=32, ny=32, sub=32)
    r = solve_mrcm(prob)
    f = solve_fine(prob)
    assert rel(r.p, f["p"]) < 1e-13
    assert rel(np.r_[r.Fx, r.Fy], np.r_[f["Fx"], f["Fy"]]) < 1e-12


@pytest.mark.parametrize("alpha", [1e-3, 1.0, 1e3])
def test_full_spaces_recover_fine(alpha):
    """T-FULL: with every fine-edge indicator in both interface spaces the
    two continuity conditions hold face by face; eliminating the face
    pressure gives the harmonic transmissibility, i.e. the fine solution."""
    prob = make_problem("gauss64", nx=32, ny=32, sub=8, space="full", alpha=alpha)
    r = solve_mrcm(prob)
    f = solve_fine(prob)
    assert rel(r.p, f["p"]) < 1e-11
    assert rel(np.r_[r.Fx, r.Fy], np.r_[f["Fx"], f["Fy"]]) < 1e-10
    assert rel(np.r_[r.Fx_raw, r.Fy_raw], np.r_[f["Fx"], f["Fy"]]) < 1e-10


def test_full_spaces_pure_neumann():
    """T-FULL on the source-driven, all-Neumann case (gauge handling)."""
    prob = make_problem("channel256_q5", nx=32, ny=32, sub=8, space="full")
    r = solve_mrcm(prob)
    f = solve_fine(prob)
    assert abs(r.p.mean()) < 1e-12
    assert rel(r.p, f["p"]) < 1e-10
    assert rel(np.r_[r.Fx, r.Fy], np.r_[f["Fx"], f["Fy"]]) < 1e-10


def _shifted_basis(itf):
    xi = itf.xi
    return np.stack([np.ones_like(xi), xi - 0.5]), np.stack([np.ones_like(xi), xi - 0.5])


def test_basis_independence():
    """T-BASIS: nodal {1-x, x} and modal {1, x - 1/2} span the same space."""
    prob = make_problem("gauss64", nx=32, ny=32, sub=8)
    r1 = solve_mrcm(prob)
    p2 = prob.replace(space="custom")
    p2.custom_space = _shifted_basis
    r2 = solve_mrcm(p2)
    assert rel(r2.p, r1.p) < 1e-12
    assert rel(np.r_[r2.Fx, r2.Fy], np.r_[r1.Fx, r1.Fy]) < 1e-11


def test_condensed_equals_monolithic():
    """T-MONO: the basis-function (static condensation) route equals one
    sparse solve of all local and interface equations together."""
    for prob in (make_problem("gauss64", nx=48, ny=32, sub=8, alpha=0.3),
                 make_problem("channel256_q5", nx=32, ny=32, sub=8)):
        r = solve_mrcm(prob)
        pm, cm = solve_mrcm_monolithic(prob)
        assert rel(pm, r.p) < 1e-11
        assert rel(cm, r.coeffs) < 1e-10


def test_conservation():
    """T-CONS: local solutions balance every cell; flux continuity tested
    with the constant (psi_0 + psi_1 = 1) makes every interface's two side
    fluxes cancel in total; the stitched flux balances every cell."""
    prob = make_problem("gauss64")
    r = solve_mrcm(prob)
    for lo, hi in r.side_flux:
        scale = np.abs(np.r_[lo, hi]).max()
        assert abs((lo + hi).sum()) < 1e-11 * scale
    assert r.imbalance < 1e-12
    assert r.imbalance_raw > 1e-6          # raw one-sided fluxes do not balance
    # the Neumann data of the floating subdomains are compatible to rounding
    # (what the stitch removes evenly is not a modelling error)
    assert 0.0 < r.stitch_defect < 1e-12
    q5 = solve_mrcm(make_problem("channel256_q5", nx=64, ny=64))
    assert q5.imbalance < 1e-12 and q5.stitch_defect < 1e-11
    # local problems: the right-hand sides are reproduced (residual check)
    from oracle.discretization import Geometry
    g = Geometry(prob)
    assert g.n_sub == 16


def test_interface_matrix_symmetric_quasidefinite():
    """T-SYM: negating the pressure-continuity rows makes the interface
    matrix symmetric, with a negative (semi)definite pressure block and a
    positive definite flux block."""
    for alpha in (1e-2, 1.0, 1e2):
        prob = make_problem("gauss64", nx=32, ny=32, sub=8, alpha=alpha)
        r = solve_mrcm(prob)
        M = r.interface_matrix.toarray()
        isP = np.zeros(M.shape[0], bool)
        for e in range(len(r.n_p)):
            isP[r.dof_offset[e]:r.dof_offset[e] + r.n_p[e]] = True
        Ms = np.where(isP, 1.0, -1.0)[:, None] * M
        assert np.abs(Ms - Ms.T).max() < 1e-12 * np.abs(Ms).max()
        Ms = 0.5 * (Ms + Ms.T)
        ePP = np.linalg.eigvalsh(Ms[np.ix_(isP, isP)])
        eUU = np.linalg.eigvalsh(Ms[np.ix_(~isP, ~isP)])
        assert ePP.max() < 1e-10 * np.abs(ePP).max()
        assert eUU.min() > 0


def test_alpha_limits():
    """T-LIMIT (section 3, limits of alpha): alpha -> 0 imposes the interface
    pressure, alpha -> infinity the interface flux."""
    for alpha, check in ((1e-9, "pressure"), (1e9, "flux")):
        prob = make_problem("gauss64", nx=32, ny=32, sub=8, alpha=alpha)
        r = solve_mrcm(prob)
        g = Geometry(prob)
        off = r.dof_offset
        worst = 0.0
        for itf in g.interfaces:
            ce = r.coeffs[off[itf.index]:off[itf.index + 1]]
            PH = (1 - itf.xi) * ce[0] + itf.xi * ce[1]
            UH = (1 - itf.xi) * ce[2] + itf.xi * ce[3]
            Flo, Fhi = r.side_flux[itf.index]
            kap = prob.perm
            for F, cells, sigma in ((Flo, itf.lo_cells, 1.0), (Fhi, itf.hi_cells, -1.0)):
                beta = alpha * itf.H / kap[cells]
                if check == "pressure":
                    pf = PH - beta * sigma * UH + beta * F / itf.flen
                    worst = max(worst, np.abs(pf - PH).max() / np.abs(r.p).max())
                else:
                    worst = max(worst, np.abs(F - itf.flen * sigma * UH).max()
                                / np.abs(r.Fx).max())
        assert worst < 1e-6, (check, worst)


def test_solver_floor():
    """T-FLOOR: the oracle with LAPACK banded Cholesky local solves and a
    dense LU interface solve against SuperLU for both.  Both refine with
    extended-precision residuals, so they agree far below the 1e-10 parity
    bar; without that refinement they differ by about the bar itself on
    high-contrast fields."""
    prob = make_problem("gauss64")
    a = solve_mrcm(prob)
    b = solve_mrcm(prob, local_solver="banded_refined", interface_solver="dense")
    assert rel(b.p, a.p) < 1e-14
    assert rel(np.r_[b.Fx, b.Fy], np.r_[a.Fx, a.Fy]) < 1e-13
    c = solve_mrcm(prob, local_solver="banded", interface_solver="dense")
    assert rel(c.p, a.p) < 1e-12


def test_edge_solution_space_reduces_to_linear():
    """Uniform permeability: the edge-solution functions are the linear ones."""
    m = 16
    ps, us = edge_solution_space(np.full(m, 2.0), np.full(m, 2.0))
    xi = (np.arange(m) + 0.5) / m
    assert np.allclose(ps[0], 1 - xi, atol=1e-14)
    assert np.allclose(ps[1], xi, atol=1e-14)
    assert np.allclose(us[0], 1.0, atol=1e-14)
    assert np.allclose(us[1], 0.5 - xi, atol=1e-14)
    rng = np.random.default_rng(3)
    ps, us = edge_solution_space(np.exp(rng.normal(size=m) * 3), np.exp(rng.normal(size=m) * 3))
    assert np.all(np.diff(ps[0]) < 0) and ps[0].max() < 1 and ps[0].min() > 0


def _edge_system(k_lo, k_hi):
    """The 1-D two-point system of the edge problem, assembled."""
    t = harmonic_mean(k_lo, k_hi)
    m = t.size
    A = np.zeros((m, m))
    rhs = np.zeros(m)
    for j in range(m):
        if j == 0:
            A[j, j] += 2 * t[0]
            rhs[j] = 2 * t[0]
        else:
            c = harmonic_mean(t[j - 1], t[j])
            A[j, j] += c
            A[j, j - 1] -= c
        if j == m - 1:
            A[j, j] += 2 * t[-1]
        else:
            c = harmonic_mean(t[j], t[j + 1])
            A[j, j] += c
            A[j, j + 1] -= c
    return A, rhs


def test_edge_solution_solves_the_edge_problem():
    """psi is the solution of the assembled 1-D two-point problem."""
    rng = np.random.default_rng(7)
    for m in (4, 16, 32):
        k_lo, k_hi = np.exp(rng.normal(size=m) * 2), np.exp(rng.normal(size=m) * 2)
        A, rhs = _edge_system(k_lo, k_hi)
        ps, _ = edge_solution_space(k_lo, k_hi)
        assert np.allclose(ps[0], np.linalg.solve(A, rhs), rtol=1e-13, atol=0)
        assert np.allclose(A @ ps[0], rhs, rtol=0, atol=1e-12 * np.abs(A).max())


def test_edge_solution_relative_accuracy_at_high_contrast():
    """Exact rational elimination of the assembled edge system at contrast
    1e8: psi and 1 - psi hold full relative accuracy in every entry."""
    from fractions import Fraction
    k_lo = np.array([1e8, 2e8, 1.0, 3.0, 0.5, 2.0, 1e8, 3e8])
    k_hi = np.array([3e8, 1e8, 2.0, 1.0, 0.7, 1e8, 1e8, 1e8])
    m = k_lo.size
    F = [Fraction(x) for x in k_lo], [Fraction(x) for x in k_hi]
    h = lambda a, b: 2 * a * b / (a + b)
    t = [h(F[0][j], F[1][j]) for j in range(m)]
    A = [[Fraction(0)] * m for _ in range(m)]
    rhs = [Fraction(0)] * m
    for j in range(m):
        if j == 0:
            A[0][0] += 2 * t[0]
            rhs[0] = 2 * t[0]
        else:
            c = h(t[j - 1], t[j])
            A[j][j] += c
            A[j][j - 1] -= c
        if j == m - 1:
            A[j][j] += 2 * t[-1]
        else:
            c = h(t[j], t[j + 1])
            A[j][j] += c
            A[j][j + 1] -= c
    for j in range(1, m):          # exact elimination
        f = A[j][j - 1] / A[j - 1][j - 1]
        A[j][j] -= f * A[j - 1][j]
        A[j][j - 1] = Fraction(0)
        rhs[j] -= f * rhs[j - 1]
    x = [Fraction(0)] * m
    x[-1] = rhs[-1] / A[-1][-1]
    for j in range(m - 2, -1, -1):
        x[j] = (rhs[j] - A[j][j + 1] * x[j + 1]) / A[j][j]
    ps, _ = edge_solution_space(k_lo, k_hi)
    exact = np.array([float(v) for v in x])
    exact_c = np.array([float(1 - v) for v in x])
    assert exact_c.min() < 1e-7 and exact.min() < 1e-7   # both functions get small
    assert np.allclose(ps[0], exact, rtol=1e-14, atol=0)
    assert np.allclose(ps[1], exact_c, rtol=1e-14, atol=0)


def test_edge_space_homogeneous_equals_linear_mrcm():
    prob = make_problem("gauss64", nx=32, ny=32, sub=8)
    hom = prob.replace(perm=np.full(prob.perm.size, 2.0))
    a = solve_mrcm(hom)
    b = solve_mrcm(hom.replace(space="edge"))
    assert rel(b.p, a.p) < 1e-12


def test_mobility_closed_forms():
    """eq. (fluxos1) with k_rw = s^2, k_ro = (1-s)^2: lambda(0) = 1/mu_o,
    lambda(1) = 1/mu_w, minimum 1/(mu_w+mu_o) at s = mu_w/(mu_w+mu_o);
    f(s) = M s^2 / (M s^2 + (1-s)^2)."""
    mw, mo = 1.0, 10.0
    assert total_mobility(0.0, mw, mo) == pytest.approx(0.1)
    assert total_mobility(1.0, mw, mo) == pytest.approx(1.0)
    s = np.linspace(0, 1, 100001)
    lam = total_mobility(s, mw, mo)
    assert s[lam.argmin()] == pytest.approx(1 / 11, abs=1e-4)
    assert lam.min() == pytest.approx(1 / 11, rel=1e-8)
    M = mo / mw
    assert np.allclose(fractional_flow(s, mw, mo), M * s**2 / (M * s**2 + (1 - s) ** 2))
