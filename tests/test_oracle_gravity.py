"""Pins of the gravity variant of the oracle (CPU only): Darcy's law with
the term lambda_g g grad h (section 5.5, eqs. (Darcy_wg), (fluxos1_wg)),
gravity along y.

* Hydrostatic equilibrium: a closed box (or one whose top and bottom
  pressures are hydrostatic) with one mobility-weighted density rho
  everywhere and no source has u = 0 and p = rho gamma y + c, whatever the
  permeability.  The MRCM reproduces it with linear interface spaces (its
  traces are constant along horizontal and linear along vertical
  interfaces).
* A vertical column, layered in y with a different saturation (hence
  density) in every layer, Dirichlet data at the bottom and the top: the
  flux is uniform and follows from summing the half-cell laws
  t (p_start - p_end) + t rho gamma h/2 from the bottom face to the top
  face; the pressure follows cell by cell.  Written from that sum, not from
  the oracle.
* Full interface spaces recover the fine solution with gravity, and one
  subdomain is the fine solution.
* The stitched fluxes balance every cell.
"""
import numpy as np

from inputs import Problem, make_problem
from inputs.problems import DIRICHLET, NEUMANN
from oracle.discretization import gravity_density, total_mobility
from oracle.fine import solve_fine
from oracle.mrcm import flux_imbalance, solve_mrcm
from oracle.discretization import Geometry


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def hydro_problem(bc, gamma=-9.8, seed=3):
    base = make_problem("gauss64", nx=32, ny=32, sub=8, seed=seed)
    vals = (None, None, None, None)
    return base.replace(bc_kind=bc, bc_value=vals, source=None, gravity=gamma)


def test_density_of_the_phases():
    # lambda_g / lambda is rho_w for water only, rho_o for oil only, and the
    # mobility-weighted mean in between
    mu_w, mu_o, rw, ro = 1.0, 10.0, 1000.0, 800.0
    assert gravity_density(1.0, mu_w, mu_o, rw, ro) == rw
    assert gravity_density(0.0, mu_w, mu_o, rw, ro) == ro
    s = 0.5
    lw, lo = s * s / mu_w, (1 - s) ** 2 / mu_o
    assert np.isclose(gravity_density(s, mu_w, mu_o, rw, ro), (lw * rw + lo * ro) / (lw + lo), rtol=1e-15)


def check_hydrostatic(prob, rho0, gamma, y0_const=None):
    rho = np.full(prob.nx * prob.ny, rho0)
    yc = (np.arange(prob.ny) + 0.5) * prob.hy
    exact = np.repeat(rho0 * gamma * yc, prob.nx)
    for name, r in (("fine", solve_fine(prob, rho=rho)), ("mrcm", solve_mrcm(prob, rho=rho))):
        p = r["p"] if isinstance(r, dict) else r.p
        Fx = r["Fx"] if isinstance(r, dict) else r.Fx
        Fy = r["Fy"] if isinstance(r, dict) else r.Fy
        scale = abs(rho0 * gamma) * prob.perm.max() * prob.hx
        assert np.abs(Fx).max() < 1e-11 * scale, name
        assert np.abs(Fy).max() < 1e-11 * scale, name
        if y0_const is None:        # pure Neumann: p up to a constant
            d = (p - p.mean()) - (exact - exact.mean())
        else:
            d = p - exact
        assert np.abs(d).max() < 1e-11 * np.abs(exact).max(), name


def test_hydrostatic_closed_box():
    prob = hydro_problem((NEUMANN,) * 4)
    check_hydrostatic(prob, 850.0 / 1000.0, prob.gravity)


def test_hydrostatic_with_dirichlet_top_and_bottom():
    gamma, rho0 = -9.8, 0.9
    base = hydro_problem((NEUMANN, NEUMANN, DIRICHLET, DIRICHLET), gamma)
    top = np.full(base.nx, rho0 * gamma * base.ly)
    prob = base.replace(bc_value=(None, None, np.zeros(base.nx), top))
    check_hydrostatic(prob, rho0, gamma, y0_const=0.0)


def column_exact(k_rows, rho_rows, hx, hy, gamma, p_bot, p_top):
    """Uniform +y flux per column face and the cell pressures of a column
    layered in y (permeability and density per row)."""
    t = k_rows * hx / (0.5 * hy)                  # half-cell transmissibilities
    F = (p_bot - p_top + gamma * hy * rho_rows.sum()) / (2.0 * np.sum(1.0 / t))
    p = np.empty(k_rows.size)
    p[0] = p_bot - F / t[0] + rho_rows[0] * gamma * 0.5 * hy
    for j in range(k_rows.size - 1):
        p[j + 1] = p[j] - F * (1.0 / t[j] + 1.0 / t[j + 1]) + gamma * 0.5 * hy * (rho_rows[j] + rho_rows[j + 1])
    return F, p


def column_problem(nx=8, ny=48, sub_y=8, seed=5, gamma=-3.0):
    rng = np.random.default_rng(seed)
    k_rows = np.exp(rng.normal(0.0, 1.5, ny))
    s_rows = rng.uniform(0.0, 1.0, ny)
    perm = np.repeat(k_rows, nx)
    bot, top = np.full(nx, 2.0), np.full(nx, 0.5)
    prob = Problem(name="column", nx=nx, ny=ny, lx=nx / ny, ly=1.0, perm=perm, sub_nx=nx, sub_ny=sub_y,
                   bc_kind=(NEUMANN, NEUMANN, DIRICHLET, DIRICHLET), bc_value=(None, None, bot, top),
                   gravity=gamma, rho_w=1.0, rho_o=0.7)
    s = np.repeat(s_rows, nx)
    lam = total_mobility(s, prob.mu_w, prob.mu_o)
    rho = gravity_density(s, prob.mu_w, prob.mu_o, prob.rho_w, prob.rho_o)
    kappa_rows = k_rows * total_mobility(s_rows, prob.mu_w, prob.mu_o)
    rho_rows = gravity_density(s_rows, prob.mu_w, prob.mu_o, prob.rho_w, prob.rho_o)
    F, p = column_exact(kappa_rows, rho_rows, prob.hx, prob.hy, gamma, 2.0, 0.5)
    return prob, lam, rho, F, p


def test_layered_column_closed_form():
    prob, lam, rho, F, p_rows = column_problem()
    nx, ny = prob.nx, prob.ny
    exact_p = np.repeat(p_rows, nx)
    for name, r in (("fine", solve_fine(prob, lam=lam, rho=rho)),
                    ("mrcm", solve_mrcm(prob, lam=lam, rho=rho))):
        p = r["p"] if isinstance(r, dict) else r.p
        Fy = (r["Fy"] if isinstance(r, dict) else r.Fy).reshape(ny + 1, nx)
        Fx = r["Fx"] if isinstance(r, dict) else r.Fx
        assert np.abs(Fy - F).max() < 1e-11 * abs(F), name
        assert np.abs(Fx).max() < 1e-11 * abs(F), name
        assert rel(p, exact_p) < 1e-12, name


def test_column_flux_depends_on_gravity():
    # the closed form is not trivially gravity-free: gamma changes F by a
    # large fraction here
    prob, lam, rho, F, _ = column_problem()
    prob0, _, _, F0, _ = column_problem(gamma=0.0)
    assert abs(F - F0) > 0.1 * abs(F0)


def two_phase_gravity_problem(space, seed=4):
    base = make_problem("gauss64", nx=32, ny=32, sub=8, seed=seed, space=space)
    prob = base.replace(gravity=-5.0, rho_w=1.0, rho_o=0.75)
    rng = np.random.default_rng(seed)
    s = np.clip(rng.uniform(-0.2, 1.2, prob.nx * prob.ny), 0.0, 1.0)
    lam = total_mobility(s, prob.mu_w, prob.mu_o)
    rho = gravity_density(s, prob.mu_w, prob.mu_o, prob.rho_w, prob.rho_o)
    return prob, lam, rho


def test_full_spaces_recover_fine_with_gravity():
    prob, lam, rho = two_phase_gravity_problem("full")
    prob = prob.replace(p_dofs=prob.sub_nx, u_dofs=prob.sub_nx)
    ref = solve_fine(prob, lam=lam, rho=rho)
    r = solve_mrcm(prob, lam=lam, rho=rho)
    assert rel(r.p, ref["p"]) < 1e-10
    assert rel(np.r_[r.Fx, r.Fy], np.r_[ref["Fx"], ref["Fy"]]) < 1e-9
    # and the gravity matters for this case
    ref0 = solve_fine(prob, lam=lam)
    assert rel(ref0["p"], ref["p"]) > 1e-3


def test_one_subdomain_is_fine_with_gravity():
    prob, lam, rho = two_phase_gravity_problem("linear")
    prob = prob.replace(sub_nx=prob.nx, sub_ny=prob.ny)
    ref = solve_fine(prob, lam=lam, rho=rho)
    r = solve_mrcm(prob, lam=lam, rho=rho)
    assert rel(r.p, ref["p"]) < 1e-12
    assert rel(np.r_[r.Fx, r.Fy], np.r_[ref["Fx"], ref["Fy"]]) < 1e-11


def test_stitched_fluxes_balance_with_gravity():
    prob, lam, rho = two_phase_gravity_problem("linear")
    r = solve_mrcm(prob, lam=lam, rho=rho)
    geom = Geometry(prob)
    assert flux_imbalance(geom, prob, r.Fx, r.Fy) < 1e-12
    assert r.imbalance < 1e-12
