"""Pins of the oracle's data terms: the source q, non-zero Neumann data u_b
and a Robin parameter that differs per interface (CPU only).

The source and boundary terms of eq. (Darcy) and the local problems of
eq. (mrc1) are fixed here by closed forms that do not use the oracle's own
conventions: on a medium layered across one axis, with boundary data and a
line source that are uniform along the other axis, the solution is one-
dimensional.  Its face flux is fixed by mass balance alone (inflow plus
injection) and its pressure by series resistances, so a flipped sign or a
wrong scale of q or u_b changes both.  With one row of subdomains across the
layers, the skeleton traces of such a solution are constant along every
interface, which the linear interface spaces contain: the MRCM then
reproduces the closed form exactly.  With full interface spaces it does so
for any decomposition (the fine solution is recovered).

The per-interface Robin parameter (eq. (beta)) is pinned by the limits of
section 3 taken on chosen interfaces: alpha -> 0 imposes the interface
pressure and alpha -> infinity the interface flux, each only where it was
asked for.
"""
import numpy as np
import pytest

from inputs import Problem, make_problem
from inputs.problems import DIRICHLET, NEUMANN
from oracle.discretization import Geometry
from oracle.fine import solve_fine
from oracle.mrcm import solve_mrcm


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def layered_column(k, h_along, h_across, west, east, q_col=None, q=0.0):
    """Exact cell pressures and +x face fluxes of one row of a layered medium.

    k: permeability of the n cells of the row; h_along / h_across: cell size
    along / across the row; west, east: ("dirichlet", p_b) or ("neumann",
    u_b) with u_b the OUTWARD normal velocity; a line source of q per unit
    area in cell q_col (Q = q h_along h_across enters that cell).

    Written from mass balance and series resistances, not from the oracle:
    the resistance between two neighbouring cell centres is the sum of the
    two half-cell resistances (h/2)/(k |f|), |f| = h_across.
    """
    n = k.size
    f = h_across
    half = 0.5 * h_along / (k * f)                 # half-cell resistances
    # resistance of the n+1 segments W face -> cell 0 -> ... -> cell n-1 -> E face;
    # segment s carries the +x flux F_s of face s
    seg = np.concatenate([[half[0]], half[:-1] + half[1:], [half[-1]]])
    inj = np.zeros(n)
    if q_col is not None:
        inj[q_col] = q * h_along * h_across
    cum = np.concatenate([[0.0], np.cumsum(inj)])   # injected left of face s
    if west[0] == "neumann" and east[0] == "neumann":
        raise ValueError("pure Neumann row is not closed-form here")
    if west[0] == "neumann":
        F = -west[1] * f + cum                     # outward u_b on W points to -x
    elif east[0] == "neumann":
        F = east[1] * f - (cum[-1] - cum)          # outward u_b on E points to +x
    else:
        # p_W - p_E is the sum of the segment drops F_s seg_s
        F = (west[1] - east[1] - (cum * seg).sum()) / seg.sum() + cum
    if west[0] == "dirichlet":
        p = west[1] - np.cumsum(F[:-1] * seg[:-1])
    else:
        p = east[1] + np.cumsum((F * seg)[::-1])[::-1][1:]
    return p, F


def x_layered(nx, ny, sub, kx, lx, ly, west, east, q_col=None, q=0.0, **kw):
    kinds = {"dirichlet": DIRICHLET, "neumann": NEUMANN}
    kind = (kinds[west[0]], kinds[east[0]], NEUMANN, NEUMANN)
    val = (np.full(ny, west[1]), np.full(ny, east[1]), None, None)
    src = None
    if q_col is not None:
        src = np.zeros(nx * ny)
        src.reshape(ny, nx)[:, q_col] = q
    return Problem(name="x-layered", nx=nx, ny=ny, lx=lx, ly=ly,
                   perm=np.tile(np.asarray(kx, float), ny), sub_nx=sub, sub_ny=sub,
                   bc_kind=kind, bc_value=val, source=src, **kw)


def y_layered(nx, ny, sub, ky, lx, ly, south, north, q_row=None, q=0.0, **kw):
    kinds = {"dirichlet": DIRICHLET, "neumann": NEUMANN}
    kind = (NEUMANN, NEUMANN, kinds[south[0]], kinds[north[0]])
    val = (None, None, np.full(nx, south[1]), np.full(nx, north[1]))
    src = None
    if q_row is not None:
        src = np.zeros(nx * ny)
        src.reshape(ny, nx)[q_row, :] = q
    return Problem(name="y-layered", nx=nx, ny=ny, lx=lx, ly=ly,
                   perm=np.repeat(np.asarray(ky, float), nx), sub_nx=sub, sub_ny=sub,
                   bc_kind=kind, bc_value=val, source=src, **kw)


def _kx(n, seed):
    return np.exp(np.random.default_rng(seed).normal(size=n) * 1.5)


CASES = [
    # (west, east, source column, q)
    (("dirichlet", 0.0), ("dirichlet", 0.0), 13, 40.0),     # point of injection, both ends open
    (("dirichlet", 1.0), ("dirichlet", -0.5), 21, -25.0),   # production with a pressure drop
    (("neumann", -2.0), ("dirichlet", 0.3), None, 0.0),     # prescribed inflow, no source
    (("neumann", -2.0), ("dirichlet", 0.0), 5, 30.0),       # inflow and injection
    (("neumann", 1.5), ("dirichlet", 0.0), 18, 60.0),       # outflow through W, injection inside
    (("dirichlet", 0.0), ("neumann", 0.7), 9, 20.0),        # prescribed outflow on E
]


def _check(r_p, r_Fx, r_Fy, p_row, F_row, nrows, ncols, scale_p, scale_F):
    P = np.asarray(r_p).reshape(nrows, ncols)
    FX = np.asarray(r_Fx).reshape(nrows, ncols + 1)
    assert np.abs(P - p_row[None, :]).max() < 1e-11 * scale_p
    assert np.abs(FX - F_row[None, :]).max() < 1e-11 * scale_F
    assert np.abs(r_Fy).max() < 1e-11 * scale_F


@pytest.mark.parametrize("case", range(len(CASES)))
def test_fine_layered_data_closed_form(case):
    """The fine solver reproduces the 1-D closed form of the data terms."""
    west, east, qc, q = CASES[case]
    nx, ny, lx, ly = 32, 8, 2.0, 0.5
    k = _kx(nx, case)
    prob = x_layered(nx, ny, 8, k, lx, ly, west, east, qc, q)
    p_row, F_row = layered_column(k, lx / nx, ly / ny, west, east, qc, q)
    r = solve_fine(prob)
    _check(r["p"], r["Fx"], r["Fy"], p_row, F_row, ny, nx, np.abs(p_row).max(), np.abs(F_row).max())


@pytest.mark.parametrize("space", ["linear", "full"])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_mrcm_layered_data_closed_form(case, space):
    """The MRCM reproduces the 1-D closed form: the pressure, the stitched
    flux and the raw one-sided fluxes.  Linear spaces: four subdomains along
    the flow, one across it (a horizontal interface would carry the
    pressure profile along the layers, which is not linear); full spaces:
    four by two subdomains."""
    west, east, qc, q = CASES[case]
    nx, lx, sub = 32, 2.0, 8
    ny = sub if space == "linear" else 2 * sub
    ly = 0.5 * ny / sub
    k = _kx(nx, case)
    dofs = dict(p_dofs=sub, u_dofs=sub) if space == "full" else {}
    prob = x_layered(nx, ny, sub, k, lx, ly, west, east, qc, q, space=space, alpha=0.6, **dofs)
    p_row, F_row = layered_column(k, lx / nx, ly / ny, west, east, qc, q)
    r = solve_mrcm(prob)
    sp, sF = np.abs(p_row).max(), np.abs(F_row).max()
    _check(r.p, r.Fx, r.Fy, p_row, F_row, ny, nx, sp, sF)
    _check(r.p, r.Fx_raw, r.Fy_raw, p_row, F_row, ny, nx, sp, sF)


@pytest.mark.parametrize("case", [0, 3, 5])
def test_mrcm_layered_data_closed_form_along_y(case):
    """The same closed form with the roles of x and y exchanged: the data of
    the S and N sides and a line source along a row."""
    south, north, qr, q = CASES[case]
    nx, ny, lx, ly, sub = 8, 32, 0.5, 2.0, 8
    k = _kx(ny, 10 + case)
    prob = y_layered(nx, ny, sub, k, lx, ly, south, north, qr, q, alpha=1.7)
    p_col, F_col = layered_column(k, ly / ny, lx / nx, south, north, qr, q)
    r = solve_mrcm(prob)
    P = r.p.reshape(ny, nx)
    FY = r.Fy.reshape(ny + 1, nx)
    sp, sF = np.abs(p_col).max(), np.abs(F_col).max()
    assert np.abs(P - p_col[:, None]).max() < 1e-11 * sp
    assert np.abs(FY - F_col[:, None]).max() < 1e-11 * sF
    assert np.abs(r.Fx).max() < 1e-11 * sF


def test_closed_form_helper_balances():
    """The helper itself: every cell's net outflow is its injection, and the
    boundary fluxes carry the prescribed data (a check of the closed form,
    independent of any solver)."""
    k = _kx(24, 3)
    for west, east, qc, q in CASES:
        p, F = layered_column(k, 0.1, 0.25, west, east, qc, q)
        inj = np.zeros(24)
        if qc is not None:
            inj[qc] = q * 0.1 * 0.25
        assert np.allclose(F[1:] - F[:-1], inj, atol=1e-12 * np.abs(F).max())
        for side, val, face, sgn in ((west, None, 0, -1.0), (east, None, 24, 1.0)):
            if side[0] == "neumann":
                assert F[face] * sgn == pytest.approx(side[1] * 0.25, rel=1e-14)
            else:   # Dirichlet: the half-cell law to the boundary pressure
                c = 0 if face == 0 else 23
                assert F[face] * sgn == pytest.approx((p[c] - side[1]) / (0.5 * 0.1 / (k[c] * 0.25)),
                                                      rel=1e-12)
        # Darcy on every interior face: F = (p_c - p_d) / (two half resistances)
        half = 0.5 * 0.1 / (k * 0.25)
        assert np.allclose(F[1:-1], (p[:-1] - p[1:]) / (half[:-1] + half[1:]), rtol=1e-12)


def test_quarter_five_spot_source_sign():
    """Injection raises pressure: with uniform permeability and the wells of
    the quarter-five-spot, the injector cell holds the highest pressure, the
    producer the lowest, the field is antisymmetric under the point
    reflection of the square, and the stitched flux leaves the injector at
    the injected rate Q (read directly from the face fluxes)."""
    prob = make_problem("channel256_q5", nx=32, ny=32, sub=8)
    prob = prob.replace(perm=np.full(32 * 32, 3.0))
    for r_p, Fx, Fy in ((lambda r: (r.p, r.Fx, r.Fy))(solve_mrcm(prob)),
                        (lambda f: (f["p"], f["Fx"], f["Fy"]))(solve_fine(prob))):
        P = r_p.reshape(32, 32)
        assert P[0, 0] == P.max() and P[0, 0] > 0
        assert P[-1, -1] == P.min() and P[-1, -1] < 0
        assert np.abs(P + P[::-1, ::-1]).max() < 1e-11 * P.max()
        FX = Fx.reshape(32, 33)
        FY = Fy.reshape(33, 32)
        out_inj = FX[0, 1] - FX[0, 0] + FY[1, 0] - FY[0, 0]
        Q = prob.lx * prob.ly           # one pore volume per unit time
        assert out_inj == pytest.approx(Q, rel=1e-11)
        out_prod = FX[-1, -1] - FX[-1, -2] + FY[-1, -1] - FY[-2, -1]
        assert out_prod == pytest.approx(-Q, rel=1e-11)


# --------------------------------------------------------------------------
# Robin parameter per interface (eq. (beta))
# --------------------------------------------------------------------------

def _n_iface(prob):
    return Geometry(prob).n_iface


def test_uniform_per_interface_alpha_equals_scalar():
    prob = make_problem("gauss64", nx=32, ny=32, sub=8, alpha=0.37)
    a = solve_mrcm(prob)
    b = solve_mrcm(prob.replace(alpha=5.0, alpha_per_interface=np.full(_n_iface(prob), 0.37)))
    assert np.array_equal(a.p, b.p) and np.array_equal(a.Fx, b.Fx) and np.array_equal(a.Fy, b.Fy)


def test_varying_alpha_full_spaces_recover_fine():
    """T-FULL holds for any positive alpha on every interface."""
    prob = make_problem("gauss64", nx=32, ny=32, sub=8, space="full")
    alpha = 10.0 ** np.random.default_rng(5).uniform(-3, 3, _n_iface(prob))
    r = solve_mrcm(prob.replace(alpha_per_interface=alpha))
    f = solve_fine(prob)
    assert rel(r.p, f["p"]) < 1e-11
    assert rel(np.r_[r.Fx, r.Fy], np.r_[f["Fx"], f["Fy"]]) < 1e-10


def test_varying_alpha_linear_exact():
    """T-LIN holds for any positive alpha on every interface."""
    from tests.test_oracle_pins import linear_dirichlet
    prob, exact = linear_dirichlet(16, 12, 4, 0.5, 2.0, -1.5)
    alpha = 10.0 ** np.random.default_rng(6).uniform(-2, 2, _n_iface(prob))
    r = solve_mrcm(prob.replace(alpha_per_interface=alpha))
    assert np.abs(r.p - exact).max() < 1e-13


def test_mixed_alpha_limits_per_interface():
    """alpha = 1e-9 on the even interfaces imposes the interface pressure
    there; alpha = 1e9 on the odd ones imposes the interface flux there.
    Each limit is checked only on the interfaces that carry it, so an alpha
    read from the wrong interface fails."""
    prob = make_problem("gauss64", nx=32, ny=32, sub=8)
    g = Geometry(prob)
    alpha = np.where(np.arange(g.n_iface) % 2 == 0, 1e-9, 1e9)
    r = solve_mrcm(prob.replace(alpha_per_interface=alpha))
    off = r.dof_offset
    worst_p = worst_f = 0.0
    miss_p = miss_f = np.inf
    for itf in g.interfaces:
        ce = r.coeffs[off[itf.index]:off[itf.index + 1]]
        PH = (1 - itf.xi) * ce[0] + itf.xi * ce[1]
        UH = (1 - itf.xi) * ce[2] + itf.xi * ce[3]
        a = alpha[itf.index]
        for F, cells, sigma in ((r.side_flux[itf.index][0], itf.lo_cells, 1.0),
                                (r.side_flux[itf.index][1], itf.hi_cells, -1.0)):
            beta = a * itf.H / prob.perm[cells]
            pf = PH - beta * sigma * UH + beta * F / itf.flen
            dp = np.abs(pf - PH).max() / np.abs(r.p).max()
            df = np.abs(F - itf.flen * sigma * UH).max() / np.abs(r.Fx).max()
            if a < 1:
                worst_p, miss_f = max(worst_p, dp), min(miss_f, df)
            else:
                worst_f, miss_p = max(worst_f, df), min(miss_p, dp)
    assert worst_p < 1e-6 and worst_f < 1e-6
    # the other limit does not hold there (the check can tell them apart)
    assert miss_f > 1e-4 and miss_p > 1e-4
