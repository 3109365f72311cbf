"""Pins of the transport oracle (section 4) against facts fixed by the
paper and the mathematics (CPU only).

* f and its derivatives: closed-form values, finite differences, and the
  inflection point of f for M = 10 (where f' is largest);
* the discrete step itself: on a row of cells with positive face fluxes the
  upwind implicit step decouples into one scalar monotone equation per cell
  in flow order, solved here by bisection, independently of Newton's method;
* mass balance of the converged step, and 0 <= s <= 1 at large time steps;
* the Buckley-Leverett limit: the implicit upwind scheme converges to the
  self-similar solution (rarefaction to the front saturation s_f with
  f'(s_f) = f(s_f) / s_f, then a shock).
"""
import numpy as np
import pytest
from scipy.optimize import brentq

import inputs
from inputs import Problem
from inputs.problems import DIRICHLET, NEUMANN
from oracle import transport as ot

M = 10.0


def test_fractional_flow_closed_forms():
    assert ot.frac_flow(0.0, M) == 0.0 and ot.frac_flow(1.0, M) == 1.0
    assert ot.frac_flow(0.5, M) == pytest.approx(M / (M + 1.0))
    s = np.linspace(0.01, 0.99, 99)
    h = 1e-6
    fd1 = (ot.frac_flow(s + h, M) - ot.frac_flow(s - h, M)) / (2 * h)
    assert np.allclose(ot.frac_flow_d1(s, M), fd1, rtol=1e-7, atol=1e-9)
    fd2 = (ot.frac_flow_d1(s + h, M) - ot.frac_flow_d1(s - h, M)) / (2 * h)
    mask = np.abs(fd2) > 1e-3
    assert np.array_equal(ot.frac_flow_d2_sign(s[mask], M), np.sign(fd2[mask]))


def test_inflection_point_for_m10():
    """f'' changes sign once, at s* = 0.18599 where f' peaks at 2.977."""
    s_star = brentq(lambda s: (ot.frac_flow_d1(s + 1e-7, M) - ot.frac_flow_d1(s - 1e-7, M)), 0.05, 0.5)
    assert s_star == pytest.approx(0.18599, abs=2e-5)
    assert ot.frac_flow_d1(s_star, M) == pytest.approx(2.977, abs=1e-3)
    assert ot.frac_flow_d2_sign(s_star - 1e-3, M) > 0 > ot.frac_flow_d2_sign(s_star + 1e-3, M)


def row_problem(n, wells=None, inflow=True):
    """One row of n unit-width cells; face fluxes are prescribed directly."""
    src = None
    if wells:
        src = np.zeros(n)
        for i, q in wells.items():
            src[i] = q
    return Problem(name="row", nx=n, ny=1, lx=float(n), ly=1.0, perm=np.ones(n), sub_nx=n, sub_ny=1,
                   bc_kind=(NEUMANN, DIRICHLET, NEUMANN, NEUMANN), bc_value=(None, None, None, None),
                   source=src)


def sequential_exact(s_old, Q_faces, dt, fin, prod_last=False):
    """Cells in flow order: s_i + dt Q_out,i f(s_i) = s_i^n + dt Q_in,i f(s_{i-1})
    (unit volumes), each by bisection on [0, 1] (left side increasing)."""
    n = s_old.size
    s = np.zeros(n)
    for i in range(n):
        inflow = Q_faces[i] * (fin if i == 0 else ot.frac_flow(s[i - 1], M))
        qout = Q_faces[i + 1] + (Q_faces[i] if (prod_last and i == n - 1) else 0.0)
        g = lambda x: x + dt * qout * ot.frac_flow(x, M) - s_old[i] - dt * inflow
        s[i] = brentq(g, 0.0, 1.0, xtol=1e-16, rtol=1e-15) if g(1.0) > 0 else 1.0
    return s


@pytest.mark.parametrize("dt", [0.3, 3.0, 30.0])
def test_row_step_equals_sequential_scalar_solves(dt):
    """Inflow through W, outflow through E: Newton's solution of the coupled
    system equals the cell-by-cell scalar solves."""
    n = 12
    prob = row_problem(n)
    rng = np.random.default_rng(1)
    s_old = np.sort(rng.uniform(0, 1, n))[::-1]
    Q = np.full(n + 1, 0.7)
    st = ot.transport_step(prob, s_old, Q, np.zeros(2 * n), dt, s_inflow=1.0, eta=1e-14, max_iter=200)
    assert st.converged
    exact = sequential_exact(s_old, Q, dt, fin=1.0)
    assert np.abs(st.s - exact).max() < 1e-12


def test_row_with_injector_and_producer():
    """No boundary flow: an injector (water only) in the first cell and a
    producer (the mixture, f(s)) in the last one."""
    n = 10
    Qw = 0.4
    prob = row_problem(n, wells={0: Qw, n - 1: -Qw})
    Q = np.full(n + 1, Qw)
    Q[0] = Q[-1] = 0.0
    s_old = np.linspace(0.6, 0.0, n)
    dt = 5.0
    st = ot.transport_step(prob, s_old, Q, np.zeros(2 * n), dt, s_inflow=0.0, eta=1e-14, max_iter=200)
    assert st.converged
    # the same sequence: the injector's water enters cell 0 like a boundary
    # inflow of f = 1, the producer takes f(s_last) out of the last cell
    Qseq = np.full(n + 1, Qw)
    Qseq[-1] = 0.0
    exact = sequential_exact(s_old, Qseq, dt, fin=1.0, prod_last=True)
    assert np.abs(st.s - exact).max() < 1e-12


def test_mass_balance_and_bounds_at_large_steps():
    """Quarter-five-spot fluxes from a Darcy solve, 20 and 200 CFL steps:
    every saturation stays in [0, 1], the step converges, and the water in
    the domain changes by dt times the net injection (sum of V H = 0)."""
    from oracle.discretization import total_mobility
    from oracle.mrcm import solve_mrcm
    prob = inputs.make_problem("channel256_q5", nx=32, ny=32, sub=8)
    s0 = np.zeros(prob.nx * prob.ny)
    r = solve_mrcm(prob, lam=total_mobility(s0, prob.mu_w, prob.mu_o))
    dt_cfl = ot.cfl_time_step(prob, r.ux, r.uy)
    s = s0
    for mult in (20.0, 200.0):
        st = ot.transport_step(prob, s, r.Fx, r.Fy, mult * dt_cfl, eta=1e-10, max_iter=200)
        assert st.converged
        assert st.s.min() >= 0.0 and st.s.max() <= 1.0
        V = prob.hx * prob.hy
        out, src = ot.water_outflow(prob, st.s, r.Fx, r.Fy, 1.0, M)
        lhs = V * (st.s - s).sum()
        rhs = mult * dt_cfl * (src.sum() - out.sum())
        assert lhs == pytest.approx(rhs, rel=1e-9, abs=1e-12)
        assert lhs > 0     # water was injected
        s = st.s


def _bl_exact(x, t):
    sf = brentq(lambda s: ot.frac_flow_d1(s, M) * s - ot.frac_flow(s, M), 0.05, 0.99)
    xf = ot.frac_flow_d1(sf, M) * t
    out = np.zeros_like(x)
    ahead = x < xf
    # rarefaction: f'(s) = x / t for s in [s_f, 1]
    for k in np.nonzero(ahead)[0]:
        target = x[k] / t
        out[k] = brentq(lambda s: ot.frac_flow_d1(s, M) - target, sf, 1.0) if target > 0 else 1.0
    return out, sf


def test_buckley_leverett_limit():
    """Unit inflow into an oil-filled row: the implicit upwind solution at
    t = 0.25 approaches the Buckley-Leverett solution as the grid and the
    time step are refined."""
    errs = []
    for n in (100, 200):
        prob = row_problem(n)
        prob = prob.replace(lx=1.0, ly=1.0 / n)
        Q = np.full(n + 1, 1.0 / n)          # u = 1 through faces of length 1/n
        dt = 0.5 / n / 2.977                  # CFL 0.5
        t_end = 0.25
        steps = int(round(t_end / dt))
        dt = t_end / steps
        s = np.zeros(n)
        for _ in range(steps):
            s = ot.transport_step(prob, s, Q, np.zeros(2 * n), dt, eta=1e-10).s
        x = (np.arange(n) + 0.5) / n
        exact, sf = _bl_exact(x, t_end)
        errs.append(np.abs(s - exact).mean())
    assert errs[1] < 0.75 * errs[0]
    assert errs[1] < 0.03


# --------------------------------------------------------------------------
# planted mistakes in the transport oracle must fail a pin
# --------------------------------------------------------------------------

def _transport_pins_pass():
    try:
        test_row_step_equals_sequential_scalar_solves(30.0)
        test_row_with_injector_and_producer()
        test_mass_balance_and_bounds_at_large_steps()
    except AssertionError:
        return False
    return True


def test_unmodified_transport_oracle_passes():
    assert _transport_pins_pass()


def test_dropped_inflection_rule_caught(monkeypatch):
    """Without the inflection-point halving, Newton's method does not
    converge at large steps."""
    monkeypatch.setattr(ot, "frac_flow_d2_sign", lambda s, M: np.ones_like(np.asarray(s, float)))
    assert not _transport_pins_pass()


def test_producer_taking_water_only_caught(monkeypatch):
    """A producer that removes water only (w = q) instead of the mixture."""
    orig = ot.water_outflow

    def wrong(prob, s, Fx, Fy, s_inflow, M):
        out, src = orig(prob, s, Fx, Fy, s_inflow, M)
        qv = ot.cell_injection(prob, prob.hx, prob.hy)
        return out, np.where(qv < 0, qv, src)
    monkeypatch.setattr(ot, "water_outflow", wrong)
    assert not _transport_pins_pass()


def test_downwind_fluxes_caught(monkeypatch):
    """f taken from the cell the flux enters instead of the one it leaves."""
    def downwind(prob, s, Fx, Fy, s_inflow, M):
        nx, ny = prob.nx, prob.ny
        FX, FY = ot._face_fluxes(prob, Fx, Fy)
        f = ot.frac_flow(np.asarray(s, float).reshape(ny, nx), M)
        fin = float(ot.frac_flow(s_inflow, M))
        WX = np.zeros_like(FX)
        WY = np.zeros_like(FY)
        WX[:, 1:-1] = np.where(FX[:, 1:-1] > 0, f[:, 1:], f[:, :-1]) * FX[:, 1:-1]
        WY[1:-1, :] = np.where(FY[1:-1, :] > 0, f[1:, :], f[:-1, :]) * FY[1:-1, :]
        WX[:, 0] = np.where(FX[:, 0] > 0, fin, f[:, 0]) * FX[:, 0]
        WX[:, -1] = np.where(FX[:, -1] > 0, f[:, -1], fin) * FX[:, -1]
        WY[0, :] = np.where(FY[0, :] > 0, fin, f[0, :]) * FY[0, :]
        WY[-1, :] = np.where(FY[-1, :] > 0, f[-1, :], fin) * FY[-1, :]
        out = (WX[:, 1:] - WX[:, :-1] + WY[1:, :] - WY[:-1, :]).reshape(-1)
        qv = ot.cell_injection(prob, prob.hx, prob.hy)
        return out, np.where(qv > 0, qv, qv * f.reshape(-1))
    monkeypatch.setattr(ot, "water_outflow", downwind)
    assert not _transport_pins_pass()


# --------------------------------------------------------------------------
# sequential fully implicit outer loop (section 5.4)
# --------------------------------------------------------------------------

def _q5(n=32):
    from oracle.discretization import total_mobility
    from oracle.mrcm import solve_mrcm
    prob = inputs.make_problem("channel256_q5", nx=n, ny=n, sub=8)
    s0 = np.zeros(prob.nx * prob.ny)
    r = solve_mrcm(prob, lam=total_mobility(s0, prob.mu_w, prob.mu_o))
    return prob, s0, ot.cfl_time_step(prob, r.ux, r.uy)


def test_sfi_is_a_fixed_point_of_darcy_and_transport():
    """At convergence the new saturation is (to the outer tolerance) the
    transport step of the fluxes of its own Darcy solve: one more outer
    iteration changes it by less than 1e-4."""
    from oracle.discretization import total_mobility
    from oracle.mrcm import solve_mrcm
    prob, s0, dt_cfl = _q5()
    st = ot.sfi_step(prob, s0, 20 * dt_cfl)
    assert st.converged and st.outer >= 2
    assert st.changes[-1] < 1e-4 and all(c < 1 for c in st.changes)
    r = solve_mrcm(prob, lam=total_mobility(st.s, prob.mu_w, prob.mu_o))
    again = ot.transport_step(prob, s0, r.Fx, r.Fy, 20 * dt_cfl)
    assert np.abs(again.s - st.s).max() < 1e-4
    # mass balance of the step with the fluxes the last transport used
    out, src = ot.water_outflow(prob, st.s, st.Fx, st.Fy, 1.0, M)
    V = prob.hx * prob.hy
    assert V * (st.s - s0).sum() == pytest.approx(20 * dt_cfl * (src.sum() - out.sum()), rel=1e-6)


def test_sfi_first_iterate_is_the_sequential_implicit_step():
    """The first outer iteration is the SI step (Darcy with s^n, then
    transport); with one outer iteration allowed they coincide."""
    prob, s0, dt_cfl = _q5()
    one = ot.sfi_step(prob, s0, 5 * dt_cfl, max_outer=1)
    traj, _ = ot.si_run(prob, s0, 1, 5 * dt_cfl)
    assert np.array_equal(one.s, traj[1])


def test_sfi_and_si_agree_as_dt_shrinks():
    """SI and SFI differ by the splitting error, which falls with dt."""
    prob, s0, dt_cfl = _q5()
    diffs = []
    for mult in (8.0, 2.0):
        sfi = ot.sfi_step(prob, s0, mult * dt_cfl, outer_tol=1e-10)
        traj, _ = ot.si_run(prob, s0, 1, mult * dt_cfl)
        diffs.append(np.abs(sfi.s - traj[1]).max())
    assert diffs[1] < 0.5 * diffs[0]
