"""Sequential-implicit transport of the water saturation (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Section 4 of the paper, step by step:

* implicit Euler in time with the velocity frozen at the previous Darcy
  solve (eq. (BL2D_Newton)); in finite-volume form
  H(s) = s - s^n + (dt / V) (F(s) - V w(s)) = 0 per cell
  (eqs. (BL2D_Newton2), (BL2D_Newton7)), F the net water outflow of the
  cell, w the water source of its wells;
* F from first-order upwind face fluxes (eqs. (fluxes_impli),
  (up_fluxes_impli)): a face carries f(s) of the cell its total flux leaves;
  a boundary face with inflow carries f of the injection saturation s_bar
  (the inlet condition of eq. (BL2D));
* Newton's method on H (eq. (BL2D_Newton8)) with the inflection-point
  strategy of the trust-region subsection: every saturation is kept in
  [0, 1], and an update that moves a cell's saturation across the
  inflection point of f (f'' changes sign) is halved.  The paper states the
  halving with f'' at the new iterate and the bound "after every
  iteration"; f and f'' are defined on [0, 1] only, so the new iterate is
  projected onto [0, 1] before f'' is evaluated there (halving first and
  clamping after oscillates between 0 and 1 at large steps: a 12-cell row
  at 60 CFL never converges that way);
* stop when the L2 norm of the change, sqrt(sum_I V_I (s^{nu+1} - s^nu)^2),
  is at most eta (1e-6 in section 5).

Wells (the quarter-five-spot reading): an injector (q > 0) injects water
only, w = q; a producer (q < 0) produces the mixture, w = q f(s).

The relative permeabilities of section 5 (k_rw = s^2, k_ro = (1-s)^2) give
f(s) = M s^2 / (M s^2 + (1-s)^2), M = mu_o / mu_w (eq. (fluxos2)).

Each Newton step solves the Jacobian system with a sparse direct solver
(SuperLU).

The sequential fully implicit variant of section 5.4 (``sfi_step``) repeats
the Darcy solve and the transport step within a time step until the
saturation changes by less than 1e-4 between successive outer iterations.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretization import DIRICHLET, E, N, S, W, cell_injection


def frac_flow(s, M):
    """f(s) = M s^2 / (M s^2 + (1-s)^2) (eq. (fluxos2) with section 5's k_r)."""
    s = np.asarray(s, dtype=np.float64)
    return M * s * s / (M * s * s + (1.0 - s) ** 2)


def frac_flow_d1(s, M):
    """f'(s) = 2 M s (1-s) / (M s^2 + (1-s)^2)^2."""
    s = np.asarray(s, dtype=np.float64)
    den = M * s * s + (1.0 - s) ** 2
    return 2.0 * M * s * (1.0 - s) / (den * den)


def frac_flow_d2_sign(s, M):
    """Sign of f''(s): f' = N / D^2 with N = 2 M s (1-s), D = M s^2 + (1-s)^2,
    so f'' = (N' D - 2 N D') / D^3 and D > 0."""
    s = np.asarray(s, dtype=np.float64)
    n, dn = 2.0 * M * s * (1.0 - s), 2.0 * M * (1.0 - 2.0 * s)
    d, dd = M * s * s + (1.0 - s) ** 2, 2.0 * M * s - 2.0 * (1.0 - s)
    return np.sign(dn * d - 2.0 * n * dd)


@dataclasses.dataclass
class TransportStep:
    s: np.ndarray          # saturation at the new time level
    iterations: int        # Newton iterations taken
    converged: bool
    changes: list          # L2 norm of the change per iteration
    residual: float        # max |H| at the returned saturation


def _face_fluxes(prob, Fx, Fy):
    """Total volumetric fluxes through the faces (+x, +y), as 2-D arrays."""
    nx, ny = prob.nx, prob.ny
    return np.asarray(Fx, float).reshape(ny, nx + 1), np.asarray(Fy, float).reshape(ny + 1, nx)


def water_outflow(prob, s, Fx, Fy, s_inflow, M):
    """Net upwind water outflow F of every cell (eq. (fluxes_impli)) and the
    water source V w of its wells."""
    nx, ny = prob.nx, prob.ny
    FX, FY = _face_fluxes(prob, Fx, Fy)
    S2 = np.asarray(s, float).reshape(ny, nx)
    f = frac_flow(S2, M)
    fin = float(frac_flow(s_inflow, M))
    # water flux through every face in +x / +y: f of the upwind cell
    WX = np.zeros_like(FX)
    WY = np.zeros_like(FY)
    WX[:, 1:-1] = np.where(FX[:, 1:-1] > 0, f[:, :-1], f[:, 1:]) * FX[:, 1:-1]
    WY[1:-1, :] = np.where(FY[1:-1, :] > 0, f[:-1, :], f[1:, :]) * FY[1:-1, :]
    # boundary faces: outflow carries the cell's f, inflow the injected one
    WX[:, 0] = np.where(FX[:, 0] > 0, fin, f[:, 0]) * FX[:, 0]
    WX[:, -1] = np.where(FX[:, -1] > 0, f[:, -1], fin) * FX[:, -1]
    WY[0, :] = np.where(FY[0, :] > 0, fin, f[0, :]) * FY[0, :]
    WY[-1, :] = np.where(FY[-1, :] > 0, f[-1, :], fin) * FY[-1, :]
    out = (WX[:, 1:] - WX[:, :-1] + WY[1:, :] - WY[:-1, :]).reshape(-1)
    qv = cell_injection(prob, prob.hx, prob.hy)
    src = np.where(qv > 0, qv, qv * f.reshape(-1))
    return out, src


def residual(prob, s, s_old, Fx, Fy, dt, s_inflow, M):
    """H(s) = s - s^n + (dt / V) (F(s) - V w(s)) (eq. (BL2D_Newton7))."""
    V = prob.hx * prob.hy
    out, src = water_outflow(prob, s, Fx, Fy, s_inflow, M)
    return np.asarray(s, float) - s_old + dt / V * (out - src)


def jacobian(prob, s, Fx, Fy, dt, M):
    """H'(s): d H_I / d s_J from the upwind fluxes (the flux of a face depends
    on the saturation of its upwind cell only)."""
    nx, ny = prob.nx, prob.ny
    n = nx * ny
    V = prob.hx * prob.hy
    FX, FY = _face_fluxes(prob, Fx, Fy)
    fp = frac_flow_d1(np.asarray(s, float), M).reshape(ny, nx)
    idx = np.arange(n).reshape(ny, nx)
    c = dt / V
    diag = np.ones((ny, nx))
    rows, cols, vals = [], [], []

    def interior(Fi, lo, hi, fp_lo, fp_hi):
        pos = Fi > 0
        # flux lo -> hi carries f(s_lo): out of lo, into hi
        np.add.at(diag.reshape(-1), lo[pos], c * fp_lo[pos] * Fi[pos])
        rows.append(hi[pos]); cols.append(lo[pos]); vals.append(-c * fp_lo[pos] * Fi[pos])
        neg = ~pos
        # flux hi -> lo carries f(s_hi): out of hi, into lo
        np.add.at(diag.reshape(-1), hi[neg], -c * fp_hi[neg] * Fi[neg])
        rows.append(lo[neg]); cols.append(hi[neg]); vals.append(c * fp_hi[neg] * Fi[neg])

    interior(FX[:, 1:-1], idx[:, :-1], idx[:, 1:], fp[:, :-1], fp[:, 1:])
    interior(FY[1:-1, :], idx[:-1, :], idx[1:, :], fp[:-1, :], fp[1:, :])
    # boundary outflow faces depend on the cell's own saturation
    diag[:, 0] += np.where(FX[:, 0] < 0, -c * fp[:, 0] * FX[:, 0], 0.0)
    diag[:, -1] += np.where(FX[:, -1] > 0, c * fp[:, -1] * FX[:, -1], 0.0)
    diag[0, :] += np.where(FY[0, :] < 0, -c * fp[0, :] * FY[0, :], 0.0)
    diag[-1, :] += np.where(FY[-1, :] > 0, c * fp[-1, :] * FY[-1, :], 0.0)
    # producers: -(dt/V) V q f(s) with q < 0
    qv = cell_injection(prob, prob.hx, prob.hy).reshape(ny, nx)
    diag += np.where(qv < 0, -c * qv * fp, 0.0)
    rows.append(idx.reshape(-1)); cols.append(idx.reshape(-1)); vals.append(diag.reshape(-1))
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(n, n))


def transport_step(prob, s_old, Fx, Fy, dt, s_inflow=1.0, eta=1e-6, max_iter=50):
    """One implicit Euler step of eq. (BL2D) from s_old with the face fluxes
    (Fx, Fy) of the last Darcy solve, by Newton's method with the
    inflection-point strategy (section 4)."""
    M = prob.mu_o / prob.mu_w
    V = prob.hx * prob.hy
    s_old = np.asarray(s_old, dtype=np.float64)
    s = s_old.copy()
    changes = []
    converged = False
    for it in range(1, max_iter + 1):
        H = residual(prob, s, s_old, Fx, Fy, dt, s_inflow, M)
        J = jacobian(prob, s, Fx, Fy, dt, M)
        d = spla.spsolve(J.tocsc(), -H)
        # keep 0 <= s <= 1 (f is defined there), then the inflection-point
        # strategy: an update that crosses the inflection point of f is
        # halved (both ends lie in [0, 1], so the half does too)
        s_new = np.clip(s + d, 0.0, 1.0)
        cross = frac_flow_d2_sign(s_new, M) * frac_flow_d2_sign(s, M) < 0
        s_new = np.where(cross, 0.5 * (s_new + s), s_new)
        change = float(np.sqrt(V * np.sum((s_new - s) ** 2)))
        changes.append(change)
        s = s_new
        if change <= eta:
            converged = True
            break
    H = residual(prob, s, s_old, Fx, Fy, dt, s_inflow, M)
    return TransportStep(s=s, iterations=it, converged=converged, changes=changes,
                         residual=float(np.abs(H).max()))


def cfl_time_step(prob, ux, uy):
    """dt_CFL = h / (max f' max |u|) for the fractional flow of section 5."""
    M = prob.mu_o / prob.mu_w
    s = np.linspace(0.0, 1.0, 200001)
    fmax = float(frac_flow_d1(s, M).max())
    umax = max(np.abs(ux).max(), np.abs(uy).max())
    return min(prob.hx, prob.hy) / (fmax * umax)


def si_run(prob, s0, n_steps, dt, s_inflow=1.0, eta=1e-6, darcy=None):
    """The sequential implicit loop of section 4: Darcy with the current
    saturation (the MRCM, or any solver ``darcy(prob, lam) -> (Fx, Fy)``),
    then one transport step with those fluxes; returns the saturations
    s^0 .. s^n and the Newton iteration counts."""
    from .discretization import total_mobility
    from .mrcm import solve_mrcm
    if darcy is None:
        def darcy(p, lam):
            r = solve_mrcm(p, lam=lam)
            return r.Fx, r.Fy
    traj = [np.asarray(s0, dtype=np.float64)]
    iters = []
    for _ in range(n_steps):
        lam = total_mobility(traj[-1], prob.mu_w, prob.mu_o)
        Fx, Fy = darcy(prob, lam)
        st = transport_step(prob, traj[-1], Fx, Fy, dt, s_inflow=s_inflow, eta=eta)
        traj.append(st.s)
        iters.append(st.iterations)
    return traj, iters


@dataclasses.dataclass
class SFIStep:
    s: np.ndarray          # saturation at the new time level
    outer: int             # outer (Darcy + transport) iterations
    converged: bool
    changes: list          # max |s^{k+1} - s^k| per outer iteration
    newton: list           # Newton iterations of each transport solve
    Fx: np.ndarray         # face fluxes of the last Darcy solve
    Fy: np.ndarray


def sfi_step(prob, s_old, dt, s_inflow=1.0, eta=1e-6, outer_tol=1e-4, max_outer=50, darcy=None):
    """One time step of the sequential fully implicit scheme (section 5.4):
    starting from s^{n+1,0} = s^n, repeat a Darcy solve with the current
    saturation and a transport step from s^n with its fluxes, until the
    largest change of the saturation between successive outer iterations
    is below outer_tol (1e-4 in the paper, with eta = 1e-6 for Newton)."""
    from .discretization import total_mobility
    from .mrcm import solve_mrcm
    if darcy is None:
        def darcy(p, lam):
            r = solve_mrcm(p, lam=lam)
            return r.Fx, r.Fy
    s_old = np.asarray(s_old, dtype=np.float64)
    s = s_old.copy()
    changes, newton = [], []
    converged = False
    for k in range(1, max_outer + 1):
        Fx, Fy = darcy(prob, total_mobility(s, prob.mu_w, prob.mu_o))
        st = transport_step(prob, s_old, Fx, Fy, dt, s_inflow=s_inflow, eta=eta)
        newton.append(st.iterations)
        change = float(np.abs(st.s - s).max())
        changes.append(change)
        s = st.s
        if change < outer_tol:
            converged = True
            break
    return SFIStep(s=s, outer=k, converged=converged, changes=changes, newton=newton, Fx=Fx, Fy=Fy)
