"""Global fine-grid solve of eq. (Darcy) (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The single-domain two-point scheme with the same face laws as the local
problems (``discretization``): harmonic transmissibility on every interior
face, Dirichlet and Neumann data on the boundary, q |V| per cell.  It is the
reference that the pins "one subdomain = fine grid" and "full interface
spaces = fine grid" compare the MRCM against.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretization import (DIRICHLET, E, N, S, W, cell_injection, gravity_face_fluxes, harmonic,
                             neumann_outflow)


def _half_trans(kappa, flen, dist):
    return kappa * flen / dist


def solve_fine(prob, lam=None, rho=None):
    """Return dict(p, ux, uy, Fx, Fy) of the fine two-point solution.

    lam: per-cell total mobility (default 1), kappa = lam * K (section 3).
    rho: per-cell lambda_g / lambda when ``prob.gravity`` is not zero
    (section 5.5; the face terms of ``gravity_face_fluxes``).
    ux, uy are +x / +y normal velocities on the x- and y-faces; Fx, Fy the
    corresponding face fluxes (velocity times face length).
    For all-Neumann data the pressure is fixed by p_0 = 0 and then shifted
    to zero mean.
    """
    nx, ny = prob.nx, prob.ny
    hx, hy = prob.hx, prob.hy
    kappa = prob.perm * (1.0 if lam is None else np.asarray(lam, float))
    K = kappa.reshape(ny, nx)
    n = nx * ny
    idx = np.arange(n).reshape(ny, nx)
    rows, cols, vals = [], [], []
    rhs = cell_injection(prob, hx, hy).astype(np.float64, copy=True)

    def couple(a, b, T):
        rows.extend([a, b, a, b])
        cols.extend([a, b, b, a])
        vals.extend([T, T, -T, -T])

    # interior x-faces
    tx = _half_trans(K, hy, 0.5 * hx)
    Tx = harmonic(tx[:, :-1], tx[:, 1:])
    couple(idx[:, :-1].ravel(), idx[:, 1:].ravel(), Tx.ravel())
    ty = _half_trans(K, hx, 0.5 * hy)
    Ty = harmonic(ty[:-1, :], ty[1:, :])
    couple(idx[:-1, :].ravel(), idx[1:, :].ravel(), Ty.ravel())
    rows = [np.concatenate([np.atleast_1d(r) for r in rows])]
    cols = [np.concatenate([np.atleast_1d(c) for c in cols])]
    vals = [np.concatenate([np.atleast_1d(v) for v in vals])]

    sides = {W: (idx[:, 0], tx[:, 0], hy), E: (idx[:, -1], tx[:, -1], hy),
             S: (idx[0, :], ty[0, :], hx), N: (idx[-1, :], ty[-1, :], hx)}
    for side, (cells, t, flen) in sides.items():
        v = prob.bc_array(side)
        if prob.bc_kind[side] == DIRICHLET:
            rows.append(cells)
            cols.append(cells)
            vals.append(t)
            np.add.at(rhs, cells, t * v)
        else:
            np.add.at(rhs, cells, -neumann_outflow(v, flen))
    # gravity: the constant part of every y-face flux moves to the data
    GY = gravity_face_fluxes(prob, kappa, rho)
    rhs -= (GY[1:, :] - GY[:-1, :]).reshape(-1)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n))
    pure_neumann = not prob.has_dirichlet()
    if pure_neumann:
        A = A.tolil()
        A[0, :] = 0.0
        A[0, 0] = 1.0
        A = A.tocsr()
        rhs[0] = 0.0
    p = spla.spsolve(A.tocsc(), rhs)
    if pure_neumann:
        p = p - p.mean()
    P = p.reshape(ny, nx)
    Fx = np.zeros((ny, nx + 1))
    Fy = np.zeros((ny + 1, nx))
    Fx[:, 1:-1] = Tx * (P[:, :-1] - P[:, 1:])
    Fy[1:-1, :] = Ty * (P[:-1, :] - P[1:, :])
    for side in (W, E, S, N):
        v = prob.bc_array(side)
        if side == W:
            out = tx[:, 0] * (P[:, 0] - v) if prob.bc_kind[W] == DIRICHLET else neumann_outflow(v, hy)
            Fx[:, 0] = -out
        elif side == E:
            out = tx[:, -1] * (P[:, -1] - v) if prob.bc_kind[E] == DIRICHLET else neumann_outflow(v, hy)
            Fx[:, -1] = out
        elif side == S:
            out = ty[0, :] * (P[0, :] - v) if prob.bc_kind[S] == DIRICHLET else neumann_outflow(v, hx)
            Fy[0, :] = -out
        else:
            out = ty[-1, :] * (P[-1, :] - v) if prob.bc_kind[N] == DIRICHLET else neumann_outflow(v, hx)
            Fy[-1, :] = out
    Fy += GY
    return dict(p=p, Fx=Fx.reshape(-1), Fy=Fy.reshape(-1),
                ux=(Fx / hy).reshape(-1), uy=(Fy / hx).reshape(-1))
