"""Helpers shared by the GPU parity tests: run the HIP path through the C
ABI, run the oracle on the same seeded inputs, and map the oracle's
per-subdomain quantities onto the library's padded layout."""
import sys

import numpy as np

from oracle.discretization import Geometry, total_mobility
from oracle.mrcm import solve_mrcm


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def run_gpu(prob, s=None, lam=None, precision="fp64", extras=True):
    from paper_2104_04653_amd import MRCMSolver
    out = {}
    with MRCMSolver(prob, precision=precision) as sol:
        if s is not None:
            sol.update_mobility(s)
        elif lam is not None:
            sol.update_mobility(lam, is_lambda=True)
        sol.solve()
        out["p"], out["ux"], out["uy"], out["imbalance"] = sol.fine_flux()
        out["stats"] = sol.stats()
        if extras:
            out["coef"] = sol.interface_solution() if sol.n_dof else np.zeros(0)
        if extras == True:  # noqa: E712 - "coef" asks for the coefficients only
            out["blocks"] = sol.local_blocks()
            out["basis"] = sol.basis()
    return out


def run_oracle(prob, s=None, lam=None, **kw):
    if s is not None:
        lam = total_mobility(s, prob.mu_w, prob.mu_o)
    return solve_mrcm(prob, lam=lam, **kw)


def padded_columns(prob, sd):
    """Library column index of every oracle column of subdomain sd."""
    g = Geometry(prob)
    D = prob.p_dofs + prob.u_dofs
    cols = [0]
    for side in range(4):
        if g.sub_iface[sd, side] >= 0:
            cols.extend(1 + side * D + k for k in range(D))
    return np.array(cols)


def oracle_blocks_padded(prob, ref):
    """Oracle blocks in the library's padded layout and sign convention."""
    g = Geometry(prob)
    D = prob.p_dofs + prob.u_dofs
    NB = 4 * D
    out = np.zeros((g.n_sub, NB, NB + 1))
    for sd in range(g.n_sub):
        cols = padded_columns(prob, sd)[1:] - 1          # padded positions of its dofs
        blk = ref.blocks[sd]                             # natural form, [rows, 1 + ndof]
        sgn = np.where((np.arange(len(cols)) % D) < prob.p_dofs, 1.0, -1.0)
        for r, pr in enumerate(cols):
            out[sd, pr, cols] = sgn[r] * blk[r, 1:1 + len(cols)]
            out[sd, pr, NB] = -sgn[r] * blk[r, 0]
    if not prob.has_dirichlet() and g.n_iface:
        # gauge: global dof 0 (first pressure dof of interface 0) is fixed to
        # zero; its row and column become the identity in the lower-index
        # subdomain's block and vanish in the other one
        itf = g.interfaces[0]
        for sd, side in ((itf.lo, itf.lo_side), (itf.hi, itf.hi_side)):
            r0 = side * D
            out[sd, r0, :] = 0.0
            out[sd, :, r0] = 0.0
            if sd == itf.lo:
                out[sd, r0, r0] = 1.0
    return out


def oracle_basis_padded(prob, ref):
    g = Geometry(prob)
    D = prob.p_dofs + prob.u_dofs
    R = 1 + 4 * D
    m = prob.sub_nx
    out = np.zeros((g.n_sub, m * m, R))
    for sd in range(g.n_sub):
        I, J = sd % g.SX, sd // g.SX
        li, lj = np.meshgrid(np.arange(m), np.arange(m))
        cells = ((J * m + lj) * g.nx + I * m + li).reshape(-1)
        cols = padded_columns(prob, sd)
        out[sd][:, cols] = ref.X[cells][:, :len(cols)]
    return out
