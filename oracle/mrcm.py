"""The Multiscale Robin Coupled Method, step by step (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Follows section 3 of the paper:

1. kappa = lambda(s) K (text after eq. (mrc2)); Robin parameter
   beta_i = alpha H / kappa_i (eq. (beta)), kappa_i taken in the cell beside
   the face on side i.
2. Local problems (eq. (mrc1)) on every subdomain: Darcy with the physical
   boundary data on the domain boundary and the Robin condition
   -beta u.n_i + p = -beta U_H (n.n_i) + P_H on the skeleton.  By linearity
   the local solution is a particular solution (interface data zero) plus one
   basis function per interface degree of freedom (section 3, paragraph after
   eq. (beta)): pressure dof l of interface e sets g = psi_l on e's faces,
   flux dof l sets g = -beta sigma phi_l.
3. Traces of every local solution on the skeleton: Robin face flux
   F = T_R (p_c - g) and face pressure p_f = g + beta F / |f|.
4. Interface system (eq. (mrc2), equivalently eq. (compatibility)):
   for every pressure function psi_l:  sum over both sides of
   sum_f psi_l(f) F_f = 0 (weak flux continuity);
   for every flux function phi_l: sum_f |f| phi_l(f) (p_f^lo - p_f^hi) = 0
   (weak pressure continuity; equal to the beta-form of eq. (mrc2) because
   beta (u.n_i - U_H sigma) = p_f - P_H and the P_H terms cancel).
5. Solve for (P_H, U_H); compose the cell pressure and the face fluxes as the
   same linear combination of the local solutions.
6. Stitch (the downscaling step that the paper cites for continuous
   interface fluxes; the cited procedure is not reproduced in the paper, so
   this is the reading adopted): the interface flux is the average of the two
   one-sided Robin fluxes, and every subdomain is re-solved with that flux as
   Neumann data, which gives a single-valued, locally conservative fine flux.

The dense "blocks" returned per subdomain are that subdomain's contribution
to the interface system in its natural form: rows are the subdomain's
interface equations, column 0 the particular solution's contribution and
columns 1.. its interface dofs, in the order of the interfaces on its W, E,
S and N sides.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .discretization import (DIRICHLET, E, N, S, W, Geometry, cell_injection, gravity_face_fluxes,
                             harmonic, interface_alpha, interface_spaces, neumann_outflow)


@dataclasses.dataclass
class MRCMResult:
    p: np.ndarray              # composed multiscale cell pressure
    ux: np.ndarray             # stitched +x velocity on x-faces, (nx+1)*ny
    uy: np.ndarray             # stitched +y velocity on y-faces, nx*(ny+1)
    Fx: np.ndarray             # stitched +x face fluxes
    Fy: np.ndarray             # stitched +y face fluxes
    Fx_raw: np.ndarray         # multiscale fluxes before stitching (skeleton: side average)
    Fy_raw: np.ndarray
    side_flux: list            # per interface: (F_lo, F_hi), outward from each side
    coeffs: np.ndarray         # interface unknowns, per interface [P.., U..]
    blocks: list               # per subdomain: natural-form interface block
    sub_dofs: list             # per subdomain: global dofs of its columns 1..
    X: np.ndarray              # local solutions, (n_cells, R) columns as in blocks
    p_stitch: np.ndarray       # pressure of the stitch re-solve
    imbalance_raw: float       # max cell imbalance / max |F| of the raw MRCM flux
    imbalance: float           # same for the stitched flux
    stitch_defect: float       # largest compatibility defect of a floating
                               # subdomain's Neumann data / max |F| (removed
                               # evenly from its cells; rounding level)
    interface_matrix: sp.csr_matrix
    interface_rhs: np.ndarray
    dof_offset: np.ndarray
    n_p: np.ndarray
    n_u: np.ndarray


def _bc_faces(geom, prob, kappa):
    """Physical boundary faces: (side, cells, half transmissibility, |f|, values)."""
    nx, ny, hx, hy = geom.nx, geom.ny, geom.hx, geom.hy
    idx = np.arange(nx * ny).reshape(ny, nx)
    out = []
    for side, cells, flen, dist in ((W, idx[:, 0], hy, 0.5 * hx), (E, idx[:, -1], hy, 0.5 * hx),
                                    (S, idx[0, :], hx, 0.5 * hy), (N, idx[-1, :], hx, 0.5 * hy)):
        t = kappa[cells] * flen / dist
        out.append((side, cells, t, flen, prob.bc_array(side)))
    return out


def local_operator(geom, prob, kappa, robin_T=None, extended=False, GY=None):
    """Block-diagonal matrix of all local problems and their data vector.

    Interior faces of a subdomain: harmonic two-point coupling; physical
    boundary faces: Dirichlet (diagonal t_c, data t_c p_b) or Neumann (data
    -u_b |f|); source q |V|.  Skeleton faces add the Robin diagonal T_R when
    ``robin_T`` (a list of (cells, T_R) pairs) is given; without it they are
    left as zero-flux faces (for the stitch re-solve the prescribed flux is
    added to the data by the caller).  GY: the gravity part of the +y face
    fluxes (``gravity_face_fluxes``); it enters the data on the faces inside
    subdomains and on the physical boundary (the skeleton faces' gravity
    terms are the callers').
    """
    nx, ny, mx, my = geom.nx, geom.ny, geom.mx, geom.my
    hx, hy = geom.hx, geom.hy
    n = nx * ny
    K = kappa.reshape(ny, nx)
    idx = np.arange(n).reshape(ny, nx)
    rows, cols, vals = [], [], []

    def couple(a, b, T):
        rows.extend([a, b, a, b])
        cols.extend([a, b, b, a])
        vals.extend([T, T, -T, -T])

    tx = K * hy / (0.5 * hx)
    ty = K * hx / (0.5 * hy)
    Tx = harmonic(tx[:, :-1], tx[:, 1:])
    same_x = (np.arange(1, nx) % mx) != 0
    couple(idx[:, :-1][:, same_x].ravel(), idx[:, 1:][:, same_x].ravel(), Tx[:, same_x].ravel())
    Ty = harmonic(ty[:-1, :], ty[1:, :])
    same_y = (np.arange(1, ny) % my) != 0
    couple(idx[:-1, :][same_y, :].ravel(), idx[1:, :][same_y, :].ravel(), Ty[same_y, :].ravel())

    rhs = cell_injection(prob, hx, hy).astype(np.float64, copy=True)
    for side, cells, t, flen, v in _bc_faces(geom, prob, kappa):
        if prob.bc_kind[side] == DIRICHLET:
            rows.append(cells)
            cols.append(cells)
            vals.append(t)
            np.add.at(rhs, cells, t * v)
        else:
            np.add.at(rhs, cells, -neumann_outflow(v, flen))
    if GY is not None:
        G = GY.copy()
        G[1:-1, :][~same_y, :] = 0.0          # skeleton faces
        rhs -= (G[1:, :] - G[:-1, :]).reshape(-1)
    if robin_T is not None:
        for cells, T in robin_T:
            rows.append(cells)
            cols.append(cells)
            vals.append(T)
    rr, cc, vv = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    A = sp.csr_matrix((vv, (rr, cc)), shape=(n, n))
    if extended:
        # the same entries with the duplicates (the diagonal's sums of
        # transmissibilities) summed in the x87 extended format: its products
        # with a solution are the cells' mass balances (flux form), where the
        # FP64-summed diagonal leaves eps T |p| per cell
        A_ext = sp.csr_matrix((vv.astype(np.longdouble), (rr, cc)), shape=(n, n))
        return A, rhs, (Tx, Ty, tx, ty, same_x, same_y), A_ext
    return A, rhs, (Tx, Ty, tx, ty, same_x, same_y)


def _side_records(geom, prob, kappa, alpha, rho=None):
    """Robin data of every skeleton face, per interface and side.  G is the
    gravity part of the Robin flux out of the side's subdomain: the half-cell
    term t_c rho_c gamma d (n . e_y) through T_R = t_c / (1 + t_c beta / |f|),
    i.e. T_R rho_c gamma d (n . e_y) (zero on vertical interfaces)."""
    recs = []
    for itf in geom.interfaces:
        a = alpha[itf.index]
        per = []
        for cells, sub, side, sigma in ((itf.lo_cells, itf.lo, itf.lo_side, 1.0),
                                        (itf.hi_cells, itf.hi, itf.hi_side, -1.0)):
            kc = kappa[cells]
            TR = itf.flen * kc / (itf.dist + a * itf.H)
            beta = a * itf.H / kc
            G = np.zeros(cells.size)
            if rho is not None and prob.gravity != 0.0 and not itf.vertical:
                ny_out = 1.0 if side == N else -1.0
                G = TR * rho[cells] * prob.gravity * itf.dist * ny_out
            per.append(dict(cells=cells, sub=sub, side=side, sigma=sigma, TR=TR, beta=beta, G=G))
        recs.append(per)
    return recs


def _dof_layout(geom, spaces):
    n_p = np.array([ps.shape[0] for ps, _ in spaces], dtype=np.int64)
    n_u = np.array([us.shape[0] for _, us in spaces], dtype=np.int64)
    off = np.zeros(geom.n_iface + 1, dtype=np.int64)
    off[1:] = np.cumsum(n_p + n_u)
    sub_dofs = []
    col_off = np.zeros((geom.n_sub, 4), dtype=np.int64)
    for sd in range(geom.n_sub):
        dofs = []
        for side in (W, E, S, N):
            e = geom.sub_iface[sd, side]
            col_off[sd, side] = 1 + len(dofs)
            if e >= 0:
                dofs.extend(range(off[e], off[e + 1]))
        sub_dofs.append(np.array(dofs, dtype=np.int64))
    R = 1 + max((len(d) for d in sub_dofs), default=0)
    return n_p, n_u, off, sub_dofs, col_off, R


def _interface_data(itf, rec, ps, us, col):
    """g on the interface's faces for each column of the side's subdomain."""
    m = itf.faces.size
    nP, nU = ps.shape[0], us.shape[0]
    G = np.zeros((m, nP + nU))
    G[:, :nP] = ps.T
    G[:, nP:] = (-rec["beta"] * rec["sigma"])[:, None] * us.T
    return G


RESIDUAL = "extended"   # or "fp64"


def _residual(A, x, b):
    """b - A x.  With RESIDUAL == "extended" the products and sums are taken
    in the x87 extended format (64-bit mantissa) and rounded once, so that
    refinement converges to the FP64 solution of the FP64 data instead of
    stalling at condition-number times FP64 rounding.  A may already hold
    extended entries (a matrix assembled in extended precision)."""
    if RESIDUAL == "extended":
        ld = np.longdouble
        return (np.asarray(b, dtype=ld) - A.astype(ld) @ np.asarray(x, dtype=ld)).astype(np.float64)
    return b - A @ x


def _refined(A, solve, b, steps=3, A_res=None):
    """x = A^-1 b by a direct solve plus iterative refinement steps; the
    residuals use A_res (default A)."""
    x = solve(b)
    A = (A if A_res is None else A_res).tocsr()
    for _ in range(steps):
        x = x + solve(_residual(A, x, b))
    return x


def _refined_extended(solve, b, residual, steps=3):
    """x = A^-1 b carried in the x87 extended format: a direct solve, then
    refinement steps x += A^-1 r with r = residual(x) formed in extended
    precision and the accumulated solution kept extended."""
    x = solve(b).astype(np.longdouble)
    for _ in range(steps):
        x = x + solve(residual(x).astype(np.float64))
    return x


def _local_solve(A, B, geom, method, A_ext=None):
    if method == "superlu":
        lu = spla.splu(A.tocsc())
        return _refined(A, lu.solve, B, A_res=A_ext)
    if method == "banded":
        # one LAPACK banded Cholesky per subdomain in the local natural
        # ordering, whose half-bandwidth is the subdomain width
        X = np.zeros_like(B)
        mx, my, nx = geom.mx, geom.my, geom.nx
        A = A.tocsr()
        for sd in range(geom.n_sub):
            I, J = sd % geom.SX, sd // geom.SX
            li, lj = np.meshgrid(np.arange(mx), np.arange(my))
            cells = ((J * my + lj) * nx + I * mx + li).reshape(-1)
            Ad = A[cells][:, cells].toarray()
            nb = mx
            ab = np.zeros((nb + 1, cells.size))
            for d in range(nb + 1):
                ab[d, : cells.size - d] = np.diagonal(Ad, -d)
            c = sla.cholesky_banded(ab, lower=True)
            X[cells] = sla.cho_solve_banded((c, True), B[cells])
        return X

    if method == "banded_refined":
        return _refined(A, lambda r: _local_solve(A, r, geom, "banded"), B, A_res=A_ext)
    raise ValueError(method)


def _interface_solve(M, b, method, ir_steps):
    if M.shape[0] == 0:
        return np.zeros(0)
    if method == "superlu":
        lu = spla.splu(M.tocsc())
        solve = lu.solve
    elif method == "dense":
        Md = M.toarray()
        lu = sla.lu_factor(Md)
        solve = lambda r: sla.lu_solve(lu, r)
    else:
        raise ValueError(method)
    x = solve(b)
    Mc = M.tocsr()
    for _ in range(ir_steps):
        x = x + solve(_residual(Mc, x, b))
    return x


def flux_imbalance(geom, prob, Fx, Fy):
    """max over cells |net outflow - q |V|| / max |F| (section 2 balance)."""
    nx, ny = geom.nx, geom.ny
    FX = Fx.reshape(ny, nx + 1)
    FY = Fy.reshape(ny + 1, nx)
    net = FX[:, 1:] - FX[:, :-1] + FY[1:, :] - FY[:-1, :]
    q = cell_injection(prob, geom.hx, geom.hy).reshape(ny, nx)
    scale = max(np.abs(FX).max(), np.abs(FY).max(), 1e-300)
    return float(np.abs(net - q).max() / scale)


def _boundary_fluxes(geom, prob, kappa, p, FX, FY, GY=None):
    """Fill the physical boundary faces of +x/+y flux arrays from pressure p
    (with the gravity part GY of the y-faces)."""
    P = p.reshape(geom.ny, geom.nx)
    for side, cells, t, flen, v in _bc_faces(geom, prob, kappa):
        if prob.bc_kind[side] == DIRICHLET:
            out = t * (p[cells] - v)
        else:
            out = neumann_outflow(v, flen)
        if side == W:
            FX[:, 0] = -out
        elif side == E:
            FX[:, -1] = out
        elif side == S:
            FY[0, :] = -out
        else:
            FY[-1, :] = out
    if GY is not None:
        FY[0, :] += GY[0, :]
        FY[-1, :] += GY[-1, :]
    del P


def solve_mrcm(prob, lam=None, local_solver="superlu", interface_solver="superlu",
               ir_steps=3, stitch=True, timings=None, rho=None):
    """Run the MRCM on ``prob`` with total mobility ``lam`` (default 1) and,
    when ``prob.gravity`` is not zero, the per-cell lambda_g / lambda ``rho``
    (section 5.5: the same matrices, gravity terms in the data).

    ``timings``: an optional dict that receives the wall time in seconds of
    each phase (local, interface, compose, stitch); it changes nothing in
    the computation."""
    import time
    clock = [time.perf_counter()]

    def lap(name):
        if timings is not None:
            now = time.perf_counter()
            timings[name] = timings.get(name, 0.0) + now - clock[0]
            clock[0] = now

    geom = Geometry(prob)
    nx, ny, mx, my = geom.nx, geom.ny, geom.mx, geom.my
    lam = np.ones(nx * ny) if lam is None else np.asarray(lam, dtype=np.float64)
    kappa = prob.perm * lam
    spaces = interface_spaces(geom, prob)
    alpha = interface_alpha(geom, prob)
    n_p, n_u, off, sub_dofs, col_off, R = _dof_layout(geom, spaces)
    n_dof = int(off[-1])
    rho = None if rho is None else np.asarray(rho, dtype=np.float64)
    GY = gravity_face_fluxes(prob, kappa, rho)
    recs = _side_records(geom, prob, kappa, alpha, rho)

    # local problems, all subdomains at once (they are uncoupled)
    robin = [(r["cells"], r["TR"]) for per in recs for r in per]
    A, rhs0, (Tx, Ty, tx, ty, same_x, same_y), A_ext = local_operator(geom, prob, kappa, robin,
                                                                    extended=True, GY=GY)
    B = np.zeros((geom.n_cells, R))
    B[:, 0] = rhs0
    for per in recs:        # gravity through the Robin faces: particular solution's data
        for rec in per:
            np.add.at(B[:, 0], rec["cells"], -rec["G"])
    for itf, per in zip(geom.interfaces, recs):
        ps, us = spaces[itf.index]
        for rec in per:
            c0 = col_off[rec["sub"], rec["side"]]
            G = _interface_data(itf, rec, ps, us, c0)
            B[rec["cells"], c0:c0 + G.shape[1]] += rec["TR"][:, None] * G
    X = _local_solve(A, B, geom, local_solver, A_ext)

    # traces and the per-subdomain blocks of the interface system
    blocks = [np.zeros((len(d), R)) for d in sub_dofs]
    for itf, per in zip(geom.interfaces, recs):
        ps, us = spaces[itf.index]
        nP = ps.shape[0]
        for rec in per:
            sd = rec["sub"]
            c0 = col_off[sd, rec["side"]]
            Gfull = np.zeros((itf.faces.size, R))
            G = _interface_data(itf, rec, ps, us, c0)
            Gfull[:, c0:c0 + G.shape[1]] = G
            F = rec["TR"][:, None] * (X[rec["cells"]] - Gfull)
            F[:, 0] += rec["G"]
            pf = Gfull + (rec["beta"] / itf.flen)[:, None] * F
            r0 = c0 - 1
            blocks[sd][r0:r0 + nP] += ps @ F
            blocks[sd][r0 + nP:r0 + G.shape[1]] += rec["sigma"] * itf.flen * (us @ pf)

    lap("local")
    # interface system, natural form
    rows, cols, vals = [], [], []
    b = np.zeros(n_dof)
    for sd, dofs in enumerate(sub_dofs):
        if dofs.size == 0:
            continue
        blk = blocks[sd]
        rr, cc = np.meshgrid(dofs, dofs, indexing="ij")
        rows.append(rr.ravel())
        cols.append(cc.ravel())
        vals.append(blk[:, 1:1 + dofs.size].ravel())
        np.add.at(b, dofs, -blk[:, 0])
    if n_dof:
        M = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(n_dof, n_dof))
    else:
        M = sp.csr_matrix((0, 0))
    pure_neumann = not prob.has_dirichlet()
    M_solve, b_solve = M, b.copy()
    if pure_neumann and n_dof:
        # gauge: the first pressure dof of interface 0 is fixed to zero in
        # place of its (dependent) flux-continuity equation
        M_solve = M.tolil()
        M_solve[0, :] = 0.0
        M_solve[0, 0] = 1.0
        M_solve = M_solve.tocsr()
        b_solve[0] = 0.0
    c = _interface_solve(M_solve, b_solve, interface_solver, ir_steps)
    lap("interface")

    # composition: p = X [1; c] per subdomain
    Cmat = np.zeros((geom.n_sub, R))
    Cmat[:, 0] = 1.0
    for sd, dofs in enumerate(sub_dofs):
        Cmat[sd, 1:1 + dofs.size] = c[dofs]
    p = np.einsum("ck,ck->c", X, Cmat[geom.cell_sub])

    # multiscale fluxes: interior of subdomains, physical boundary, and the
    # two one-sided Robin fluxes on the skeleton
    P = p.reshape(ny, nx)
    FX = np.zeros((ny, nx + 1))
    FY = np.zeros((ny + 1, nx))
    FX[:, 1:-1] = np.where(same_x[None, :], Tx * (P[:, :-1] - P[:, 1:]), 0.0)
    FY[1:-1, :] = np.where(same_y[:, None], Ty * (P[:-1, :] - P[1:, :]) + GY[1:-1, :], 0.0)
    _boundary_fluxes(geom, prob, kappa, p, FX, FY, GY)
    side_flux = []
    FXf, FYf = FX.reshape(-1), FY.reshape(-1)
    for itf, per in zip(geom.interfaces, recs):
        ps, us = spaces[itf.index]
        nP = ps.shape[0]
        ce = c[off[itf.index]:off[itf.index + 1]]
        PH = ps.T @ ce[:nP]
        UH = us.T @ ce[nP:]
        Fs = []
        for rec in per:
            g = PH - rec["beta"] * rec["sigma"] * UH
            Fs.append(rec["TR"] * (p[rec["cells"]] - g) + rec["G"])
        side_flux.append((Fs[0], Fs[1]))
        avg = 0.5 * (Fs[0] - Fs[1])
        if itf.vertical:
            FXf[itf.faces] = avg
        else:
            FYf[itf.faces] = avg
    Fx_raw, Fy_raw = FXf.copy(), FYf.copy()
    imb_raw = flux_imbalance(geom, prob, Fx_raw, Fy_raw)

    if pure_neumann:
        p = p - p.mean()

    lap("compose")
    # stitch: Neumann re-solve per subdomain with the averaged skeleton flux
    p_st = np.full_like(p, np.nan)
    Fx, Fy = Fx_raw.copy(), Fy_raw.copy()
    if stitch and geom.n_iface:
        AN, rhsN, _ = local_operator(geom, prob, kappa, None, GY=GY)
        rhsN = rhsN.copy()
        for itf, per in zip(geom.interfaces, recs):
            avg = 0.5 * (side_flux[itf.index][0] - side_flux[itf.index][1])
            np.add.at(rhsN, per[0]["cells"], -avg)   # outflow of lo is +avg
            np.add.at(rhsN, per[1]["cells"], avg)    # outflow of hi is -avg
        AN = AN.tolil()
        diag = AN.diagonal()
        pins = []
        shift = np.zeros(geom.n_cells, dtype=np.longdouble)
        defect_max = 0.0
        for sd in range(geom.n_sub):
            I, J = sd % geom.SX, sd // geom.SX
            touches_dirichlet = ((I == 0 and prob.bc_kind[W] == DIRICHLET)
                                 or (I == geom.SX - 1 and prob.bc_kind[E] == DIRICHLET)
                                 or (J == 0 and prob.bc_kind[S] == DIRICHLET)
                                 or (J == geom.SY - 1 and prob.bc_kind[N] == DIRICHLET))
            if not touches_dirichlet:
                # A Neumann problem has a solution only if its data sum to
                # zero.  The averaged skeleton fluxes meet this to the
                # rounding of the composed solution and of the interface
                # solve; the defect is removed evenly from the subdomain's
                # cells (a uniform source correction at rounding level)
                # instead of being left to the pinned cell.
                li, lj = np.meshgrid(np.arange(mx), np.arange(my))
                cells = ((J * my + lj) * nx + I * mx + li).reshape(-1)
                defect = np.sum(rhsN[cells].astype(np.longdouble)) / cells.size
                rhsN[cells] = (rhsN[cells] - defect).astype(np.float64)
                shift[cells] = defect
                defect_max = max(defect_max, float(abs(defect)) * cells.size)
                c0 = (J * my) * nx + I * mx
                Tpin = diag[c0]
                AN[c0, c0] = diag[c0] + Tpin
                rhsN[c0] += Tpin * p[c0]
                pins.append((c0, Tpin, p[c0]))
        AN = AN.tocsc()
        ld = np.longdouble
        inj = (cell_injection(prob, geom.hx, geom.hy).astype(ld) - shift).reshape(ny, nx)

        def stitched_fluxes(x):
            """Face fluxes of the re-solve from pressure x (extended): the
            face laws inside subdomains and on the physical boundary, the
            averaged flux on skeleton faces."""
            PS = x.reshape(ny, nx)
            FXl = Fx_raw.reshape(ny, nx + 1).astype(ld)
            FYl = Fy_raw.reshape(ny + 1, nx).astype(ld)
            FXl[:, 1:-1] = np.where(same_x[None, :], Tx * (PS[:, :-1] - PS[:, 1:]), FXl[:, 1:-1])
            FYl[1:-1, :] = np.where(same_y[:, None], Ty * (PS[:-1, :] - PS[1:, :]) + GY[1:-1, :],
                                    FYl[1:-1, :])
            _boundary_fluxes(geom, prob, kappa, x, FXl, FYl, GY)
            return FXl, FYl

        def balance_residual(x):
            """q |V| minus the net outflow of every cell (and the pin), in
            extended precision: the residual of the re-solve written as the
            cell balances themselves, so that its solution balances the
            fluxes formed from it (a residual of the assembled matrix would
            carry the FP64 rounding of its diagonal sums, eps T |p| per
            cell)."""
            FXl, FYl = stitched_fluxes(x)
            net = FXl[:, 1:] - FXl[:, :-1] + FYl[1:, :] - FYl[:-1, :]
            r = (inj - net).reshape(-1)
            for c0, Tpin, pref in pins:
                r[c0] -= Tpin * (x[c0] - pref)
            return r

        # the stitched pressure in extended precision; the fluxes are formed
        # from it and rounded once (section 2: every cell balances)
        p_ext = _refined_extended(spla.splu(AN).solve, rhsN, balance_residual)
        p_st = p_ext.astype(np.float64)
        FXl, FYl = stitched_fluxes(p_ext)
        Fx, Fy = FXl.astype(np.float64).reshape(-1), FYl.astype(np.float64).reshape(-1)
    imb = flux_imbalance(geom, prob, Fx, Fy)
    lap("stitch")
    fscale = max(np.abs(Fx).max(), np.abs(Fy).max(), 1e-300)
    defect = defect_max / fscale if stitch and geom.n_iface else 0.0
    return MRCMResult(p=p, ux=Fx / geom.hy, uy=Fy / geom.hx, Fx=Fx, Fy=Fy,
                      Fx_raw=Fx_raw, Fy_raw=Fy_raw, side_flux=side_flux, coeffs=c,
                      blocks=blocks, sub_dofs=sub_dofs, X=X, p_stitch=p_st,
                      imbalance_raw=imb_raw, imbalance=imb, stitch_defect=defect,
                      interface_matrix=M,
                      interface_rhs=b, dof_offset=off, n_p=n_p, n_u=n_u)


def solve_mrcm_monolithic(prob, lam=None):
    """All local pressures and interface unknowns in one sparse system.

    Rows: every cell balance of every local problem (eq. (mrc1) with the
    interface data left as unknowns) and every interface equation
    (eq. (mrc2)).  Used to pin the static condensation of ``solve_mrcm``.
    Returns (p, coeffs).
    """
    geom = Geometry(prob)
    nx, ny = geom.nx, geom.ny
    n = nx * ny
    lam = np.ones(n) if lam is None else np.asarray(lam, dtype=np.float64)
    kappa = prob.perm * lam
    spaces = interface_spaces(geom, prob)
    alpha = interface_alpha(geom, prob)
    n_p, n_u, off, sub_dofs, col_off, R = _dof_layout(geom, spaces)
    n_dof = int(off[-1])
    recs = _side_records(geom, prob, kappa, alpha)
    robin = [(r["cells"], r["TR"]) for per in recs for r in per]
    A, rhs0, _ = local_operator(geom, prob, kappa, robin)
    A = A.tocoo()
    rows = [A.row]
    cols = [A.col]
    vals = [A.data]
    rhs = np.concatenate([rhs0, np.zeros(n_dof)])
    for itf, per in zip(geom.interfaces, recs):
        ps, us = spaces[itf.index]
        nP = ps.shape[0]
        d0 = off[itf.index]
        nd = off[itf.index + 1] - d0
        for rec in per:
            G = _interface_data(itf, rec, ps, us, 0)       # (m, nd)
            TR, beta = rec["TR"], rec["beta"]
            cells = rec["cells"]
            # cell rows: A p - T_R g = data  ->  -T_R G c
            for k in range(nd):
                rows.append(cells)
                cols.append(np.full(cells.size, n + d0 + k))
                vals.append(-TR * G[:, k])
            # flux-continuity rows: sum psi_l T_R (p_c - G c)
            for l in range(nP):
                rows.append(np.full(cells.size, n + d0 + l))
                cols.append(cells)
                vals.append(ps[l] * TR)
                for k in range(nd):
                    rows.append(np.array([n + d0 + l]))
                    cols.append(np.array([n + d0 + k]))
                    vals.append(np.array([-(ps[l] * TR * G[:, k]).sum()]))
            # pressure-continuity rows: sigma sum |f| phi_l p_f,
            # p_f = G c + beta T_R (p_c - G c) / |f|
            for l in range(us.shape[0]):
                row = n + d0 + nP + l
                w = rec["sigma"] * itf.flen * us[l]
                rows.append(np.full(cells.size, row))
                cols.append(cells)
                vals.append(w * beta * TR / itf.flen)
                for k in range(nd):
                    rows.append(np.array([row]))
                    cols.append(np.array([n + d0 + k]))
                    vals.append(np.array([(w * (G[:, k] - beta * TR * G[:, k] / itf.flen)).sum()]))
    Mfull = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(n + n_dof, n + n_dof))
    if not prob.has_dirichlet() and n_dof:
        Mfull = Mfull.tolil()
        Mfull[n, :] = 0.0
        Mfull[n, n] = 1.0
        Mfull = Mfull.tocsr()
        rhs[n] = 0.0
    Mfull = Mfull.tocsc()
    sol = _refined(Mfull, spla.splu(Mfull).solve, rhs)
    p = sol[:n]
    if not prob.has_dirichlet():
        p = p - p.mean()
    return p, sol[n:]
