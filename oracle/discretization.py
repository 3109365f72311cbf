"""Geometry, face laws and interface spaces of the oracle (CPU, FP64).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Discretisation (section 2 asks for a mixed formulation of eq. (Darcy); on an
orthogonal, uniformly spaced grid the lowest-order Raviart-Thomas space with
trapezoidal quadrature is the cell-centred two-point flux scheme used here):

* unknowns are one pressure per cell and one flux per face;
* a face flux is F = integral of u.n over the face (face length times the
  normal velocity), positive out of the cell it is written for;
* half-cell transmissibility t = kappa |f| / d with d the centre-to-face
  distance; two half cells in series give the harmonic transmissibility
  1 / (1/t_c + 1/t_d);
* Dirichlet face: F = t_c (p_c - p_b); Neumann face: F = u_b |f|;
* Robin face on the skeleton (eq. (mrc1), last line, with eq. (beta)):
  beta = alpha H / kappa_c and p_f = g + beta F / |f| with
  g = P_H - beta U_H (n . n_i).  Eliminating p_f from
  F = t_c (p_c - p_f) gives F = T_R (p_c - g), T_R = |f| kappa_c / (d + alpha H).

Index conventions (all flat, row-major):
cell (i, j) -> j*nx + i; x-face at x = i*hx in row j -> j*(nx+1) + i;
y-face at y = j*hy in column i -> j*nx + i; subdomain (I, J) -> J*SX + I.
Interfaces: vertical ones first, (I, J) between subdomains (I, J) and
(I+1, J) -> J*(SX-1) + I; then horizontal ones between (I, J) and (I, J+1)
-> nV + J*SX + I.  The fixed skeleton normal points +x on vertical and +y on
horizontal interfaces, i.e. out of the subdomain with the smaller index
(section 3), so sigma = n . n_i is +1 on the lower-index side and -1 on the
other.  Dofs of interface e are [P_0 .. P_{nP-1}, U_0 .. U_{nU-1}].
"""
from __future__ import annotations

import dataclasses

import numpy as np

W, E, S, N = 0, 1, 2, 3
NEUMANN, DIRICHLET = 0, 1


def total_mobility(s, mu_w, mu_o):
    """lambda(s) = k_rw/mu_w + k_ro/mu_o (eq. fluxos1) with the quadratic
    relative permeabilities k_rw = s^2, k_ro = (1-s)^2 of section 5."""
    s = np.asarray(s, dtype=np.float64)
    return s * s / mu_w + (1.0 - s) * (1.0 - s) / mu_o


def fractional_flow(s, mu_w, mu_o):
    """f(s) = lambda_w / lambda (eq. fluxos2) = M s^2 / (M s^2 + (1-s)^2), M = mu_o/mu_w."""
    s = np.asarray(s, dtype=np.float64)
    lw = s * s / mu_w
    lo = (1.0 - s) ** 2 / mu_o
    return lw / (lw + lo)


def gravity_density(s, mu_w, mu_o, rho_w, rho_o):
    """lambda_g / lambda: the gravitational mobility of eq. (fluxos1_wg),
    lambda_g = lambda_w rho_w + lambda_o rho_o, over the total mobility
    (quadratic relative permeabilities of section 5), i.e. the
    mobility-weighted density of the two phases."""
    s = np.asarray(s, dtype=np.float64)
    lw = s * s / mu_w
    lo = (1.0 - s) * (1.0 - s) / mu_o
    return (lw * rho_w + lo * rho_o) / (lw + lo)


def gravity_face_fluxes(prob, kappa, rho):
    """The gravity part of the +y face fluxes, shape (ny + 1, nx).

    Darcy's law with gravity (section 5.5, eq. (Darcy_wg)) is
    u = -kappa (grad p - rho g grad h) with kappa = lambda K and
    rho = lambda_g / lambda per cell; gravity acts along y with
    gamma = g dh/dy (``prob.gravity``).  Reading (the paper gives no
    discretisation of this term): on a half cell the flux is
    t_c (p_c - p_f) + t_c rho_c gamma d in the +y direction (t_c = kappa_c
    |f| / d), and the face pressure is eliminated between the two half
    cells as in the two-point law, which gives
    F = T (p_below - p_above) + T gamma (h/2) (rho_below + rho_above) on an
    interior face and t_c gamma (h/2) rho_c on a Dirichlet boundary face.
    Neumann boundary faces carry the prescribed total flux: zero here."""
    nx, ny = prob.nx, prob.ny
    GY = np.zeros((ny + 1, nx))
    if prob.gravity == 0.0 or rho is None:
        return GY
    hx, hy = prob.lx / nx, prob.ly / ny
    K = np.asarray(kappa, dtype=np.float64).reshape(ny, nx)
    R = np.asarray(rho, dtype=np.float64).reshape(ny, nx)
    t = K * hx / (0.5 * hy)
    g = prob.gravity
    GY[1:-1, :] = harmonic(t[:-1, :], t[1:, :]) * g * (0.5 * hy) * (R[:-1, :] + R[1:, :])
    if prob.bc_kind[S] == DIRICHLET:
        GY[0, :] = t[0, :] * g * (0.5 * hy) * R[0, :]
    if prob.bc_kind[N] == DIRICHLET:
        GY[-1, :] = t[-1, :] * g * (0.5 * hy) * R[-1, :]
    return GY


def cell_injection(prob, hx, hy):
    """Volume injected per unit time into every cell: q |V| (eq. (Darcy),
    div u = q; q > 0 is a source such as an injection well)."""
    if prob.source is None:
        return np.zeros(prob.nx * prob.ny)
    return prob.source * hx * hy


def neumann_outflow(u_b, flen):
    """Flux leaving the domain through a Neumann face: the prescribed outward
    normal velocity u_b times the face length (u . n = u_b, section 2)."""
    return u_b * flen


def harmonic(a, b):
    """Two conductances in series: 1 / (1/a + 1/b)."""
    return 1.0 / (1.0 / a + 1.0 / b)


def harmonic_mean(a, b):
    """2 a b / (a + b)."""
    return 2.0 * harmonic(a, b)


@dataclasses.dataclass
class Interface:
    """One interface Gamma_ij: a subdomain edge between two cross-points."""
    index: int
    vertical: bool
    lo: int            # subdomain with the smaller index (sigma = +1)
    hi: int            # the other subdomain (sigma = -1)
    lo_side: int       # side of `lo` the interface lies on (E or N)
    hi_side: int       # side of `hi` the interface lies on (W or S)
    faces: np.ndarray  # global x-face (vertical) or y-face (horizontal) ids
    lo_cells: np.ndarray
    hi_cells: np.ndarray
    flen: float        # |f|, the fine-face length
    dist: float        # centre-to-face distance d
    H: float           # interface length (the H of eq. (beta))
    xi: np.ndarray     # normalised face-midpoint coordinate (x - a)/(b - a)


class Geometry:
    """Grid, decomposition and interface table of a ``Problem``."""

    def __init__(self, prob):
        self.prob = prob
        nx, ny = prob.nx, prob.ny
        mx, my = prob.sub_nx, prob.sub_ny
        if nx % mx or ny % my:
            raise ValueError("grid must be divisible by the subdomain size")
        self.nx, self.ny, self.mx, self.my = nx, ny, mx, my
        self.hx, self.hy = prob.lx / nx, prob.ly / ny
        self.SX, self.SY = nx // mx, ny // my
        self.n_cells = nx * ny
        self.n_sub = self.SX * self.SY
        ii, jj = np.meshgrid(np.arange(nx), np.arange(ny))
        self.cell_i = ii.reshape(-1)
        self.cell_j = jj.reshape(-1)
        self.cell_sub = (self.cell_j // my) * self.SX + (self.cell_i // mx)
        self.nV = (self.SX - 1) * self.SY
        self.nH = self.SX * (self.SY - 1)
        self.interfaces = []
        for J in range(self.SY):
            for I in range(self.SX - 1):
                i = (I + 1) * mx
                js = J * my + np.arange(my)
                self.interfaces.append(Interface(
                    index=len(self.interfaces), vertical=True,
                    lo=J * self.SX + I, hi=J * self.SX + I + 1, lo_side=E, hi_side=W,
                    faces=js * (nx + 1) + i, lo_cells=js * nx + i - 1, hi_cells=js * nx + i,
                    flen=self.hy, dist=0.5 * self.hx, H=my * self.hy,
                    xi=(np.arange(my) + 0.5) / my))
        for J in range(self.SY - 1):
            for I in range(self.SX):
                j = (J + 1) * my
                iis = I * mx + np.arange(mx)
                self.interfaces.append(Interface(
                    index=len(self.interfaces), vertical=False,
                    lo=J * self.SX + I, hi=(J + 1) * self.SX + I, lo_side=N, hi_side=S,
                    faces=j * nx + iis, lo_cells=(j - 1) * nx + iis, hi_cells=j * nx + iis,
                    flen=self.hx, dist=0.5 * self.hy, H=mx * self.hx,
                    xi=(np.arange(mx) + 0.5) / mx))
        self.n_iface = len(self.interfaces)
        # interface on each side of each subdomain (-1: physical boundary)
        self.sub_iface = -np.ones((self.n_sub, 4), dtype=np.int64)
        for itf in self.interfaces:
            self.sub_iface[itf.lo, itf.lo_side] = itf.index
            self.sub_iface[itf.hi, itf.hi_side] = itf.index

    def sub_of(self, I, J):
        return J * self.SX + I


# ----------------------------------------------------------------------------
# Interface spaces (section 3.1).  Every space is a list of per-fine-face
# vectors on each interface: the piecewise-constant space on skeleton edges
# defined in section 3 and its subspaces.
# ----------------------------------------------------------------------------

def linear_space(xi):
    """Nodal linear polynomials (b - x)/(b - a), (x - a)/(b - a) at the face
    midpoints; these are the pressure functions of eqs. (new_basis1)-(new_basis3)
    with no channel (N_high = 0) and span the linear flux space as well."""
    return np.stack([1.0 - xi, xi])


def full_space(m):
    """All fine-edge indicator functions: the whole piecewise-constant space."""
    return np.eye(m)


def edge_solution_space(k_lo, k_hi):
    """Non-polynomial two-function spaces from a 1-D edge problem.

    The paper does not define these spaces: section 3.1 defines the
    physics-based spaces of eqs. (new_basis1)-(new_basis6), built from the
    channel structure of the edge.  What follows is the reading taken for a
    space of "two pressure and two flux functions built from local edge
    solutions"; its only pins are the reductions below and the exact
    solution of the edge problem.

    t_j is the harmonic mean of the permeabilities across fine face j.
    psi solves the 1-D two-point problem along the edge with conductances
    harm(t_j, t_{j+1}) between neighbouring faces, 2 t_0 and 2 t_{m-1} to the
    interface ends, psi = 1 at a and psi = 0 at b.  Pressure space:
    {psi, 1 - psi}; flux space: {t / mean t, t (psi - mean psi) / mean t}.
    With uniform permeability both reduce to the linear space.

    The 1-D problem is a chain of conductances in series, so its solution is
    the fraction of the total resistance that lies between face j and the
    b end; 1 - psi is the fraction on the a side, summed directly, so both
    functions keep their relative accuracy where they are small (high
    contrast along the edge).
    """
    t = harmonic_mean(np.asarray(k_lo, float), np.asarray(k_hi, float))
    m = t.size
    r_in = 1.0 / harmonic_mean(t[:-1], t[1:]) if m > 1 else np.zeros(0)
    r_a, r_b = 1.0 / (2.0 * t[0]), 1.0 / (2.0 * t[-1])
    # resistance from the a end to face j, and from face j to the b end
    up = r_a + np.concatenate([[0.0], np.cumsum(r_in)])
    down = r_b + np.concatenate([np.cumsum(r_in[::-1])[::-1], [0.0]])
    total = r_a + r_in.sum() + r_b
    psi = down / total
    pspace = np.stack([psi, up / total])
    tm = t.mean()
    uspace = np.stack([t / tm, t * (psi - psi.mean()) / tm])
    return pspace, uspace


# Physics-based spaces (section 3.1, eqs. (new_basis1)-(new_basis6)) and the
# adaptive Robin parameter.  Readings (the paper gives the functions for
# given channel and barrier supports, not how the supports are found):
# * t_j, the harmonic mean of the permeabilities across fine face j, is
#   compared with the median of t over the interface: faces with
#   t_j >= 10 median are high-permeability, faces with t_j <= median / 10
#   low-permeability; maximal runs of such faces are the channels and the
#   barriers, face j covering [j/m, (j+1)/m] of the normalised interface;
# * at most NH_MAX channels and NL_MAX barriers are kept (the widest, the
#   left one first on ties), the others count as background;
# * a space whose kind of structure is absent is the linear space (the
#   paper's rule for interfaces without structures, applied per space);
# * functions with no support (a structure touching the interface end) are
#   left out, so a space has at most 2 + NH_MAX pressure and 1 + 2 NL_MAX
#   flux functions;
# * alpha: alpha_channel on interfaces crossed by a kept channel,
#   alpha_other elsewhere (section 5.5 uses 1e-2 and 1e2).
NH_MAX, NL_MAX = 2, 1
STRUCTURE_RATIO = 10.0


def face_conductance(k_lo, k_hi):
    """t_j: the harmonic mean of the permeabilities on both sides of face j."""
    return harmonic_mean(np.asarray(k_lo, float), np.asarray(k_hi, float))


def _runs(mask):
    """Maximal runs of True in mask as (first, last) face indices."""
    runs, j, m = [], 0, mask.size
    while j < m:
        if mask[j]:
            k = j
            while k + 1 < m and mask[k + 1]:
                k += 1
            runs.append((j, k))
            j = k + 1
        else:
            j += 1
    return runs


def _keep_widest(runs, n):
    order = sorted(range(len(runs)), key=lambda r: (-(runs[r][1] - runs[r][0]), runs[r][0]))
    return sorted(runs[r] for r in order[:n])


def classify_interface(t):
    """(channels, barriers): kept runs of high and low faces of one interface."""
    t = np.asarray(t, float)
    med = float(np.median(t))
    high = _runs(t >= STRUCTURE_RATIO * med)
    low = _runs(t <= med / STRUCTURE_RATIO)
    return _keep_widest(high, NH_MAX), _keep_widest(low, NL_MAX)


def physics_pressure_space(channels, m):
    """Eqs. (new_basis1)-(new_basis3) at the face midpoints, for channels
    given as face runs; the functions with no support are left out."""
    x = (np.arange(m) + 0.5) / m
    a = [j0 / m for j0, _ in channels]
    b = [(j1 + 1) / m for _, j1 in channels]
    n = len(channels)
    funcs = []
    # psi_0: falls from 1 at the interface start to 0 where channel 1 begins
    if a[0] > 0.0:
        funcs.append(np.where(x < a[0], (a[0] - x) / a[0], 0.0))
    for k in range(n):
        lo = 0.0 if k == 0 else b[k - 1]          # b_0 = a
        hi = 1.0 if k == n - 1 else a[k + 1]      # a_{N+1} = b
        f = np.zeros(m)
        up = (x > lo) & (x < a[k])
        f[up] = (x[up] - lo) / (a[k] - lo)
        f[(x >= a[k]) & (x <= b[k])] = 1.0
        down = (x > b[k]) & (x < hi)
        f[down] = (hi - x[down]) / (hi - b[k])
        funcs.append(f)
    # psi_{N+1}: rises from 0 where the last channel ends to 1 at the end
    if b[-1] < 1.0:
        funcs.append(np.where(x > b[-1], (x - b[-1]) / (1.0 - b[-1]), 0.0))
    return np.stack(funcs)


def physics_flux_space(barriers, m):
    """Eqs. (new_basis4)-(new_basis6): indicators of the segments before,
    on and after each barrier; the empty ones are left out."""
    x = (np.arange(m) + 0.5) / m
    edges = [0.0]
    for j0, j1 in barriers:
        edges += [j0 / m, (j1 + 1) / m]
    edges.append(1.0)
    funcs = []
    for lo, hi in zip(edges[:-1], edges[1:]):
        if hi > lo:
            funcs.append(((x > lo) & (x < hi)).astype(np.float64))
    return np.stack(funcs)


def physics_space(t):
    """(pressure functions, flux functions) of one interface from t."""
    m = np.asarray(t).size
    channels, barriers = classify_interface(t)
    xi = (np.arange(m) + 0.5) / m
    ps = physics_pressure_space(channels, m) if channels else linear_space(xi)
    us = physics_flux_space(barriers, m) if barriers else linear_space(xi)
    return ps, us


def interface_spaces(geom, prob):
    """Per interface: (psi [nP, m], phi [nU, m]) evaluated on its fine faces."""
    out = []
    perm = prob.perm
    for itf in geom.interfaces:
        m = itf.faces.size
        if prob.space == "linear":
            if prob.p_dofs != 2 or prob.u_dofs != 2:
                raise ValueError("linear spaces have 2 pressure and 2 flux functions")
            ps = linear_space(itf.xi)
            us = linear_space(itf.xi)
        elif prob.space == "full":
            if prob.p_dofs != m or prob.u_dofs != m:
                raise ValueError("full spaces have one function per fine face")
            ps = full_space(m)
            us = full_space(m)
        elif prob.space == "edge":
            if prob.p_dofs != 2 or prob.u_dofs != 2:
                raise ValueError("edge-solution spaces have 2 + 2 functions")
            ps, us = edge_solution_space(perm[itf.lo_cells], perm[itf.hi_cells])
        elif prob.space == "physics":
            ps, us = physics_space(face_conductance(perm[itf.lo_cells], perm[itf.hi_cells]))
        elif prob.space == "custom":
            ps, us = prob.custom_space(itf)
        else:
            raise ValueError("unknown interface space %r" % prob.space)
        out.append((np.asarray(ps, float), np.asarray(us, float)))
    return out


def interface_alpha(geom, prob):
    if prob.adaptive_alpha is not None:
        a_ch, a_other = prob.adaptive_alpha
        out = np.empty(geom.n_iface)
        for itf in geom.interfaces:
            channels, _ = classify_interface(face_conductance(prob.perm[itf.lo_cells],
                                                              prob.perm[itf.hi_cells]))
            out[itf.index] = a_ch if channels else a_other
        return out
    if prob.alpha_per_interface is not None:
        a = np.asarray(prob.alpha_per_interface, dtype=np.float64)
        if a.shape != (geom.n_iface,):
            raise ValueError("alpha_per_interface must have one value per interface")
        return a
    return np.full(geom.n_iface, float(prob.alpha))
