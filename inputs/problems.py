"""Problem data for the Darcy solves: grids, fields, boundary data, workloads.

A ``Problem`` is plain data: the model of the paper's section 2 (Darcy's law
with total mobility, Dirichlet/Neumann boundary data, a source term) plus the
domain decomposition and interface-space choice of section 3.  Solvers (the
CPU oracle and the GPU library) receive the same ``Problem`` and compute from
it independently.

Conventions
-----------
* cell (i, j), i along x: flat index ``j * nx + i``;
* boundary sides are ordered W (x = 0), E (x = lx), S (y = 0), N (y = ly);
  W/E carry ``ny`` face values (bottom to top), S/N carry ``nx`` values;
* ``bc_kind[side]`` is 1 for Dirichlet (value = boundary pressure) and 0 for
  Neumann (value = outward normal velocity);
* ``source`` is q per unit area (so a cell receives q * hx * hy).
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Sequence

import numpy as np

from .fields import channelized_field, lognormal_grf

NEUMANN = 0
DIRICHLET = 1

SPACE_LINEAR = "linear"
SPACE_EDGE = "edge"      # edge-solution spaces built from local 1-D problems
SPACE_FULL = "full"      # all fine-edge indicator functions
SPACE_PHYSICS = "physics"  # channel / barrier spaces of section 3.1 (at most 4 + 4 slots)
SPACES = (SPACE_LINEAR, SPACE_EDGE, SPACE_FULL, SPACE_PHYSICS)


@dataclasses.dataclass
class Problem:
    name: str
    nx: int
    ny: int
    lx: float
    ly: float
    perm: np.ndarray                      # (nx*ny,) float64, > 0
    sub_nx: int
    sub_ny: int
    bc_kind: tuple                        # 4 ints, W E S N
    bc_value: tuple                       # 4 arrays (or None = zeros)
    source: Optional[np.ndarray] = None   # (nx*ny,) per unit area, or None
    mu_w: float = 1.0
    mu_o: float = 10.0
    space: str = SPACE_LINEAR
    p_dofs: int = 2
    u_dofs: int = 2
    alpha: float = 1.0
    alpha_per_interface: Optional[np.ndarray] = None
    # adaptive Robin parameter: (alpha on interfaces crossed by a
    # high-permeability channel, alpha elsewhere), or None
    adaptive_alpha: Optional[tuple] = None
    seed: int = 1
    steps: int = 1                        # time steps of the two-phase workload
    # gravity: the term lambda_g g grad h of Darcy's law with gravity, acting
    # along y: gravity = g dh/dy (0: no gravity); phase densities
    gravity: float = 0.0
    rho_w: float = 0.0
    rho_o: float = 0.0

    @property
    def hx(self) -> float:
        return self.lx / self.nx

    @property
    def hy(self) -> float:
        return self.ly / self.ny

    @property
    def n_sub_x(self) -> int:
        return self.nx // self.sub_nx

    @property
    def n_sub_y(self) -> int:
        return self.ny // self.sub_ny

    @property
    def n_sub(self) -> int:
        return self.n_sub_x * self.n_sub_y

    def bc_array(self, side: int) -> np.ndarray:
        n = self.ny if side < 2 else self.nx
        v = self.bc_value[side]
        if v is None:
            return np.zeros(n)
        v = np.asarray(v, dtype=np.float64)
        if v.shape != (n,):
            raise ValueError("boundary data of side %d must have %d values" % (side, n))
        return v

    def has_dirichlet(self) -> bool:
        return any(k == DIRICHLET for k in self.bc_kind)

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


def _left_right_bc(nx: int, ny: int, p_left: float = 1.0, p_right: float = 0.0):
    """p = p_left on x = 0, p = p_right on x = lx, no flow on y = 0, ly."""
    return ((DIRICHLET, DIRICHLET, NEUMANN, NEUMANN),
            (np.full(ny, p_left), np.full(ny, p_right), None, None))


def quarter_five_spot_source(nx: int, ny: int, lx: float, ly: float, rate: float = 1.0):
    """Injector in the bottom-left cell, producer in the top-right cell.

    ``rate`` is the injected volume per unit time (one pore volume per unit
    time for rate = lx * ly with unit porosity); stored per unit area.
    """
    q = np.zeros(nx * ny)
    area = (lx / nx) * (ly / ny)
    q[0] = rate / area
    q[nx * ny - 1] = -rate / area
    return q


# Workloads.  Sizes, fields and boundary data follow the five configurations
# of the benchmark: a 64^2 single-phase case, a 256^2 channelized
# quarter-five-spot case, the 1024^2 log-normal two-phase case, a 2048x1024
# channelized case with 32^2 subdomains and edge-solution spaces, and the
# 1024^2 surrogate case.
WORKLOADS = {
    "gauss64": dict(nx=64, ny=64, lx=1.0, ly=1.0, sub=16, field="grf",
                    variance=4.0, corr_len=0.1, bc="lr", space=SPACE_LINEAR, steps=1),
    "channel256_q5": dict(nx=256, ny=256, lx=1.0, ly=1.0, sub=16, field="channel",
                          contrast=1e4, bc="q5", space=SPACE_LINEAR, steps=20),
    "gauss1024": dict(nx=1024, ny=1024, lx=1.0, ly=1.0, sub=16, field="grf",
                      variance=6.0, corr_len=0.05, bc="lr", space=SPACE_LINEAR, steps=10),
    "channel2048x1024": dict(nx=2048, ny=1024, lx=2.0, ly=1.0, sub=32, field="channel",
                             contrast=1e6, bc="lr", space=SPACE_EDGE, steps=5),
}


def make_problem(workload: str, seed: int = 1, **over) -> Problem:
    """Build one of the named workloads (``WORKLOADS``), optionally resized.

    Keyword overrides: nx, ny, lx, ly, sub (subdomain edge in cells), space,
    alpha, variance, corr_len, contrast.
    """
    spec = dict(WORKLOADS[workload])
    spec.update(over)
    nx, ny, lx, ly = spec["nx"], spec["ny"], spec["lx"], spec["ly"]
    if spec["field"] == "grf":
        perm = lognormal_grf(nx, ny, lx, ly, spec["variance"], spec["corr_len"], seed)
    else:
        perm = channelized_field(nx, ny, lx, ly, 1.0, spec["contrast"], seed)
    source = None
    if spec["bc"] == "lr":
        kind, val = _left_right_bc(nx, ny)
    else:
        kind = (NEUMANN, NEUMANN, NEUMANN, NEUMANN)
        val = (None, None, None, None)
        source = quarter_five_spot_source(nx, ny, lx, ly, rate=lx * ly)
    space = spec.get("space", SPACE_LINEAR)
    sub = spec["sub"]
    if space == SPACE_FULL:
        pd = ud = sub
    elif space == SPACE_PHYSICS:
        pd = ud = 4          # slots: up to 2 channels (4 pressure) and 1 barrier (3 flux)
    else:
        pd = ud = 2
    return Problem(name=workload, nx=nx, ny=ny, lx=lx, ly=ly, perm=perm,
                   sub_nx=sub, sub_ny=sub, bc_kind=kind, bc_value=val,
                   source=source, space=space, p_dofs=pd, u_dofs=ud,
                   alpha=float(spec.get("alpha", 1.0)), seed=seed,
                   steps=int(spec.get("steps", 1)))


def synthetic_saturation(prob: Problem, step: int, n_steps: Optional[int] = None) -> np.ndarray:
    """A water-saturation snapshot with the shape of a displacement front.

    Stand-in for the saturation of time step ``step`` of a two-phase run:
    water (s = 1) enters from the inflow side and a front with a trailing
    rarefaction, s falling from 1 to 0.4 and then to 0, advances
    by an equal distance per step.  The front runs ahead in high-permeability
    rows (or radially from the injector for source-driven problems), so the
    mobility field has the fingered structure of a heterogeneous
    displacement.  Values lie in [0, 1].
    """
    n_steps = n_steps or max(prob.steps, 1)
    nx, ny = prob.nx, prob.ny
    hx, hy = prob.hx, prob.hy
    xc = (np.arange(nx) + 0.5) * hx
    yc = (np.arange(ny) + 0.5) * hy
    X, Y = np.meshgrid(xc, yc)
    lnk = np.log(prob.perm.reshape(ny, nx))
    frac = (step + 1.0) / (n_steps + 1.0)
    if prob.source is not None:
        dist = np.sqrt(X ** 2 + Y ** 2)
        reach = np.sqrt(prob.lx ** 2 + prob.ly ** 2)
        z = (lnk - lnk.mean()) / (lnk.std() + 1e-300)
        front = frac * reach * (1.0 + 0.15 * np.tanh(z))
    else:
        dist = X
        row = lnk.mean(axis=1)
        z = (row - row.mean()) / (row.std() + 1e-300)
        front = (frac * prob.lx * (1.0 + 0.3 * np.tanh(z)))[:, None] * np.ones((1, nx))
    t = np.clip(dist / np.maximum(front, 1e-12), 0.0, None)
    s = np.where(t < 1.0, 1.0 - 0.6 * np.sqrt(t), 0.0)
    return np.clip(s, 0.0, 1.0).reshape(-1)
