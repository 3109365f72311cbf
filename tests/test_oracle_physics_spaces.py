"""Pins of the physics-based interface spaces and the adaptive Robin
parameter (section 3.1, eqs. (new_basis1)-(new_basis6)) in the oracle (CPU
only).

What the equations fix, checked on random channel and barrier layouts:
* the pressure functions are a partition of unity; psi_k is 1 on channel k
  and 0 on every other channel; on each segment between structures the
  functions are linear in x (zero second differences), falling from 1 to 0
  across the segment; psi_0 and psi_{N+1} exist only when the first channel
  does not start, or the last does not end, at the interface end;
* the flux functions are the indicators of the segments before, on and
  after each barrier: disjoint, a partition of unity, 1 + 2 N_low of them
  when no structure touches an end;
* with no structure of a kind the space is the linear one (bitwise);
* the classification finds the runs of faces a decade above or below the
  interface's median conductance;
* the adaptive alpha follows the classification;
* an MRCM solve with these spaces is exact where the exact traces lie in
  them (barrier bands crossing the interfaces, where the linear spaces are
  not exact), and balances every cell.
"""
import numpy as np
import pytest

import inputs
from inputs import Problem
from inputs.problems import DIRICHLET, NEUMANN
from oracle import discretization as od
from oracle.discretization import (Geometry, classify_interface, interface_alpha, linear_space,
                                   physics_flux_space, physics_pressure_space, physics_space)
from oracle.fine import solve_fine
from oracle.mrcm import flux_imbalance, solve_mrcm


def random_runs(rng, m, n):
    """n disjoint runs of faces separated by at least one face."""
    while True:
        starts = np.sort(rng.choice(m, size=2 * n, replace=False))
        runs = [(int(starts[2 * k]), int(starts[2 * k + 1])) for k in range(n)]
        if all(runs[k][1] + 1 < runs[k + 1][0] for k in range(n - 1)):
            return runs


def second_differences_vanish(f, x):
    if f.size < 3:
        return True
    d = np.diff(f) / np.diff(x)
    return np.allclose(np.diff(d), 0.0, atol=1e-12)


@pytest.mark.parametrize("seed", range(12))
def test_pressure_functions(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.choice([16, 32]))
    n = int(rng.integers(1, 3))
    ch = random_runs(rng, m, n)
    ps = physics_pressure_space(ch, m)
    x = (np.arange(m) + 0.5) / m
    # partition of unity
    assert np.allclose(ps.sum(axis=0), 1.0, atol=1e-15)
    assert ps.min() >= 0.0 and ps.max() <= 1.0
    # number of functions: N, plus psi_0 / psi_{N+1} unless a channel touches the end
    has0, has_last = ch[0][0] > 0, ch[-1][1] < m - 1
    assert ps.shape[0] == n + int(has0) + int(has_last)
    plateau = ps[int(has0):int(has0) + n]
    for k, (j0, j1) in enumerate(ch):
        assert np.all(plateau[k, j0:j1 + 1] == 1.0)
        for q, (i0, i1) in enumerate(ch):
            if q != k:
                assert np.all(plateau[k, i0:i1 + 1] == 0.0)
    # linear on every segment between structures (and between a structure
    # and an end)
    bounds = [0] + [b for r in ch for b in (r[0], r[1] + 1)] + [m]
    for lo, hi in zip(bounds[0::2], bounds[1::2]):
        seg = np.arange(lo, hi)
        for f in ps:
            assert second_differences_vanish(f[seg], x[seg])


@pytest.mark.parametrize("seed", range(8))
def test_flux_functions(seed):
    rng = np.random.default_rng(100 + seed)
    m = int(rng.choice([16, 32]))
    bar = random_runs(rng, m, 1)
    us = physics_flux_space(bar, m)
    assert set(np.unique(us)) <= {0.0, 1.0}
    assert np.array_equal(us.sum(axis=0), np.ones(m))
    j0, j1 = bar[0]
    n_expected = 1 + int(j0 > 0) + int(j1 < m - 1)
    assert us.shape[0] == n_expected
    on = [f for f in us if np.all(f[j0:j1 + 1] == 1.0)]
    assert len(on) == 1 and on[0].sum() == j1 - j0 + 1


def test_no_structure_gives_the_linear_space():
    for m in (8, 16, 32):
        t = np.exp(np.random.default_rng(m).uniform(-1, 1, m))   # within a decade of the median
        ps, us = physics_space(t)
        xi = (np.arange(m) + 0.5) / m
        assert np.array_equal(ps, linear_space(xi)) and np.array_equal(us, linear_space(xi))


def test_classification():
    t = np.ones(16)
    t[3:6] = 1e4            # channel
    t[9] = 50.0             # a decade and more above: a one-face channel
    t[12:14] = 1e-2         # barrier
    t[15] = 5.0             # below the threshold
    ch, bar = classify_interface(t)
    assert ch == [(3, 5), (9, 9)] and bar == [(12, 13)]
    # more channels than kept: the widest two, in order
    t2 = np.ones(32)
    for r in ((1, 1), (4, 7), (12, 13), (20, 25)):
        t2[r[0]:r[1] + 1] = 1e3
    ch2, _ = classify_interface(t2)
    assert ch2 == [(4, 7), (20, 25)]


def channel_problem(space="physics", adaptive=None, seed=3):
    base = inputs.make_problem("channel256_q5", nx=64, ny=64, seed=seed)
    return base.replace(space=space, p_dofs=4 if space == "physics" else 2,
                        u_dofs=4 if space == "physics" else 2, adaptive_alpha=adaptive)


def test_adaptive_alpha_follows_the_classification():
    prob = channel_problem(adaptive=(1e-2, 1e2))
    geom = Geometry(prob)
    a = interface_alpha(geom, prob)
    n_ch = 0
    for itf in geom.interfaces:
        ch, _ = classify_interface(od.face_conductance(prob.perm[itf.lo_cells], prob.perm[itf.hi_cells]))
        assert a[itf.index] == (1e-2 if ch else 1e2)
        n_ch += bool(ch)
    assert 0 < n_ch < geom.n_iface      # the case has both kinds


def barrier_problem(space):
    """K = 1e3 with low-permeability (K = 1) bands of rows, flow along x
    (p = 1 on W, 0 on E, no flow on S and N), 4 x 4 subdomains of 8 x 8:
    every vertical interface crosses one barrier band."""
    n = 32
    k_rows = np.full(n, 1e3)
    for r in ((2, 3), (12, 13), (19, 19), (28, 30)):
        k_rows[r[0]:r[1] + 1] = 1.0
    pd = 4 if space == "physics" else 2
    return Problem(name="barriers", nx=n, ny=n, lx=1.0, ly=1.0, perm=np.repeat(k_rows, n), sub_nx=8,
                   sub_ny=8, bc_kind=(DIRICHLET, DIRICHLET, NEUMANN, NEUMANN),
                   bc_value=(np.ones(n), np.zeros(n), None, None), space=space, p_dofs=pd, u_dofs=pd)


def test_barrier_flux_space_is_exact_where_linear_is_not():
    """K depending on y only and flow along x: p = 1 - x exactly and
    u_x = K(y): on a vertical interface the pressure is constant and the
    flux is 1e3 off the barrier and 1 on it, which the barrier functions of
    eqs. (new_basis4)-(new_basis6) hold and the linear functions do not; on
    the horizontal interfaces (uniform K along them: linear spaces) the
    pressure is linear and the flux zero.  So the MRCM with the physics
    spaces reproduces the fine solution, the one with linear spaces does
    not."""
    ref = solve_fine(barrier_problem("physics"))
    r = solve_mrcm(barrier_problem("physics"))
    assert max(int(n) for n in r.n_u) == 3                 # the barrier spaces are in use
    assert np.linalg.norm(r.p - ref["p"]) < 1e-12 * np.linalg.norm(ref["p"])
    F, Fr = np.r_[r.Fx, r.Fy], np.r_[ref["Fx"], ref["Fy"]]
    assert np.linalg.norm(F - Fr) < 1e-11 * np.linalg.norm(Fr)
    lin = solve_mrcm(barrier_problem("linear"))
    assert np.linalg.norm(np.r_[lin.Fx, lin.Fy] - Fr) > 1e-3 * np.linalg.norm(Fr)


def test_physics_spaces_balance_every_cell():
    prob = channel_problem(adaptive=(1e-2, 1e2))
    r = solve_mrcm(prob)
    assert flux_imbalance(Geometry(prob), prob, r.Fx, r.Fy) < 1e-12
    # the spaces of the case have more than 2 + 2 functions on some interfaces
    sizes = {int(n) for n in r.n_p} | {int(n) for n in r.n_u}
    assert max(sizes) > 2
