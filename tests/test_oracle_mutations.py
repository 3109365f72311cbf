"""Planted mistakes in the oracle (CPU only) must be caught by the pins.

Each case monkeypatches one plausible slip into the oracle - a wrong mean,
a flipped normal sign, a dropped Robin factor - and checks that the closed
form / reduction pins reject it.  This shows the pins constrain every part
of the chain, not only the parts that happen to be exercised.
"""
import numpy as np
import pytest

import oracle.discretization as od
import oracle.fine as of
import oracle.mrcm as om
from inputs import make_problem
from oracle.fine import solve_fine
from tests import test_oracle_pins as P
from tests import test_oracle_pins_data as PD
from tests.test_oracle_pins import linear_dirichlet


PINS = [
    lambda: P.test_tiny_mrcm_closed_form(),
    lambda: P.test_linear_pressure_reproduced(0.7),
    lambda: P.test_full_spaces_recover_fine(0.7),
    lambda: P.test_full_spaces_pure_neumann(),
    lambda: P.test_conservation(),
    lambda: P.test_alpha_limits(),
    lambda: PD.test_fine_layered_data_closed_form(3),
    lambda: PD.test_mrcm_layered_data_closed_form(1, "linear"),
    lambda: PD.test_mrcm_layered_data_closed_form(3, "linear"),
    lambda: PD.test_mrcm_layered_data_closed_form(5, "full"),
    lambda: PD.test_mrcm_layered_data_closed_form_along_y(3),
    lambda: PD.test_quarter_five_spot_source_sign(),
    lambda: PD.test_mixed_alpha_limits_per_interface(),
]


def _pins_pass():
    """True when every pin passes on the (possibly mutated) oracle."""
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            return False
    return True


def test_unmodified_oracle_passes():
    assert _pins_pass()


def test_arithmetic_mean_caught(monkeypatch):
    monkeypatch.setattr(om, "harmonic", lambda a, b: 0.25 * (a + b))
    assert not _pins_pass()


def test_reversed_normal_is_harmless(monkeypatch):
    """Reversing the fixed skeleton normal on both sides only flips the sign
    of the flux unknowns: the pins must still pass."""
    orig = om._side_records

    def flipped(geom, prob, kappa, alpha, rho=None):
        recs = orig(geom, prob, kappa, alpha, rho)
        for per in recs:
            per[0]["sigma"], per[1]["sigma"] = -1.0, 1.0
        return recs
    prob = make_problem("gauss64", nx=32, ny=32, sub=8, alpha=0.7)
    ref = om.solve_mrcm(prob)
    monkeypatch.setattr(om, "_side_records", flipped)
    r = om.solve_mrcm(prob)
    assert np.linalg.norm(r.p - ref.p) < 1e-12 * np.linalg.norm(ref.p)
    assert np.linalg.norm(r.Fx - ref.Fx) < 1e-11 * np.linalg.norm(ref.Fx)


def test_one_sided_normal_sign_caught(monkeypatch):
    orig = om._side_records

    def flipped(geom, prob, kappa, alpha, rho=None):
        recs = orig(geom, prob, kappa, alpha, rho)
        for per in recs:
            per[1]["sigma"] = 1.0
        return recs
    monkeypatch.setattr(om, "_side_records", flipped)
    assert not _pins_pass()


def test_dropped_beta_in_flux_data_caught(monkeypatch):
    def nobeta(itf, rec, ps, us, col):
        m = itf.faces.size
        nP, nU = ps.shape[0], us.shape[0]
        G = np.zeros((m, nP + nU))
        G[:, :nP] = ps.T
        G[:, nP:] = (-rec["sigma"]) * us.T
        return G
    monkeypatch.setattr(om, "_interface_data", nobeta)
    assert not _pins_pass()


def test_transposed_projection_caught(monkeypatch):
    # use the pressure functions where the flux functions belong
    def swapped(geom, prob):
        from oracle.discretization import interface_spaces
        sp = interface_spaces(geom, prob)
        return [(ps, ps[::-1].copy()) for ps, us in sp]
    monkeypatch.setattr(om, "interface_spaces", swapped)
    prob = make_problem("gauss64", nx=32, ny=32, sub=8, alpha=0.7)
    lin, exact = linear_dirichlet(16, 12, 4, 0.5, 2.0, -1.5, alpha=0.7)
    # a reversed basis spans the same space: still exact (basis independence)
    assert np.abs(om.solve_mrcm(lin).p - exact).max() < 1e-12


def _flipped_injection(prob, hx, hy):
    return -od.cell_injection(prob, hx, hy)


def _flipped_outflow(u_b, flen):
    return -od.neumann_outflow(u_b, flen)


def test_source_sign_flip_in_mrcm_caught(monkeypatch):
    """q enters the local problems and the balance check with the wrong sign
    (consistently, so the MRCM still conserves its own flipped source)."""
    monkeypatch.setattr(om, "cell_injection", _flipped_injection)
    assert not _pins_pass()


def test_source_sign_flip_in_fine_caught(monkeypatch):
    monkeypatch.setattr(of, "cell_injection", _flipped_injection)
    assert not _pins_pass()


def test_source_scale_caught(monkeypatch):
    """q per cell instead of q per unit area (|V| dropped)."""
    monkeypatch.setattr(om, "cell_injection",
                        lambda prob, hx, hy: od.cell_injection(prob, hx, hy) / (hx * hy))
    assert not _pins_pass()


def test_neumann_sign_flip_in_mrcm_caught(monkeypatch):
    """u_b read as the inward instead of the outward normal velocity, in the
    local problems and in the boundary fluxes alike."""
    monkeypatch.setattr(om, "neumann_outflow", _flipped_outflow)
    assert not _pins_pass()


def test_neumann_sign_flip_in_fine_caught(monkeypatch):
    monkeypatch.setattr(of, "neumann_outflow", _flipped_outflow)
    assert not _pins_pass()


def test_alpha_from_wrong_interface_caught(monkeypatch):
    """Per-interface alpha read in reverse interface order."""
    orig = om.interface_alpha
    monkeypatch.setattr(om, "interface_alpha", lambda geom, prob: orig(geom, prob)[::-1].copy())
    assert not _pins_pass()


# ---------------------------------------------------------------------------
# gravity variant (section 5.5)
# ---------------------------------------------------------------------------

from tests import test_oracle_gravity as PG  # noqa: E402

GRAVITY_PINS = [
    lambda: PG.test_hydrostatic_closed_box(),
    lambda: PG.test_hydrostatic_with_dirichlet_top_and_bottom(),
    lambda: PG.test_layered_column_closed_form(),
    lambda: PG.test_full_spaces_recover_fine_with_gravity(),
    lambda: PG.test_one_subdomain_is_fine_with_gravity(),
    lambda: PG.test_stitched_fluxes_balance_with_gravity(),
]


def _gravity_pins_pass():
    for pin in GRAVITY_PINS:
        try:
            pin()
        except AssertionError:
            return False
    return True


def test_unmodified_oracle_passes_gravity_pins():
    assert _gravity_pins_pass()


def _patch_face_fluxes(monkeypatch, fn):
    monkeypatch.setattr(om, "gravity_face_fluxes", fn)
    monkeypatch.setattr(of, "gravity_face_fluxes", fn)


def test_gravity_face_density_of_one_side_caught(monkeypatch):
    """The lower cell's density on a whole interior face instead of the two
    half cells' densities."""
    orig = od.gravity_face_fluxes

    def lower_only(prob, kappa, rho):
        GY = orig(prob, kappa, rho)
        if rho is None or prob.gravity == 0.0:
            return GY
        R = np.asarray(rho).reshape(prob.ny, prob.nx)
        fix = np.where(R[:-1, :] + R[1:, :] != 0, 2.0 * R[:-1, :] / (R[:-1, :] + R[1:, :] + 1e-300), 1.0)
        GY[1:-1, :] *= fix
        return GY
    _patch_face_fluxes(monkeypatch, lower_only)
    assert not _gravity_pins_pass()


def test_gravity_sign_flip_caught(monkeypatch):
    orig = od.gravity_face_fluxes
    _patch_face_fluxes(monkeypatch, lambda prob, kappa, rho: -orig(prob, kappa, rho))
    assert not _gravity_pins_pass()


def test_gravity_missing_on_dirichlet_faces_caught(monkeypatch):
    orig = od.gravity_face_fluxes

    def no_boundary(prob, kappa, rho):
        GY = orig(prob, kappa, rho)
        GY[0, :] = 0.0
        GY[-1, :] = 0.0
        return GY
    _patch_face_fluxes(monkeypatch, no_boundary)
    assert not _gravity_pins_pass()


def test_gravity_sign_flip_on_robin_faces_caught(monkeypatch):
    orig = om._side_records

    def flipped(geom, prob, kappa, alpha, rho=None):
        recs = orig(geom, prob, kappa, alpha, rho)
        for per in recs:
            for r in per:
                r["G"] = -r["G"]
        return recs
    monkeypatch.setattr(om, "_side_records", flipped)
    assert not _gravity_pins_pass()


def test_gravity_dropped_on_robin_faces_caught(monkeypatch):
    orig = om._side_records

    def dropped(geom, prob, kappa, alpha, rho=None):
        recs = orig(geom, prob, kappa, alpha, rho)
        for per in recs:
            for r in per:
                r["G"] = 0.0 * r["G"]
        return recs
    monkeypatch.setattr(om, "_side_records", dropped)
    assert not _gravity_pins_pass()


def test_gravity_robin_distance_caught(monkeypatch):
    """The full cell height in place of the centre-to-face distance in the
    Robin faces' gravity term."""
    orig = om._side_records

    def doubled(geom, prob, kappa, alpha, rho=None):
        recs = orig(geom, prob, kappa, alpha, rho)
        for per in recs:
            for r in per:
                r["G"] = 2.0 * r["G"]
        return recs
    monkeypatch.setattr(om, "_side_records", doubled)
    assert not _gravity_pins_pass()


# ---------------------------------------------------------------------------
# physics-based interface spaces (section 3.1)
# ---------------------------------------------------------------------------

from tests import test_oracle_physics_spaces as PS  # noqa: E402

PHYSICS_PINS = [lambda seed=seed: PS.test_pressure_functions(seed) for seed in range(12)] + \
    [lambda seed=seed: PS.test_flux_functions(seed) for seed in range(8)] + [
    lambda: PS.test_no_structure_gives_the_linear_space(),
    lambda: PS.test_classification(),
    lambda: PS.test_barrier_flux_space_is_exact_where_linear_is_not(),
]


def _physics_pins_pass():
    for pin in PHYSICS_PINS:
        try:
            pin()
        except AssertionError:
            return False
    return True


def test_unmodified_oracle_passes_physics_pins():
    assert _physics_pins_pass()


def test_ramp_towards_the_wrong_end_caught(monkeypatch):
    """psi_0 rising instead of falling across the first segment."""
    orig = od.physics_pressure_space

    def flipped(channels, m):
        ps = orig(channels, m)
        if channels[0][0] > 0:
            x = (np.arange(m) + 0.5) / m
            a1 = channels[0][0] / m
            ps = ps.copy()
            ps[0] = np.where(x < a1, x / a1, 0.0)
        return ps
    monkeypatch.setattr(od, "physics_pressure_space", flipped)
    monkeypatch.setattr(PS, "physics_pressure_space", flipped)
    assert not _physics_pins_pass()


def test_barrier_segment_off_by_one_caught(monkeypatch):
    """The barrier indicator one face short at its end."""
    orig = od.physics_flux_space

    def short(barriers, m):
        return orig([(j0, max(j0, j1 - 1)) for j0, j1 in barriers], m)
    monkeypatch.setattr(od, "physics_flux_space", short)
    monkeypatch.setattr(PS, "physics_flux_space", short)
    assert not _physics_pins_pass()


def test_classification_against_the_mean_caught(monkeypatch):
    """Structures judged against the mean conductance instead of the median
    (a channel then raises the reference and is no longer found)."""
    orig_median = np.median
    monkeypatch.setattr(od.np, "median", lambda t: float(np.mean(t)))
    try:
        assert not _physics_pins_pass()
    finally:
        monkeypatch.setattr(od.np, "median", orig_median)
