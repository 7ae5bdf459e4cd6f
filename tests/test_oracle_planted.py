"""Planted mistakes: each test breaks the oracle on purpose (on the CPU, through
monkeypatch) and checks that at least one of the pins of test_oracle_step catches it.
This shows the pins are sharp enough to detect a dropped term, a wrong sign, a wrong
index or a transposed operand."""
import numpy as np
import pytest

from oracle import lbm
from oracle.lattice import lattice
from tests import oracle_pins as pins

FAST_PINS = [pins.conservation_error, pins.srt_bgk_error, pins.dense_lambda_error,
             pins.stencil_polynomial_error, pins.fixed_point_error, pins.neutral_wall_error,
             pins.periodic_momentum_drift, pins.wall_mass_drift]


def caught(Q=27, tol=1e-12):
    errs = [p(Q=Q) for p in FAST_PINS]
    return any(not (e < tol) for e in errs)


def test_clean_oracle_passes_every_pin():
    assert not caught(19) and not caught(27)


@pytest.mark.parametrize("Q", [19, 27])
def test_wrong_sign_in_equilibrium_moment(monkeypatch, Q):
    lat = lattice(Q)
    orig = lat.meq

    def bad(rho, ux, uy, uz):
        m = orig(rho, ux, uy, uz)
        m[4] = -m[4]
        return m
    monkeypatch.setattr(lat, "meq", bad)
    assert caught(Q)


@pytest.mark.parametrize("Q", [19, 27])
def test_dropped_term_in_forcing_moment(monkeypatch, Q):
    lat = lattice(Q)
    orig = lat.forcing_moments

    def bad(Fx, Fy, Fz, ux, uy, uz):
        Ft = orig(Fx, Fy, Fz, ux, uy, uz)
        Ft[9] = Ft[9] + 2.0 * Fz * uz     # 2(Fx ux - Fz uz) -> 2 Fx ux
        return Ft
    monkeypatch.setattr(lat, "forcing_moments", bad)
    assert caught(Q)


@pytest.mark.parametrize("Q", [19, 27])
def test_velocity_without_half_force_shift(monkeypatch, Q):
    orig = lbm.macroscopic

    def bad(f, P, solid=None):
        mac = orig(f, P, solid)
        mac["u"] = mac["u"] - 0.5 * mac["F"] / mac["rho"]
        return mac
    monkeypatch.setattr(lbm, "macroscopic", bad)
    assert caught(Q)


@pytest.mark.parametrize("Q", [19, 27])
def test_transposed_inverse(monkeypatch, Q):
    lat = lattice(Q)
    monkeypatch.setattr(lat, "Minv", lat.Minv.T.copy())
    assert caught(Q)


@pytest.mark.parametrize("Q", [19, 27])
def test_forcing_without_half_relaxation_factor(monkeypatch, Q):
    orig = lbm.modified_forcing

    def bad(P, mac, S):
        return orig(P, mac, S) / (1.0 - S / 2.0)
    monkeypatch.setattr(lbm, "modified_forcing", bad)
    assert caught(Q)


@pytest.mark.parametrize("Q", [19, 27])
def test_wrong_sign_of_surface_tension_source(monkeypatch, Q):
    orig = lbm.forces

    def bad(psi, solid, P):
        F_int, F_ads, Qab, phi = orig(psi, solid, P)
        Qab["xy"] = -Qab["xy"]
        return F_int, F_ads, Qab, phi
    monkeypatch.setattr(lbm, "forces", bad)
    assert caught(Q)


@pytest.mark.parametrize("Q", [19, 27])
def test_force_weights_not_normalised(monkeypatch, Q):
    lat = lattice(Q)
    monkeypatch.setattr(lat, "w", lat.omega.copy())
    assert caught(Q)


@pytest.mark.parametrize("Q", [19, 27])
def test_bounce_back_to_wrong_direction(monkeypatch, Q):
    lat = lattice(Q)
    monkeypatch.setattr(lat, "opp", np.arange(lat.Q))
    assert caught(Q)


@pytest.mark.parametrize("Q", [19, 27])
def test_swapped_moment_rows(monkeypatch, Q):
    lat = lattice(Q)
    M = lat.M.copy()
    M[[10, 12]] = M[[12, 10]]
    monkeypatch.setattr(lat, "M", M)
    assert caught(Q)


def _totals_pin_caught():
    import tests.test_oracle_diagnostics as d
    try:
        for Q in (19, 27):
            d.test_totals_of_a_uniform_moving_state_closed_form(Q)
    except AssertionError:
        return True
    return False


def test_clean_totals_pass_their_pin():
    assert not _totals_pin_caught()


@pytest.mark.parametrize("mistake", ["no_half_in_kinetic_energy", "momentum_without_half_force",
                                     "swapped_momentum_components"])
def test_planted_mistakes_in_totals(monkeypatch, mistake):
    """The closed-form pin of the totals catches a dropped 1/2 in E_k, momentum summed
    without the F/2 shift and two momentum components swapped."""
    orig_moments = lbm.moments

    def bad_moments(f, P, solid=None):
        rho, u, p, mac = orig_moments(f, P, solid)
        if mistake == "momentum_without_half_force":
            u = u - 0.5 * mac["F"] / rho
        elif mistake == "swapped_momentum_components":
            u = u[[1, 0, 2]]
        return rho, u, p, mac
    monkeypatch.setattr(lbm, "moments", bad_moments)
    if mistake == "no_half_in_kinetic_energy":
        orig_totals = lbm.totals

        def bad_totals(f, P, solid=None):
            t = orig_totals(f, P, solid)
            t[4] = 2.0 * t[4]
            return t
        monkeypatch.setattr(lbm, "totals", bad_totals)
    assert _totals_pin_caught()
