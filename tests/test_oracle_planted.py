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
