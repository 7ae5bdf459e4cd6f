"""Pins of the oracle's equations of state and coexistence solver (no GPU)."""
import math

import numpy as np
import pytest

from oracle import eos
from oracle.lattice import CS2
from tests.test_oracle_lattice import golden_values


def test_piecewise_spinodals_match_printed_values():
    """Sec. III A prints rho_1 = 0.001325 and rho_2 = 0.9758 for rho_v = 0.001, rho_l = 1
    with the slopes of Eq. (20)."""
    g = golden_values()
    pw = eos.Piecewise.paper_default()
    assert abs(pw.rho1 - g["pw_rho1"]) < 0.5e-6
    assert abs(pw.rho2 - g["pw_rho2"]) < 0.5e-4


def test_general_maxwell_solver_recovers_piecewise_coexistence():
    """The equal-area solver, run on the piecewise EOS built from the printed spinodals,
    returns the printed coexistence densities rho_v = 0.001 and rho_l = 1."""
    g = golden_values()
    tv, tm, tl = CS2 / 2, -CS2 / 40, CS2
    pw = eos.Piecewise(tv, tm, tl, 0.0013246030524, 0.9758004064415)
    rv, rl = eos.maxwell_densities(pw, 1e-6, 2.0)
    assert abs(rv - g["pw_rho_v"]) < 1e-9
    assert abs(rl - g["pw_rho_l"]) < 1e-8


def cs_chemical_potential(cs, rho):
    """Closed-form Carnahan-Starling chemical potential (up to a constant):
    mu = R T [ln rho + (8 eta - 9 eta^2 + 3 eta^3)/(1 - eta)^3] - 2 a rho."""
    eta = cs.b * rho / 4
    return cs.R * cs.T * (math.log(rho) + (8 * eta - 9 * eta ** 2 + 3 * eta ** 3)
                          / (1 - eta) ** 3) - 2 * cs.a * rho


@pytest.mark.parametrize("t", [0.5, 0.55, 0.6, 0.7])
def test_carnahan_starling_maxwell_densities(t):
    """Equal pressure and equal chemical potential at the solver's answer, checked with the
    closed-form chemical potential (independent of the solver's quadrature)."""
    cs = eos.CarnahanStarling(0.5, 4.0, 1.0, t)
    rv, rl = eos.maxwell_densities(cs, 1e-9, 0.7)
    assert rv < rl
    pv, pl = float(cs.p(rv)), float(cs.p(rl))
    assert abs(pv - pl) < 1e-13
    assert abs(cs_chemical_potential(cs, rv) - cs_chemical_potential(cs, rl)) < 1e-11


def test_carnahan_starling_critical_temperature():
    """T_c = 0.3773 a / (b R): an unstable branch (dp/drho < 0) exists just below it and not
    just above it."""
    def min_slope(t):
        cs = eos.CarnahanStarling(0.5, 4.0, 1.0, t)
        r = np.linspace(0.01, 0.6, 60001)
        return np.diff(cs.p(r)).min()
    assert min_slope(0.995) < 0
    assert min_slope(1.005) > 0


@pytest.mark.parametrize("which", ["cs", "pw"])
def test_pseudopotential_reproduces_eos_pressure(which):
    """Eq. (17) with the square-root psi of Sec. II C gives back p_EOS wherever psi^2 >= 0."""
    e = (eos.CarnahanStarling(0.5, 4.0, 1.0, 0.6) if which == "cs"
         else eos.Piecewise.paper_default())
    rho = np.linspace(1e-4, 0.5 if which == "cs" else 1.1, 500)
    G = -1.0
    ps = eos.psi(e, rho, G)
    assert np.all(ps >= 0)
    assert np.allclose(eos.bulk_pressure(rho, ps, G), e.p(rho), rtol=0, atol=1e-15)
