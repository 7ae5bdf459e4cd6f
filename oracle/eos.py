"""Equations of state, the square-root pseudopotential and Maxwell coexistence densities.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* Piecewise-linear EOS: Sec. III A, Eq. (18), slopes of Eq. (20), spinodal densities from
  the two conditions of Eq. (19). Eq. (19) is garbled in print (its first integral has no
  integrand); it is read as equal pressure, p(rho_v) = p(rho_l), and equal chemical
  potential, int_{rho_v}^{rho_l} dp / rho = 0, the conditions its right-hand sides state.
* Carnahan-Starling EOS: named in Sec. III A without a formula; the standard form
  p = rho R T (1 + eta + eta^2 - eta^3) / (1 - eta)^3 - a rho^2 with eta = b rho / 4 is used.
* Square-root pseudopotential: Sec. II C, psi = sqrt(2 (p_EOS - rho c_s^2) / (G c^2)),
  with c = 1. Where the argument is negative (outside the phase diagram) psi is 0.
* Bulk pressure of the model: Sec. II C, Eq. (17), p = rho c_s^2 + G c^2 psi^2 / 2.
"""
import math

import numpy as np
from scipy import integrate, optimize

from .lattice import CS2


class Piecewise:
    """Eq. (18): slopes theta_v, theta_m, theta_l joined at rho1, rho2."""

    def __init__(self, theta_v, theta_m, theta_l, rho1, rho2):
        self.theta_v, self.theta_m, self.theta_l = theta_v, theta_m, theta_l
        self.rho1, self.rho2 = rho1, rho2

    def p(self, rho):
        rho = np.asarray(rho, dtype=np.float64)
        tv, tm, tl, r1, r2 = self.theta_v, self.theta_m, self.theta_l, self.rho1, self.rho2
        return np.where(rho <= r1, rho * tv,
                        np.where(rho <= r2, r1 * tv + (rho - r1) * tm,
                                 r1 * tv + (r2 - r1) * tm + (rho - r2) * tl))

    @staticmethod
    def paper_default():
        """Eq. (20) slopes with rho1, rho2 solved from Eq. (19) for rho_v = 0.001, rho_l = 1."""
        tv, tm, tl = CS2 / 2.0, -CS2 / 40.0, CS2
        r1, r2 = piecewise_spinodals(tv, tm, tl, 0.001, 1.0)
        return Piecewise(tv, tm, tl, r1, r2)


def piecewise_spinodals(theta_v, theta_m, theta_l, rho_v, rho_l):
    """Solve Eq. (19) for (rho1, rho2) given the coexistence densities and the slopes.

    Condition 1 (equal pressure): (rho1-rho_v) th_v + (rho2-rho1) th_m + (rho_l-rho2) th_l = 0.
    Condition 2 (equal chemical potential):
        th_v log(rho1/rho_v) + th_m log(rho2/rho1) + th_l log(rho_l/rho2) = 0.
    Condition 1 is linear in rho2 given rho1; the remaining scalar equation in rho1 is
    solved by bracketing root search.
    """
    def rho2_of(r1):
        return ((r1 - rho_v) * theta_v - r1 * theta_m + rho_l * theta_l) / (theta_l - theta_m)

    def g(r1):
        r2 = rho2_of(r1)
        return (theta_v * math.log(r1 / rho_v) + theta_m * math.log(r2 / r1)
                + theta_l * math.log(rho_l / r2))

    # rho1 lies between rho_v and the point where rho2 would reach rho_l.
    lo = rho_v * (1.0 + 1e-12)
    hi = min(rho_l, rho_v + (rho_l - rho_v) * 0.5)
    r1 = optimize.brentq(g, lo, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    return r1, rho2_of(r1)


class CarnahanStarling:
    """Standard Carnahan-Starling EOS; T_c = 0.3773 a / (b R) as the workloads state."""

    def __init__(self, a, b, R, T_over_Tc):
        self.a, self.b, self.R = a, b, R
        self.Tc = 0.3773 * a / (b * R)
        self.T = T_over_Tc * self.Tc

    def p(self, rho):
        rho = np.asarray(rho, dtype=np.float64)
        eta = self.b * rho / 4.0
        return (rho * self.R * self.T * (1.0 + eta + eta * eta - eta ** 3) / (1.0 - eta) ** 3
                - self.a * rho * rho)


def psi(eos, rho, G):
    """Square-root pseudopotential of Sec. II C (c = 1), clamped at 0."""
    arg = 2.0 * (eos.p(rho) - np.asarray(rho) * CS2) / G
    return np.sqrt(np.maximum(arg, 0.0))


def bulk_pressure(rho, psi_, G):
    """Eq. (17): p = rho c_s^2 + G c^2 psi^2 / 2."""
    return rho * CS2 + 0.5 * G * psi_ * psi_


def maxwell_densities(eos, lo, hi):
    """Coexistence densities (rho_v, rho_l) by the equal-area rule.

    Unknowns rho_v < rho_l with p(rho_v) = p(rho_l) = p0 and
    int_{rho_v}^{rho_l} dp / rho = 0. Integrating by parts, the second condition reads
    p0 (1/rho_l - 1/rho_v) + int_{rho_v}^{rho_l} p(rho) / rho^2 d rho = 0.
    ``lo`` and ``hi`` bracket the spinodal region (p decreasing between them).
    """
    # spinodals: where dp/drho = 0
    def dp(r, h=1e-7):
        return (float(eos.p(r + h)) - float(eos.p(r - h))) / (2.0 * h)

    grid = np.linspace(lo, hi, 20001)
    slope = np.array([dp(r) for r in grid])
    neg = np.where(slope < 0)[0]
    if len(neg) == 0:
        raise ValueError("no unstable branch in the bracket: above the critical point")
    sp_lo = optimize.brentq(dp, grid[neg[0] - 1], grid[neg[0]])
    sp_hi = optimize.brentq(dp, grid[neg[-1]], grid[neg[-1] + 1])
    p_min, p_max = float(eos.p(sp_hi)), float(eos.p(sp_lo))

    def roots_at(p0):
        rv = optimize.brentq(lambda r: float(eos.p(r)) - p0, lo, sp_lo, xtol=1e-16, rtol=1e-15)
        rl = optimize.brentq(lambda r: float(eos.p(r)) - p0, sp_hi, hi, xtol=1e-16, rtol=1e-15)
        return rv, rl

    def area(p0):
        rv, rl = roots_at(p0)
        # in the variable s = ln(rho): int p / rho^2 d rho = int p(e^s) e^-s ds
        val, _ = integrate.quad(lambda s: float(eos.p(math.exp(s))) * math.exp(-s),
                                math.log(rv), math.log(rl), epsabs=1e-14, epsrel=1e-12,
                                limit=400)
        return p0 * (1.0 / rl - 1.0 / rv) + val

    eps = 1e-12 * max(abs(p_max), abs(p_min), 1e-30)
    p_floor = max(p_min, float(eos.p(lo)))
    p0 = optimize.brentq(area, p_floor + eps, p_max - eps, xtol=1e-18, rtol=1e-14)
    return roots_at(p0)
