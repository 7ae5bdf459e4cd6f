"""Pins of the oracle's lattice tables against what the paper prints and what the
mathematics fixes (no GPU)."""
import os
from fractions import Fraction
from itertools import product

import numpy as np
import pytest

from oracle.lattice import CS2, lattice

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def golden_values():
    out = {}
    with open(os.path.join(GOLDEN, "paper_printed_values.txt")) as fh:
        for line in fh:
            line = line.split("--")[0].strip()
            if not line or line.startswith("#"):
                continue
            name, val = line.split()
            out[name] = Fraction(val) if "/" in val else float(val)
    return out


def printed_M(Q):
    return np.loadtxt(os.path.join(GOLDEN, f"M_d3q{Q}_printed.txt"))


@pytest.mark.parametrize("Q", [19, 27])
def test_M_from_moment_definitions_equals_printed_matrix(Q):
    """Eq. (2) with the moment set of Eq. (11)/(C2) reproduces Eq. (13)/(C4) entry by entry;
    a wrong velocity order or moment order fails here."""
    assert np.array_equal(lattice(Q).M, printed_M(Q))


@pytest.mark.parametrize("Q", [19, 27])
def test_nonzero_counts_match_table_I(Q):
    g = golden_values()
    lat = lattice(Q)
    nnz_M = sum(1 for row in lat.M_frac for x in row if x != 0)
    nnz_Minv = sum(1 for row in lat.Minv_frac for x in row if x != 0)
    assert nnz_M == g[f"nnz_M_d3q{Q}"]
    assert nnz_Minv == g[f"nnz_Minv_d3q{Q}"]


@pytest.mark.parametrize("Q", [19, 27])
def test_inverse_is_exact(Q):
    lat = lattice(Q)
    n = lat.Q
    for i in range(n):
        for j in range(n):
            s = sum(lat.M_frac[i][k] * lat.Minv_frac[k][j] for k in range(n))
            assert s == (1 if i == j else 0)
    # the float copies agree with the rationals
    assert np.abs(lat.M @ lat.Minv - np.eye(n)).max() < 1e-15


def test_d3q19_inverse_is_extracted_from_d3q27_inverse():
    """Appendix C states that the D3Q19 M^-1 is the corresponding rows and columns of the
    D3Q27 M^-1: rows = populations 0..18, columns = moments 0..15, 17, 18, 19."""
    q19, q27 = lattice(19), lattice(27)
    cols = list(range(16)) + [17, 18, 19]
    for i in range(19):
        for k, c in enumerate(cols):
            assert q19.Minv_frac[i][k] == q27.Minv_frac[i][c]


def test_d3q27_weights_are_the_printed_ones():
    g = golden_values()
    lat = lattice(27)
    norm2 = (lat.e ** 2).sum(1)
    for i in range(27):
        assert lat.omega_frac[i] == g[f"d3q27_w{int(norm2[i])}"]


@pytest.mark.parametrize("Q", [19, 27])
def test_weights_isotropy(Q):
    """sum w = 1, sum w e_a e_b = c_s^2 delta, fourth moments = c_s^4 (dd + dd + dd); the
    force stencil of Eq. (16) and the expansion of Eq. (B4) need this (also for the D3Q19
    weights, which the paper does not print)."""
    lat = lattice(Q)
    e = lat.e.astype(float)
    w = lat.omega
    assert abs(w.sum() - 1) < 1e-15
    d = np.eye(3)
    for a, b in product(range(3), repeat=2):
        assert abs((w * e[:, a] * e[:, b]).sum() - CS2 * d[a, b]) < 1e-15
    for a, b, c, dd in product(range(3), repeat=4):
        want = CS2 ** 2 * (d[a, b] * d[c, dd] + d[a, c] * d[b, dd] + d[a, dd] * d[b, c])
        assert abs((w * e[:, a] * e[:, b] * e[:, c] * e[:, dd]).sum() - want) < 1e-15
    for a, b, c in product(range(3), repeat=3):
        assert abs((w * e[:, a] * e[:, b] * e[:, c]).sum()) < 1e-15


def test_d3q19_rest_equilibrium_gives_the_weights():
    """M^-1 m^eq(rho=1, u=0) of the printed D3Q19 model is 1/3, 1/18 (x6), 1/36 (x12): this
    pins the D3Q19 weight reading used by the force stencil."""
    lat = lattice(19)
    f = lat.Minv @ lat.meq(np.array(1.0), np.array(0.0), np.array(0.0), np.array(0.0))
    assert np.allclose(f, lat.omega, rtol=0, atol=1e-16)


def test_d3q27_equilibrium_moments_equal_M_times_hermite_equilibrium():
    """Eq. (14) is M f^eq with f^eq of Eq. (5), for arbitrary rho, u."""
    lat = lattice(27)
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = rng.uniform(0.01, 2.0)
        u = rng.uniform(-0.2, 0.2, 3)
        m = lat.meq(np.array(rho), *map(np.array, u))
        assert np.allclose(lat.M @ lat.feq_hermite(rho, u), m, rtol=0, atol=1e-15)


def test_d3q27_forcing_moments_equal_M_times_guo_forcing():
    """Eq. (15) is M F_bar with the Guo forcing term of Eq. (6)."""
    lat = lattice(27)
    rng = np.random.default_rng(2)
    for _ in range(20):
        u = rng.uniform(-0.2, 0.2, 3)
        F = rng.uniform(-0.05, 0.05, 3)
        Ft = lat.forcing_moments(*map(np.array, F), *map(np.array, u))
        assert np.allclose(lat.M @ lat.guo_force(u, F), Ft, rtol=0, atol=1e-16)


def test_d3q19_low_order_moments_agree_with_hermite_forms():
    """For D3Q19 the printed m^eq and F~ equal M f^eq and M F_bar in moments 0..15; the
    three fourth-order moments differ, which is why the printed moment-space forms are
    taken as the D3Q19 definition."""
    lat = lattice(19)
    rng = np.random.default_rng(3)
    rho = 0.7
    u = rng.uniform(-0.1, 0.1, 3)
    F = rng.uniform(-0.05, 0.05, 3)
    m = lat.meq(np.array(rho), *map(np.array, u))
    Ft = lat.forcing_moments(*map(np.array, F), *map(np.array, u))
    assert np.allclose((lat.M @ lat.feq_hermite(rho, u))[:16], m[:16], atol=1e-15)
    assert np.allclose((lat.M @ lat.guo_force(u, F))[:16], Ft[:16], atol=1e-16)
    assert not np.allclose((lat.M @ lat.feq_hermite(rho, u))[16:], m[16:], atol=1e-6)


@pytest.mark.parametrize("Q", [19, 27])
def test_opposite_directions(Q):
    lat = lattice(Q)
    assert np.array_equal(lat.e[lat.opp], -lat.e)
