"""Host-side pieces of the impact diagnostics: the piecewise-EOS knees of Eq. (19), the
contact-angle fit and the spreading diameter, on exact geometry."""
import math

import numpy as np
import pytest

from oracle.eos import Piecewise
from paper_2306_16274_amd import impact


def test_piecewise_knees_reproduce_printed_values():
    r1, r2 = impact.piecewise_knees()
    assert abs(r1 - 0.001325) < 5e-7 and abs(r2 - 0.9758) < 5e-5      # Sec. III A
    pw = Piecewise.paper_default()                                       # independent solver
    assert abs(r1 - pw.rho1) < 1e-12 * pw.rho1 and abs(r2 - pw.rho2) < 1e-12


def _voxel_cap(theta_deg, Rs, n=160):
    zc = 0.5 - Rs * math.cos(math.radians(theta_deg))
    z, y, x = np.meshgrid(np.arange(n // 2), np.arange(n), np.arange(n), indexing="ij")
    inside = ((x - n / 2) ** 2 + (y - n / 2) ** 2 + (z - zc) ** 2 <= Rs * Rs) & (z >= 1)
    return inside.sum(axis=(1, 2))


@pytest.mark.parametrize("theta", [60.0, 90.0, 120.0, 157.0])
def test_contact_angle_fit_on_voxelised_caps(theta):
    counts = _voxel_cap(theta, 30.0)
    got, rs, _ = impact.contact_angle_from_planes(counts)
    assert abs(got - theta) < 1.5, (got, theta)
    assert abs(rs - 30.0) < 0.5


def test_spreading_diameter_of_a_disc():
    n = 200
    y, x = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    disc = ((x - 100.3) ** 2 + (y - 99.7) ** 2 <= 40.0 ** 2).sum()
    counts = np.array([0, disc, 0])
    assert abs(impact.spreading_diameter(counts, 1) - 80.0) < 0.1


def test_impact_geometry():
    c = impact.ImpactCase(r_cyl=20.0, R0=50.0, gap=4.0)
    assert c.centre()[2] == pytest.approx(0.5 + 40.0 + 4.0 + 50.0)
    assert impact.capillary_time(1.0, 50.0, 0.01) == pytest.approx(math.sqrt(125000 / 0.01))
