"""Pins of the oracle's liquid diagnostics (Sec. IV A/B): brute force over nodes on tiny
boxes and a closed form for a flat film on a wall."""
import numpy as np
import pytest

from oracle import lbm as olbm
from oracle.eos import CarnahanStarling


def _params(Q, nx, ny, nz, **kw):
    return olbm.Params(Q=Q, nx=nx, ny=ny, nz=nz, eos=CarnahanStarling(0.5, 4.0, 1.0, 0.7), **kw)


@pytest.mark.parametrize("reach", [1, 2, 3])
@pytest.mark.parametrize("Q", [19, 27])
def test_liquid_stats_brute_force(Q, reach):
    P = _params(Q, 7, 6, 5, walls={"z_lo": True}, cylinder=(2.0, 3.0, 1.2))
    solid = olbm.solid_mask(P)
    rng = np.random.default_rng(3)
    f = rng.uniform(0.0, 0.1, size=(Q,) + P.shape)
    f[:, solid] = 0.0
    thr, rv, rl = 0.9, 0.3, 1.5
    cz, wet, vol = olbm.liquid_stats(f, P, thr, rv, rl, solid, reach=reach)
    e = P.lat.e
    bc = np.zeros(P.nz, dtype=np.int64)
    bw = np.zeros(P.nz, dtype=np.int64)
    bv = 0.0
    for z in range(P.nz):
        for y in range(P.ny):
            for x in range(P.nx):
                if solid[z, y, x]:
                    continue
                rho = sum(float(f[i, z, y, x]) for i in range(Q))
                bv += min(max((rho - rv) / (rl - rv), 0.0), 1.0)
                if rho > thr:
                    bc[z] += 1
                    if any(solid[(z + k * e[i][2]) % P.nz, (y + k * e[i][1]) % P.ny,
                                 (x + k * e[i][0]) % P.nx]
                           for i in range(1, Q) for k in range(1, reach + 1)):
                        bw[z] += 1
    assert np.array_equal(cz, bc)
    assert np.array_equal(wet, bw)
    assert abs(vol - bv) <= 1e-12 * bv


def test_liquid_stats_flat_film_on_wall():
    """A film of rho_l filling planes z = 1..3 above the wall z = 0, vapour elsewhere:
    three full planes of liquid, one of them (z = 1) wetting the wall, volume 3 nx ny."""
    P = _params(19, 8, 6, 10, walls={"z_lo": True})
    solid = olbm.solid_mask(P)
    rv, rl = 0.01, 0.4
    rho = np.full(P.shape, rv)
    rho[1:4] = rl
    f = olbm.equilibrium_populations(P, rho, np.zeros((3,) + P.shape), solid)
    cz, wet, vol = olbm.liquid_stats(f, P, 0.5 * (rv + rl), rv, rl, solid)
    assert list(cz) == [0, 48, 48, 48, 0, 0, 0, 0, 0, 0]
    assert list(wet) == [0, 48, 0, 0, 0, 0, 0, 0, 0, 0]
    # reach 2: the second liquid plane is two steps from the wall; reach 3: the third too
    assert list(olbm.liquid_stats(f, P, 0.5 * (rv + rl), rv, rl, solid, reach=2)[1][:5]) == [0, 48, 48, 0, 0]
    assert list(olbm.liquid_stats(f, P, 0.5 * (rv + rl), rv, rl, solid, reach=3)[1][:5]) == [0, 48, 48, 48, 0]
    assert abs(vol - 3 * 48) < 1e-9


@pytest.mark.parametrize("Q", [19, 27])
def test_totals_of_a_uniform_moving_state_closed_form(Q):
    """The five totals of a uniform state rho0, u0 (equilibrium populations, periodic box,
    no interaction force since psi is uniform) with a uniform body force b: by Eq. (10) the
    momentum of each node is sum_i f_i e_i + b/2 = rho0 u0 + b/2, so the totals are
    N rho0, N (rho0 u0 + b/2) and N |rho0 u0 + b/2|^2 / (2 rho0) (kinetic energy
    rho |u|^2 / 2 with u the momentum over rho). A dropped 1/2 in the kinetic energy, a
    missing F/2 or a wrong component would each break one of these."""
    b = np.array([2e-4, -3e-4, 5e-4])
    P = _params(Q, 5, 4, 3, body_force=tuple(b))
    rho0, u0 = 0.27, np.array([0.03, -0.02, 0.05])
    rho = np.full(P.shape, rho0)
    u = np.broadcast_to(u0.reshape(3, 1, 1, 1), (3,) + P.shape).copy()
    f = olbm.equilibrium_populations(P, rho, u)
    N = P.nx * P.ny * P.nz
    j = rho0 * u0 + 0.5 * b
    want = np.array([N * rho0, *(N * j), N * float(j @ j) / (2 * rho0)])
    got = olbm.totals(f, P)
    assert np.allclose(got, want, rtol=1e-13, atol=0.0), (got, want)


def test_totals_exclude_solid_nodes():
    """Totals run over fluid nodes only: a uniform resting state between two walls has the
    mass of its fluid layers (nz - 2 planes) and no momentum or kinetic energy."""
    P = _params(19, 4, 3, 6, walls={"z_lo": True, "z_hi": True})
    rho = np.full(P.shape, 0.3)
    f = olbm.equilibrium_populations(P, rho, np.zeros((3,) + P.shape))
    got = olbm.totals(f, P)
    assert abs(got[0] - 0.3 * 4 * 3 * 4) < 1e-13
    assert np.all(np.abs(got[1:]) < 1e-15)
