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
