"""The Carnahan-Starling workloads on their own terms (CS EOS a = 0.5, b = 4, R = 1, G = -1).

The paper fixes sigma (the coefficient of the mechanical-stability source term of Eq. (B1))
for its piecewise EOS only. For CS the coexistence densities of a flat interface depend on
sigma steeply, so sigma is fitted so that a planar interface reproduces the Maxwell
construction, and the Laplace law (Eq. (17)) with its kappa tuning is then measured on the
256^3 static droplets of the Laplace workload."""
import numpy as np
import pytest

import synth_inputs as si
from tests.helpers import gpu_params, maxwell

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2306_16274_amd import lbm
    lbm.library()
    return lbm


def _flat_interface(L, T, rates, sigma, Q=19, n=256, steps=40000):
    """Liquid slab 64 < z < 192 in a 4 x 4 x 256 periodic box (FP64), started from a tanh
    profile between the Maxwell densities; (rho_v, rho_l, Maxwell rho_v, Maxwell rho_l)."""
    w = si.Workload("slab", Q, 4, 4, n, T_over_Tc=T, rates=rates, nu=0.1)
    rv, rl = maxwell(w)
    z = np.arange(n)
    rho = 0.5 * (rl + rv) + 0.5 * (rl - rv) * np.tanh(2.0 * np.minimum(z - 64, 192 - z) / 5.0)
    with L.Lattice(gpu_params(w, "fp64", sigma=sigma, reduce_every=1000)) as lat:
        lat.init_fields(np.broadcast_to(rho.reshape(n, 1, 1), (n, 4, 4)).copy())
        lat.step(steps)
        r = lat.moments(want=("rho",))["rho"][:, 0, 0]
    return float(r[0]), float(r[n // 2]), rv, rl


# Fitted sigma per (temperature, rate set, lattice): the Laplace, impact and cylinder
# workloads take the first three; the serving physics (0.7 T_c with the paper's rates, s4 = 1
# and nu = 0.05) takes its own fit, checked in test_serving_physics_sigma_fit below; the 32^3
# parity droplet keeps sigma = 0.1.
SIGMA_FITS = [(0.5, "unit", 19, si.LAPLACE_256.sigma, 0.005),
              (0.55, "paper", 19, si.IMPACT_384.sigma, 0.005),
              (0.6, "paper", 27, si.CYLINDER_D3Q27.sigma, 0.01),
              (0.7, "unit", 19, 0.1165, 0.015)]


@pytest.mark.parametrize("T,rates,Q,sigma,dsig", SIGMA_FITS)
def test_fitted_sigma_reproduces_maxwell_on_a_flat_interface(L, T, rates, Q, sigma, dsig):
    """With the fitted sigma (0.1153 at 0.5 T_c with unit non-viscous rates, 0.1190 at
    0.55 T_c and 0.1186 at 0.6 T_c (D3Q27) with the paper's rates, 0.1165 at 0.7 T_c with
    unit rates) a planar interface settles within 3 % of the Maxwell vapour density and
    0.1 % of the liquid density after 40000 steps (measured: +0.3 % / -0.04 %, +0.4 % /
    -0.001 %, +0.6 % / -0.005 %, +0.2 % / -0.03 %). The fit is sharp: dsig either side
    moves the vapour density by more than 10 % (at 0.5 T_c: -40 % at 0.11, +42 % at 0.12)."""
    rv_s, rl_s, rv, rl = _flat_interface(L, T, rates, sigma, Q)
    print(f"T {T} sigma {sigma}: rho_v {rv_s:.5e} ({rv_s / rv - 1:+.4f}) "
          f"rho_l {rl_s:.6f} ({rl_s / rl - 1:+.5f})")
    assert abs(rv_s / rv - 1) < 0.03
    assert abs(rl_s / rl - 1) < 1e-3
    lo = _flat_interface(L, T, rates, sigma - dsig, Q)[0]
    hi = _flat_interface(L, T, rates, sigma + dsig, Q)[0]
    assert lo < 0.9 * rv and hi > 1.1 * rv, (lo, hi)


def test_serving_physics_sigma_fit(L):
    """The serving physics (CS 0.7 T_c, D3Q19, the paper's rates with s4 = 1, nu = 0.05) with
    its sigma (serving.SIGMA = 0.1175): a planar interface within 3 % of the Maxwell vapour
    density and 0.1 % of the liquid density after 40000 steps (measured +0.2 %, -0.01 %)."""
    from paper_2306_16274_amd import serving
    n = 256
    w = si.Workload("slab", 19, 4, 4, n, T_over_Tc=0.7, rates="paper", nu=0.05)
    rv, rl = maxwell(w)
    z = np.arange(n)
    rho = 0.5 * (rl + rv) + 0.5 * (rl - rv) * np.tanh(2.0 * np.minimum(z - 64, 192 - z) / 5.0)
    p = gpu_params(w, "fp64", sigma=serving.SIGMA, s4=1.0, reduce_every=1000)
    with L.Lattice(p) as lat:
        lat.init_fields(np.broadcast_to(rho.reshape(n, 1, 1), (n, 4, 4)).copy())
        lat.step(40000)
        r = lat.moments(want=("rho",))["rho"][:, 0, 0]
    print(f"serving physics: rho_v {r[0] / rv - 1:+.4f}, rho_l {r[n // 2] / rl - 1:+.5f}")
    assert abs(r[0] / rv - 1) < 0.03
    assert abs(r[n // 2] / rl - 1) < 1e-3


def _droplet_dp(L, R, kappa, steps):
    """Laplace jump of Eq. (17) (mean p at r <= R/3 minus mean p at r >= R + 15) of a
    droplet of the Laplace workload (256^3, FP32 shifted storage) after `steps`."""
    w = si.LAPLACE_256.with_(R=float(R), kappa=kappa)
    rv, rl = maxwell(w)
    n = w.nx
    c = n / 2
    with L.Lattice(gpu_params(w, "fp32", rho_ref=rv, reduce_every=500)) as lat:
        lat.init_droplet(c, c, c, float(R), w.W, rl, rv, 0.0, 0.0, 0.0, w.noise, w.seed)
        lat.step(steps)
        m = lat.moments(want=("rho", "p"))
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    vol = float(np.clip((m["rho"][r < R + 10] - rv) / (rl - rv), 0.0, 1.0).sum())
    Re = (3.0 * vol / (4.0 * np.pi)) ** (1.0 / 3.0)
    return Re, float(m["p"][r <= R / 3].mean() - m["p"][r >= R + 15].mean())


def test_laplace_law_and_kappa_tuning_on_the_laplace_workload(L):
    """The Laplace workload (256^3, CS 0.5 T_c, density ratio 725, fitted sigma) after 20000
    steps: droplets of R = 30, 40, 50 give dp linear in 1/R (R^2 > 0.99; measured 0.999 over
    R = 30-60 at 30000 steps, gamma = 0.0101 through the origin), and the tuning of Sec. III C
    scales gamma by 1 - kappa within 5 % at R = 40 (measured 0.596 and 0.196 for kappa = 0.4
    and 0.8). The shape oscillations that the tanh start excites decay over about 2 10^4
    steps at R >= 50 with nu = 0.1, which is why the runs are longer than the 5000 steps of
    the workload; a droplet of R = 20 evaporates into the box after about 1.4 10^4 steps."""
    pts = [_droplet_dp(L, R, 0.0, 20000) for R in (30, 40, 50)]
    Rs = np.array([a for a, _ in pts])
    dps = np.array([b for _, b in pts])
    A = np.vstack([2.0 / Rs, np.ones_like(Rs)]).T
    (g, c0), res, _, _ = np.linalg.lstsq(A, dps, rcond=None)
    r2 = 1 - res[0] / ((dps - dps.mean()) ** 2).sum()
    g_origin = float((dps * 2.0 / Rs).sum() / ((2.0 / Rs) ** 2).sum())
    ratios = [_droplet_dp(L, 40, k, 20000)[1] / pts[1][1] for k in (0.4, 0.8)]
    print(f"CS Laplace: R_eff {np.round(Rs, 2).tolist()} dp {dps.tolist()} gamma {g:.5f} "
          f"(through origin {g_origin:.5f}) R^2 {r2:.4f}; gamma(kappa)/gamma(0) {ratios}")
    assert r2 > 0.99
    assert 0.008 < g_origin < 0.012
    assert abs(ratios[0] / 0.6 - 1) < 0.05
    assert abs(ratios[1] / 0.2 - 1) < 0.05
