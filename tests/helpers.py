"""Translation of a synthetic Workload into oracle parameters and into lbm_params, and
the comparison helpers used by the parity tests."""
import numpy as np

from oracle import eos as oeos
from oracle import lbm as olbm

RATES = {
    "paper": dict(s2b=0.6, s3=1.2, s3b=0.6, s4=1.2, s4b=1.2, s5=1.2, s6=1.2),
    "unit": dict(s2b=1.0, s3=1.0, s3b=1.0, s4=1.0, s4b=1.0, s5=1.0, s6=1.0),
}


def oracle_eos(w):
    if w.eos == "cs":
        return oeos.CarnahanStarling(w.cs_a, w.cs_b, w.cs_R, w.T_over_Tc)
    return oeos.Piecewise.paper_default()


def oracle_params(w, **over):
    kw = dict(Q=w.Q, nx=w.nx, ny=w.ny, nz=w.nz, eos=oracle_eos(w), G=w.G, sigma=w.sigma,
              kappa=w.kappa, G_ads=w.G_ads, nu_l=w.nu, walls={k: True for k in w.walls},
              cylinder=w.cylinder, wall_psi=w.wall_psi, **RATES[w.rates])
    kw.update(over)
    return olbm.Params(**kw)


def maxwell(w):
    e = oracle_eos(w)
    return oeos.maxwell_densities(e, 1e-9, 0.7 if w.eos == "cs" else 2.0)


def gpu_params(w, storage="fp64", rho_ref=0.0, **over):
    from paper_2306_16274_amd import lbm as L
    p = L.lbm_params_default()
    p.lattice = w.Q
    p.storage = {"fp64": L.LBM_FP64, "fp32": L.LBM_FP32, "fp16": L.LBM_FP16}[storage]
    p.nx, p.ny, p.nz = w.nx, w.ny, w.nz
    p.rho_ref = rho_ref
    if w.eos == "cs":
        p.eos = L.LBM_EOS_CS
        p.cs_a, p.cs_b, p.cs_R, p.T_over_Tc = w.cs_a, w.cs_b, w.cs_R, w.T_over_Tc
    else:
        pw = oeos.Piecewise.paper_default()
        p.eos = L.LBM_EOS_PIECEWISE
        p.pw_theta_v, p.pw_theta_m, p.pw_theta_l = pw.theta_v, pw.theta_m, pw.theta_l
        p.pw_rho1, p.pw_rho2 = pw.rho1, pw.rho2
    p.G, p.sigma, p.kappa, p.G_ads = w.G, w.sigma, w.kappa, w.G_ads
    p.nu_l = p.nu_v = w.nu
    for k, v in RATES[w.rates].items():
        setattr(p, k, v)
    axes = {"x": 0, "y": 1, "z": 2}
    for name in w.walls:
        ax, side = name.split("_")
        p.bc[axes[ax]][0 if side == "lo" else 1] = L.LBM_BC_WALL
    p.wall_psi = {"node": L.LBM_WALL_PSI_NODE, "fluid_mean": L.LBM_WALL_PSI_FLUID_MEAN,
                  "zero": L.LBM_WALL_PSI_ZERO, "mirror": L.LBM_WALL_PSI_MIRROR}[w.wall_psi]
    if w.cylinder is not None:
        p.cylinder = 1
        p.cyl_y, p.cyl_z, p.cyl_r = w.cylinder
    for k, v in over.items():
        setattr(p, k, v)
    return p


def rel_err(a, b, mask=None):
    """max |a - b| / |b| over the mask (pointwise relative error)."""
    if mask is not None:
        a, b = a[..., mask], b[..., mask]
    return float(np.max(np.abs(a - b) / np.abs(b)))


def abs_err(a, b, mask=None):
    if mask is not None:
        a, b = a[..., mask], b[..., mask]
    return float(np.max(np.abs(a - b)))


def totals_err(gpu_totals, f, P, solid=None):
    """Largest error of the GPU's five totals (mass, momentum, kinetic energy) against the
    oracle's for the state f, each scaled by the sum of the magnitudes it adds up (mass,
    sum |rho u_a|, E_k), so that near-zero momentum totals are compared at the rounding
    level of their terms."""
    from oracle import lbm as olbm
    want = olbm.totals(f, P, solid)
    rho, u, _, mac = olbm.moments(f, P, solid)
    fl = ~mac["solid"]
    scale = np.array([want[0]] + [np.abs(rho * u[a])[fl].sum() for a in range(3)] + [want[4]])
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.abs(np.asarray(gpu_totals) - want) / scale))


def piecewise_slab(w, z_a, z_b, W, f_amp=0.02, seed=3):
    """Oracle populations of a liquid slab z_a < z < z_b between the piecewise EOS's
    coexistence densities (rho_l = 1, rho_v = 0.001), a planar tanh profile of width W
    (Eq. (21)) on each face, at rest, with multiplicative noise amp U(-1, 1) on every
    population; and the oracle params. A slab is the stationary state of a planar
    interface, so the liquid stays above rho_2 and the vapour far from it below rho_1."""
    import synth_inputs as si
    from oracle import lbm as olbm
    P = oracle_params(w)
    solid = olbm.solid_mask(P)
    z = np.arange(w.nz, dtype=np.float64).reshape(-1, 1, 1)
    d = np.minimum(z - z_a, z_b - z)
    rho = np.broadcast_to(0.5 * 1.001 + 0.5 * 0.999 * np.tanh(2.0 * d / W), w.shape).copy()
    f = olbm.equilibrium_populations(P, rho, np.zeros((3,) + w.shape), solid)
    f = f * si.random_factors(w.Q, w.shape, seed=seed, amp=f_amp)
    f[:, solid] = 0.0
    return P, solid, f
