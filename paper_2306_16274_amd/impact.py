"""Droplet-on-wall diagnostics and the impact driver (Sec. III E wetting, Sec. IV A spreading,
Sec. IV B contact time and liquid volume).

Every number here comes from what the device reduces (`lbm_liquid_stats`: liquid nodes per
z plane, liquid nodes touching a solid, liquid volume); the host only fits and records a
handful of values per sample.

Geometry conventions: the bottom wall is the solid layer z = 0; with halfway bounce-back
its surface lies at z = 1/2. A cylinder lying on that wall along x has its axis at
(y, z) = (ny/2, 1/2 + r).
"""
import math
from dataclasses import dataclass

import numpy as np

from . import lbm as L

# Piecewise EOS of Sec. III A: slopes of Eq. (20) in units of c_s^2 = 1/3
THETA_V, THETA_M, THETA_L = 1.0 / 6.0, -1.0 / 120.0, 1.0 / 3.0


def piecewise_knees(rho_v=0.001, rho_l=1.0, theta_v=THETA_V, theta_m=THETA_M, theta_l=THETA_L):
    """rho_1, rho_2 of the piecewise-linear EOS (Eq. (18)) whose coexistence densities are
    rho_v, rho_l under the two conditions of Eq. (19): equal pressure,
        theta_v rho_v = theta_v rho_1 + theta_m (rho_2 - rho_1) + theta_l (rho_l - rho_2),
    and a vanishing integral of dp / rho between the two phases,
        theta_v ln(rho_1/rho_v) + theta_m ln(rho_2/rho_1) + theta_l ln(rho_l/rho_2) = 0.
    The first is linear: rho_1 follows from rho_2; the second is solved by bisection."""
    def rho1_of(r2):
        return (theta_v * rho_v - theta_l * rho_l - (theta_m - theta_l) * r2) / (theta_v - theta_m)

    def g(r2):
        r1 = rho1_of(r2)
        return (theta_v * math.log(r1 / rho_v) + theta_m * math.log(r2 / r1)
                + theta_l * math.log(rho_l / r2))

    # rho_1 > rho_v requires rho_2 above r_lo; rho_2 < rho_l
    r_lo = (theta_v * rho_v - theta_l * rho_l - (theta_v - theta_m) * rho_v) / (theta_m - theta_l)
    lo, hi = r_lo * (1 + 1e-15) + 1e-300, rho_l
    glo, ghi = g(lo), g(hi)
    if glo * ghi > 0:
        raise ValueError("no piecewise EOS with these slopes has coexistence at rho_v, rho_l")
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        gm = g(mid)
        if (gm < 0) == (glo < 0):
            lo, glo = mid, gm
        else:
            hi = mid
        if hi - lo <= 1e-16 * hi:
            break
    r2 = 0.5 * (lo + hi)
    return rho1_of(r2), r2


def set_piecewise(p, rho_v=0.001, rho_l=1.0):
    """Piecewise EOS of Sec. III A on an lbm_params."""
    p.eos = L.LBM_EOS_PIECEWISE
    p.pw_theta_v, p.pw_theta_m, p.pw_theta_l = THETA_V, THETA_M, THETA_L
    p.pw_rho1, p.pw_rho2 = piecewise_knees(rho_v, rho_l)
    return p


def contact_angle_from_planes(count_z, z_wall=0.5, trim=0.15):
    """Static contact angle (degrees) of a sessile droplet from its liquid area per plane.

    A spherical cap of radius Rs centred at height zc has cross-section area
    A(z) = pi (Rs^2 - (z - zc)^2). A least-squares fit of that parabola through the planes
    whose area exceeds `trim` of the largest (leaving out the first fluid layer and the
    topmost liquid plane, where the diffuse interface cuts the cap) gives Rs and zc, and
    cos(theta) = -(zc - z_wall) / Rs, theta measured inside the liquid.
    Returns (theta, Rs, zc)."""
    a = np.asarray(count_z, dtype=np.float64)
    z = np.arange(a.size, dtype=np.float64)
    big = a > trim * a.max()
    top = np.nonzero(big)[0].max()
    sel = big & (z > z_wall + 1.0) & (z < top)
    if sel.sum() < 3:
        raise ValueError("too few planes to fit the droplet profile")
    # A/pi + z^2 = 2 zc z + (Rs^2 - zc^2)
    b1, b0 = np.polyfit(z[sel], a[sel] / math.pi + z[sel] ** 2, 1)
    zc = 0.5 * b1
    rs2 = b0 + zc * zc
    if rs2 <= 0:
        raise ValueError("degenerate droplet profile")
    rs = math.sqrt(rs2)
    c = max(-1.0, min(1.0, -(zc - z_wall) / rs))
    return math.degrees(math.acos(c)), rs, zc


def spreading_diameter(count_z, z=1):
    """Diameter of the disc with the liquid area of plane z (D_f of Sec. IV A)."""
    return 2.0 * math.sqrt(float(count_z[z]) / math.pi)


@dataclass
class ImpactCase:
    """A droplet of radius R0 moving at -U along z towards the wall z = 0 (periodic in x
    and y, walls at z = 0 and z = nz - 1), optionally onto an x-aligned cylinder of radius
    r_cyl lying on that wall. Defaults follow Sec. IV B: piecewise EOS of Sec. III A
    (rho_v = 0.001, rho_l = 1), G = -1, sigma = 0.1, G_ads = 0.23, nu_l = 0.0075, R0 = 50
    in about 6 R0 x 6 R0 x 5 R0. The vapour viscosity is not given there; nu_v = 0.05 through
    the density-dependent viscosity of Eq. (24) keeps a cold start stable."""
    nx: int = 300
    ny: int = 300
    nz: int = 250
    R0: float = 50.0
    U: float = 0.044
    r_cyl: float = 0.0
    gap: float = 10.0             # initial distance between the R0 sphere and the solid below
    Q: int = 27
    storage: str = "fp32"
    G_ads: float = 0.23
    nu_l: float = 0.0075
    nu_v: float = 0.05
    kappa: float = 0.0
    W: float = 5.0
    rho_v: float = 0.001
    rho_l: float = 1.0

    def params(self):
        p = L.lbm_params_default()
        p.lattice = self.Q
        p.storage = {"fp64": L.LBM_FP64, "fp32": L.LBM_FP32, "fp16": L.LBM_FP16}[self.storage]
        p.nx, p.ny, p.nz = self.nx, self.ny, self.nz
        set_piecewise(p, self.rho_v, self.rho_l)
        p.G, p.sigma, p.kappa, p.G_ads = -1.0, 0.1, self.kappa, self.G_ads
        p.nu_l, p.nu_v = self.nu_l, self.nu_v
        p.rho_l, p.rho_v = self.rho_l, self.rho_v
        p.rho_ref = self.rho_v if self.storage != "fp64" else 0.0
        p.bc[2][0] = p.bc[2][1] = L.LBM_BC_WALL
        if self.r_cyl > 0:
            p.cylinder = 1
            p.cyl_y, p.cyl_z, p.cyl_r = self.ny / 2.0, 0.5 + self.r_cyl, self.r_cyl
        p.reduce_every = 500
        return p

    def centre(self):
        top = 0.5 + (2.0 * self.r_cyl if self.r_cyl > 0 else 0.0)
        return self.nx / 2.0, self.ny / 2.0, top + self.gap + self.R0


def capillary_time(rho_l, R0, gamma):
    """Inertia-capillary time tau = sqrt(rho_l R0^3 / gamma) (Eq. (23))."""
    return math.sqrt(rho_l * R0 ** 3 / gamma)


def run_impact(case, steps, every=50, stream=None, log=None, keep_going=False, reach=2,
               surface_top=None):
    """Run an impact case and sample the device diagnostics every `every` steps.

    Contact (Sec. IV B: from first touching the surface to bouncing off) is taken as liquid
    within `reach` lattice steps of a solid node (wall or cylinder) along a lattice
    velocity, in the planes z < surface_top (default: the lower half of the box, so that a
    rebounding droplet near the top wall does not count): on strongly hydrophobic walls the
    first fluid layer holds vapour even under a resting droplet, so liquid next to a solid
    node (reach 1) is not a usable criterion there.

    Returns a dict with the series t, spreading diameter D_f (largest over the planes
    z = 1 .. reach), liquid nodes in contact, liquid volume, liquid nodes in the planes
    z = 1..8, the lowest liquid plane and the liquid centroid height, plus t_contact (first
    sample in contact) and t_detach (first later sample out of contact, None while still in
    contact), and the total mass at the start (mass0) and the end (mass).
    keep_going: sample until `steps` even after the droplet has left the solid."""
    p = case.params()
    if stream is not None:
        p.stream = stream
    thr = 0.5 * (case.rho_v + case.rho_l)
    top = case.nz // 2 if surface_top is None else surface_top
    out = dict(t=[], D_f=[], wetted=[], volume=[], low=[], z_min=[], z_c=[],
               t_contact=None, t_detach=None)
    with L.Lattice(p, use_torch_stream=stream is None) as lat:
        cx, cy, cz = case.centre()
        lat.init_droplet(cx, cy, cz, case.R0, case.W, case.rho_l, case.rho_v, 0.0, 0.0, -case.U)
        out["mass0"] = float(lat.moments(want=("totals",))["totals"][0])
        done = 0
        while True:
            cz_, wz, vol = lat.liquid_stats(thr, case.rho_v, case.rho_l, reach)
            wet = int(wz[:top].sum())
            out["t"].append(done)
            out["D_f"].append(max(spreading_diameter(cz_, z) for z in range(1, reach + 1)))
            out["wetted"].append(wet)
            out["volume"].append(vol)
            out["low"].append([int(v) for v in cz_[1:9]])
            nzl = np.nonzero(cz_)[0]
            out["z_min"].append(int(nzl.min()) if nzl.size else -1)
            zz = np.arange(cz_.size)
            out["z_c"].append(float((zz * cz_).sum() / max(cz_.sum(), 1)))
            touching = wet > 0
            if touching and out["t_contact"] is None:
                out["t_contact"] = done
            if not touching and out["t_contact"] is not None and out["t_detach"] is None:
                out["t_detach"] = done
            if log:
                log(done, wet, vol, out["D_f"][-1])
            if (out["t_detach"] is not None and not keep_going) or done >= steps:
                break
            n = min(every, steps - done)
            lat.step(n)
            done += n
        out["mass"] = float(lat.moments(want=("totals",))["totals"][0])
    return out
