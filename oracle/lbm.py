"""One time step of the non-orthogonal MRT-LBM with the pseudopotential multiphase model.

TEST INFRASTRUCTURE ONLY (see the package docstring).

State convention: ``f`` has shape (Q, nz, ny, nx), x fastest, and holds the populations
f_bar(x, t) after streaming (the quantities whose sums give rho and rho u, Sec. II A,
Eq. (10)). ``step`` performs, in the paper's order:

1. rho = sum_i f_bar_i                                         Sec. II A, Eq. (10)
2. psi(rho) from the equation of state (all nodes first)      Sec. II C
3. F_int                                                       Sec. II C, Eq. (16)
   F_ads (wetting)                                             Sec. III E, Eq. (22)
   Q_ab  (surface-tension tuning)                              Appendix B, Eq. (B2)
4. u = (sum_i f_bar_i e_i + F/2) / rho                         Sec. II A, Eq. (10)
5. m = M f_bar, m^eq(rho,u), F~(F,u)                           Sec. II B, Eqs. (13)-(15); App. C
6. F~' with the sigma and Q_ab modifications                   Appendix B, Eq. (B1)
7. m* = m - S (m - m^eq) + (I - S/2) F~'                       Sec. II A, Eq. (8)
8. f_bar* = M^-1 m*                                            Sec. II A, below Eq. (8)
9. f_bar_i(x + e_i, t+1) = f_bar*_i(x, t)                      Sec. II A, Eq. (9)
   with halfway bounce-back at solid nodes.

Readings taken where the paper is silent (each is listed with its reason in the design notes):
* walls are halfway bounce-back: a population that would stream into a solid node returns
  to its origin in the opposite direction at the next time level; solid nodes carry no
  populations (they are held at 0 here);
* psi at a solid neighbour, in F_int and Q_ab (not specified by the paper), follows
  Params.wall_psi: "node" (psi of the evaluating fluid node), "fluid_mean"
  (the w-weighted mean of psi over the node's fluid neighbours), "zero", or "mirror"
  (psi at x + e' where e' is e_i without the components along which the axis neighbour
  of x is solid: for a flat wall the mirror image of x + e_i across the wall; psi of the
  node where e' = 0 or x + e' is solid; the default: of these readings it alone makes
  G_ads = 0 neutral and G_ads = 0.23 about 157 degrees, the two statements of Sec. III E);
* the s_e of Eq. (B1) is the bulk rate s_2b of Eq. (12);
* |F_int|^2 / psi^2 where psi = 0 is its limit G^2 |sum_i w_i psi(x+e_i) e_i|^2;
* the kinematic viscosity may vary linearly with rho (Sec. IV A, Eq. (24)); s_nu follows
  from nu = c_s^2 (1/s_nu - 1/2) (Sec. II B, below Eq. (12)).
"""
from dataclasses import dataclass, field

import numpy as np

from . import eos as eos_mod
from .lattice import CS2, lattice
from .splitmix import uniform_array


@dataclass
class Params:
    Q: int
    nx: int
    ny: int
    nz: int
    eos: object                       # eos.Piecewise or eos.CarnahanStarling
    G: float = -1.0                   # interaction strength, Eq. (16)
    sigma: float = 0.0                # mechanical-stability parameter, Eq. (B1)
    kappa: float = 0.0                # surface-tension tuning, Eq. (B2)
    G_ads: float = 0.0                # fluid-solid interaction strength, Eq. (22)
    nu_l: float = 0.1                 # kinematic viscosity (liquid), Eq. (24)
    nu_v: float = None                # vapour viscosity; None means uniform nu_l
    rho_l: float = 1.0                # densities that anchor Eq. (24)
    rho_v: float = 0.001
    s0: float = 1.0
    s1: float = 1.0
    s2b: float = 0.6
    s3: float = 1.2
    s3b: float = 0.6
    s4: float = 1.2
    s4b: float = 1.2
    s5: float = 1.2
    s6: float = 1.2
    walls: dict = field(default_factory=dict)   # {'z_lo': True, 'z_hi': True, ...}
    cylinder: tuple = None            # x-aligned: (y_c, z_c, radius)
    body_force: tuple = (0.0, 0.0, 0.0)
    wall_psi: str = "mirror"          # psi at solid neighbours: node|fluid_mean|zero|mirror

    @property
    def lat(self):
        return lattice(self.Q)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)


def s_nu_of(nu):
    """Sec. II B: nu = c_s^2 (1/s_nu - 1/2)  =>  s_nu = 1 / (nu / c_s^2 + 1/2)."""
    return 1.0 / (nu / CS2 + 0.5)


def solid_mask(P):
    """Boolean (nz, ny, nx): wall layers at the domain faces and an x-aligned cylinder."""
    z, y, x = np.meshgrid(np.arange(P.nz), np.arange(P.ny), np.arange(P.nx), indexing="ij")
    s = np.zeros(P.shape, dtype=bool)
    for axis, coord, n in (("x", x, P.nx), ("y", y, P.ny), ("z", z, P.nz)):
        if P.walls.get(axis + "_lo"):
            s |= coord == 0
        if P.walls.get(axis + "_hi"):
            s |= coord == n - 1
    if P.cylinder is not None:
        yc, zc, r = P.cylinder
        s |= (y - yc) ** 2 + (z - zc) ** 2 <= r * r
    return s


def neighbour(a, e):
    """a(x + e) on the periodic lattice, for an array shaped (nz, ny, nx)."""
    return np.roll(a, shift=(-int(e[2]), -int(e[1]), -int(e[0])), axis=(0, 1, 2))


def mirror_psi(psi, solid, P, e):
    """psi at the image of the solid neighbour x + e under the "mirror" reading: drop
    every component of e along which the axis neighbour of x (one step in that component's
    direction) is solid; psi(x + e') if e' != 0 and x + e' is fluid, else psi(x)."""
    keep = []
    for a in range(3):
        if e[a] == 0:
            keep.append(np.zeros(psi.shape, dtype=bool))
        else:
            step = np.zeros(3, dtype=np.int64)
            step[a] = e[a]
            keep.append(~neighbour(solid, step))
    out = psi.copy()
    for kx in (0, 1):
        for ky in (0, 1):
            for kz in (0, 1):
                ep = np.array([e[0] * kx, e[1] * ky, e[2] * kz])
                if not ep.any():
                    continue
                sel = ((keep[0] == bool(kx)) & (keep[1] == bool(ky)) & (keep[2] == bool(kz))
                       & ~neighbour(solid, ep))
                out = np.where(sel, neighbour(psi, ep), out)
    return out


def wall_psi_values(psi, solid, P):
    """psi assigned to the solid neighbours of each node (Params.wall_psi): the node's own
    psi, 0, or sum_i w_i psi(x + e_i) / sum_i w_i over the fluid neighbours x + e_i of x
    (psi of the node where it has no fluid neighbour). None for the "mirror" reading,
    whose value depends on the link (mirror_psi)."""
    if P.wall_psi == "node":
        return psi
    if P.wall_psi == "zero":
        return np.zeros_like(psi)
    if P.wall_psi == "mirror":
        return None
    if P.wall_psi != "fluid_mean":
        raise ValueError("wall_psi must be node, fluid_mean, zero or mirror")
    lat = P.lat
    num = np.zeros(psi.shape)
    den = np.zeros(psi.shape)
    for i in range(1, lat.Q):
        fl = ~neighbour(solid, lat.e[i])
        num += lat.w[i] * np.where(fl, neighbour(psi, lat.e[i]), 0.0)
        den += lat.w[i] * fl
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(den > 0, num / np.where(den > 0, den, 1.0), psi)


def forces(psi, solid, P):
    """F_int (Eq. (16)), F_ads (Eq. (22)), Q_ab (Eq. (B2)) and |F_int|^2/psi^2 at every node.

    Returns (F_int (3,...), F_ads (3,...), Qab dict, phi)."""
    lat = P.lat
    psi_w = wall_psi_values(psi, solid, P)
    F_int = np.zeros((3,) + psi.shape)
    F_ads = np.zeros((3,) + psi.shape)
    Qab = {k: np.zeros(psi.shape) for k in ("xx", "yy", "zz", "xy", "xz", "yz")}
    S_int = np.zeros((3,) + psi.shape)      # sum_i w_i psi(x + e_i) e_i
    for i in range(1, lat.Q):
        e = lat.e[i]
        w = lat.w[i]
        nb_solid = neighbour(solid, e)
        pw = psi_w if psi_w is not None else mirror_psi(psi, solid, P, e)
        psi_nb = np.where(nb_solid, pw, neighbour(psi, e))
        for a in range(3):
            S_int[a] += w * psi_nb * e[a]
            F_ads[a] += -P.G_ads * psi * w * psi * nb_solid * e[a]
        d = psi_nb - psi
        ex, ey, ez = (float(c) for c in e)
        Qab["xx"] += w * d * ex * ex
        Qab["yy"] += w * d * ey * ey
        Qab["zz"] += w * d * ez * ez
        Qab["xy"] += w * d * ex * ey
        Qab["xz"] += w * d * ex * ez
        Qab["yz"] += w * d * ey * ez
    for a in range(3):
        F_int[a] = -P.G * psi * S_int[a]
    for k in Qab:
        Qab[k] = P.kappa * (P.G / 2.0) * psi * Qab[k]
    F2 = (F_int ** 2).sum(0)
    with np.errstate(divide="ignore", invalid="ignore"):
        phi = np.where(psi > 0, F2 / (psi * psi), P.G ** 2 * (S_int ** 2).sum(0))
    return F_int, F_ads, Qab, phi


def macroscopic(f, P, solid=None):
    """rho, psi, total force F, velocity u and the force-stencil terms at time t."""
    lat = P.lat
    if solid is None:
        solid = solid_mask(P)
    rho = f.sum(0)
    psi = np.where(solid, 0.0, eos_mod.psi(P.eos, np.where(solid, 0.0, rho), P.G))
    F_int, F_ads, Qab, phi = forces(psi, solid, P)
    F = F_int + F_ads + np.array(P.body_force, dtype=np.float64).reshape(3, 1, 1, 1)
    j = np.tensordot(lat.e.T.astype(np.float64), f, axes=(1, 0))    # sum_i f_i e_i, (3,...)
    with np.errstate(divide="ignore", invalid="ignore"):
        u = np.where(solid, 0.0, (j + 0.5 * F) / np.where(solid, 1.0, rho))
    return dict(rho=rho, psi=psi, F=F, F_int=F_int, F_ads=F_ads, Qab=Qab, phi=phi, u=u,
                solid=solid)


def relaxation_diagonal(P, rho):
    """Per-node diagonal of S, shape (Q, ...). s_nu may depend on rho through Eq. (24)."""
    lat = P.lat
    if P.nu_v is None or P.nu_v == P.nu_l:
        nu = np.full(rho.shape, P.nu_l)
    else:
        nu = P.nu_v + (P.nu_l - P.nu_v) * (rho - P.rho_v) / (P.rho_l - P.rho_v)
    s_nu = s_nu_of(nu)
    base = lat.relaxation_rates(P.s0, P.s1, 0.0, P.s2b, P.s3, P.s3b, P.s4, P.s4b, P.s5, P.s6)
    S = np.broadcast_to(base.reshape((lat.Q,) + (1,) * rho.ndim), (lat.Q,) + rho.shape).copy()
    for k in (4, 5, 6, 8, 9):
        S[k] = s_nu
    return S


def modified_forcing(P, mac, S):
    """F~' of Eq. (B1): F~ of Eq. (15)/(C6) with the sigma and Q_ab source terms added."""
    lat = P.lat
    F, u, Qab, phi, psi = mac["F"], mac["u"], mac["Qab"], mac["phi"], mac["psi"]
    Ft = lat.forcing_moments(F[0], F[1], F[2], u[0], u[1], u[2])
    tau_nu = 1.0 / S[4] - 0.5          # (s_nu^-1 - 0.5) dt, dt = 1
    tau_e = 1.0 / S[7] - 0.5           # (s_e^-1 - 0.5) dt with s_e = s_2b
    Ft[4] = Ft[4] - Qab["xy"] / tau_nu
    Ft[5] = Ft[5] - Qab["xz"] / tau_nu
    Ft[6] = Ft[6] - Qab["yz"] / tau_nu
    Ft[7] = (Ft[7] + 6.0 * P.sigma * phi / tau_e
             + 4.0 * (Qab["xx"] + Qab["yy"] + Qab["zz"]) / (5.0 * tau_e))
    Ft[8] = Ft[8] - (Qab["xx"] - Qab["yy"]) / tau_nu
    Ft[9] = Ft[9] - (Qab["xx"] - Qab["zz"]) / tau_nu
    return Ft


def collide(f, P, mac):
    """Moment-space collision, Eq. (8), then f_bar* = M^-1 m*. Returns f_bar* (Q, ...)."""
    lat = P.lat
    shape = f.shape[1:]
    rho, u = mac["rho"], mac["u"]
    S = relaxation_diagonal(P, rho)
    Ft = modified_forcing(P, mac, S)
    meq = lat.meq(rho, u[0], u[1], u[2])
    m = (lat.M @ f.reshape(lat.Q, -1)).reshape(f.shape)
    m_star = m - S * (m - meq) + (1.0 - S / 2.0) * Ft
    f_star = (lat.Minv @ m_star.reshape(lat.Q, -1)).reshape((lat.Q,) + shape)
    return np.where(mac["solid"], 0.0, f_star)


def collide_dense_lambda(f, P, mac):
    """The same collision written in velocity space with Lambda = M^-1 S M, Eq. (7):
    f* = f - Lambda (f - f^eq) + (I - Lambda/2) F_bar, f^eq = M^-1 m^eq, F_bar = M^-1 F~'.
    Only for a uniform S (no density-dependent viscosity)."""
    lat = P.lat
    rho, u = mac["rho"], mac["u"]
    S = relaxation_diagonal(P, rho)
    if not np.all(S == S.reshape(lat.Q, -1)[:, :1].reshape((lat.Q,) + (1,) * rho.ndim)):
        raise ValueError("dense-Lambda form needs a uniform relaxation matrix")
    Sd = S.reshape(lat.Q, -1)[:, 0]
    Lam = lat.Minv @ np.diag(Sd) @ lat.M
    Ft = modified_forcing(P, mac, S)
    feq = lat.Minv @ lat.meq(rho, u[0], u[1], u[2]).reshape(lat.Q, -1)
    Fbar = lat.Minv @ Ft.reshape(lat.Q, -1)
    ff = f.reshape(lat.Q, -1)
    out = ff - Lam @ (ff - feq) + (np.eye(lat.Q) - Lam / 2.0) @ Fbar
    return np.where(mac["solid"], 0.0, out.reshape(f.shape))


def stream(f_star, P, solid):
    """Eq. (9) with halfway bounce-back: f_i(x+e_i) = f*_i(x); if x+e_i is solid the
    population returns as f_opp(i)(x) = f*_i(x)."""
    lat = P.lat
    out = np.empty_like(f_star)
    for i in range(lat.Q):
        e = lat.e[i]
        out[i] = np.roll(f_star[i], shift=(int(e[2]), int(e[1]), int(e[0])), axis=(0, 1, 2))
    for i in range(lat.Q):
        hits = ~solid & neighbour(solid, lat.e[i])
        out[lat.opp[i]][hits] = f_star[i][hits]
    out[:, solid] = 0.0
    return out


def step(f, P, solid=None, dense_lambda=False):
    """Advance f_bar(x, t) to f_bar(x, t+1)."""
    if solid is None:
        solid = solid_mask(P)
    mac = macroscopic(f, P, solid)
    f_star = collide_dense_lambda(f, P, mac) if dense_lambda else collide(f, P, mac)
    return stream(f_star, P, solid)


def run(f, P, nsteps, solid=None):
    if solid is None:
        solid = solid_mask(P)
    for _ in range(nsteps):
        f = step(f, P, solid)
    return f


def equilibrium_populations(P, rho, u, solid=None):
    """f_bar = M^-1 m^eq(rho, u) on fluid nodes, 0 on solid nodes (initial state)."""
    lat = P.lat
    if solid is None:
        solid = solid_mask(P)
    meq = lat.meq(rho, u[0], u[1], u[2])
    f = (lat.Minv @ meq.reshape(lat.Q, -1)).reshape((lat.Q,) + rho.shape)
    return np.where(solid, 0.0, f)


def droplet_fields(P, cx, cy, cz, R, W, rho_in, rho_out, U=(0.0, 0.0, 0.0),
                   noise_amp=0.0, seed=0):
    """Initial density and velocity of a droplet (tanh profile of Sec. III A, Eq. (21), in
    radial form). The velocity U is carried by the liquid fraction
    phi = clamp((rho - rho_out) / (rho_in - rho_out), 0, 1) of the noise-free profile. Inside
    the band |r - R| < W the density is multiplied by 1 + a (2 U_n - 1) with U_n the
    SplitMix64 uniform of node n (n = x + nx (y + ny z))."""
    z, y, x = np.meshgrid(np.arange(P.nz), np.arange(P.ny), np.arange(P.nx), indexing="ij")
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2)
    rho0 = 0.5 * (rho_in + rho_out) - 0.5 * (rho_in - rho_out) * np.tanh(2.0 * (r - R) / W)
    phi = np.clip((rho0 - rho_out) / (rho_in - rho_out), 0.0, 1.0)
    u = np.array([U[0] * phi, U[1] * phi, U[2] * phi])
    if noise_amp != 0.0:
        un = uniform_array(seed, P.nx * P.ny * P.nz).reshape(P.shape)
        band = np.abs(r - R) < W
        rho0 = np.where(band, rho0 * (1.0 + noise_amp * (2.0 * un - 1.0)), rho0)
    return rho0, u


def moments(f, P, solid=None):
    """rho, u (with the F/2 shift) and the bulk pressure of Eq. (17) at time t."""
    mac = macroscopic(f, P, solid)
    p = eos_mod.bulk_pressure(mac["rho"], mac["psi"], P.G)
    return mac["rho"], mac["u"], p, mac


def totals(f, P, solid=None):
    """Mass, momentum (3) and kinetic energy summed over fluid nodes."""
    rho, u, _, mac = moments(f, P, solid)
    fl = ~mac["solid"]
    mass = rho[fl].sum()
    mom = [(rho * u[a])[fl].sum() for a in range(3)]
    ek = (0.5 * rho * (u ** 2).sum(0))[fl].sum()
    return np.array([mass] + mom + [ek])


def liquid_stats(f, P, threshold, rho_v, rho_l, solid=None, reach=1):
    """Liquid-phase diagnostics at time t (Sec. IV A spreading film, Sec. IV B contact time
    and liquid volume): liquid nodes (fluid, rho > threshold) per z plane, per z plane the
    liquid nodes with a solid node at x + k e_i for some lattice velocity e_i and
    1 <= k <= reach, and the liquid volume sum over fluid nodes of
    clamp((rho - rho_v) / (rho_l - rho_v), 0, 1)."""
    if solid is None:
        solid = solid_mask(P)
    rho = f.sum(0)
    liquid = ~solid & (rho > threshold)
    touches = np.zeros(P.shape, dtype=bool)
    for k in range(1, reach + 1):
        for e in P.lat.e[1:]:
            touches |= neighbour(solid, k * np.asarray(e))
    vol = np.clip((rho - rho_v) / (rho_l - rho_v), 0.0, 1.0)[~solid].sum()
    return (liquid.sum(axis=(1, 2)).astype(np.int64),
            (liquid & touches).sum(axis=(1, 2)).astype(np.int64), float(vol))
