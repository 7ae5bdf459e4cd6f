"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no lattice-Boltzmann arithmetic: only the workload descriptions (the
physical parameters of each synthetic case, as plain numbers) and seeded random arrays.
Both the HIP path and the CPU oracle translate a Workload into their own parameters.
"""
from dataclasses import dataclass, field, replace

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    Q: int
    nx: int
    ny: int
    nz: int
    eos: str = "cs"                   # "cs" (Carnahan-Starling) or "piecewise"
    cs_a: float = 0.5
    cs_b: float = 4.0
    cs_R: float = 1.0
    T_over_Tc: float = 0.7
    G: float = -1.0
    sigma: float = 0.1
    kappa: float = 0.0
    G_ads: float = 0.0
    nu: float = 0.1
    rates: str = "paper"              # "paper": s2b = s3b = 0.6, others 1.2; "unit": all 1
    walls: tuple = ()                 # e.g. ("z_lo", "z_hi")
    cylinder: tuple = None            # (y_c, z_c, r) of an x-aligned cylinder
    wall_psi: str = "mirror"          # psi at solid neighbours: mirror, node, fluid_mean, zero
    R: float = 8.0                    # droplet radius
    W: float = 5.0                    # interface width
    centre: tuple = None              # None: box centre (nx/2, ny/2, nz/2)
    U: tuple = (0.0, 0.0, 0.0)        # droplet velocity
    noise: float = 0.0                # relative density noise in the interface band
    seed: int = 0
    steps: int = 100
    extra: dict = field(default_factory=dict)

    def with_(self, **kw):
        return replace(self, **kw)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    @property
    def nodes(self):
        return self.nx * self.ny * self.nz

    def droplet_centre(self):
        if self.centre is not None:
            return self.centre
        return (self.nx // 2, self.ny // 2, self.nz // 2)


# Static droplet, 32^3 periodic D3Q19, CS EOS at 0.7 T_c, radius 8, width 5, no noise;
# all relaxation rates 1 except the viscous one (nu = 0.1). The small parity case.
STATIC_32 = Workload("static-droplet-32^3-d3q19", 19, 32, 32, 32, T_over_Tc=0.7,
                     rates="unit", R=8.0, W=5.0, steps=200)

# Static droplet for the Laplace law, 256^3 periodic D3Q19, CS EOS at 0.5 T_c, +-1 % density
# noise in the interface band. The headline throughput workload. Non-viscous rates 1: with
# the paper's rate set (bulk 0.6, others 1.2) droplets of R >= 30 at this temperature blow up
# after 1100-1500 steps (the liquid density climbs to the psi^2 = 0 bound near 0.59), with
# rates 1 they run. sigma = 0.1153: the value at which a flat interface of this EOS and rate
# set settles on the Maxwell densities (0.1 leaves the vapour 88 % below them).
LAPLACE_256 = Workload("laplace-droplet-256^3-d3q19", 19, 256, 256, 256, T_over_Tc=0.5,
                       rates="unit", sigma=0.1153, R=40.0, W=5.0, noise=0.01, seed=0,
                       steps=5000)

# Droplet impact on a flat wall: 384x384x192, walls at z = 0 and z = 191, 90 degree
# contact angle (G_ads = 0: a neutral wall with psi at the wall read at its mirror image),
# R = 40 at z = 50, U_z = -0.05, CS EOS at 0.55 T_c, nu = 0.001 (Re = 2000); sigma = 0.119
# puts a flat interface of this EOS and the paper's rates on the Maxwell densities.
IMPACT_384 = Workload("impact-384x384x192-d3q19", 19, 384, 384, 192, T_over_Tc=0.55,
                      rates="paper", sigma=0.119, walls=("z_lo", "z_hi"), R=40.0, W=5.0,
                      centre=(192, 192, 50), U=(0.0, 0.0, -0.05), nu=0.001, steps=20000)

# D3Q27 impact on a wall with an x-aligned cylinder: 320x256x192, CS at 0.6 T_c, sigma =
# 0.1186 (a flat interface of this EOS and rate set settles on the Maxwell densities). The
# configuration's 160 degree wall: a sessile drop (R = 25) stands at 143.4 degrees for
# G_ads = 0.24, 157.6 at 0.27, 165.6 at 0.28 and leaves the wall from 0.32, so G_ads = 0.273.
CYLINDER_D3Q27 = Workload("cylinder-impact-320x256x192-d3q27", 27, 320, 256, 192,
                          T_over_Tc=0.6, rates="paper", sigma=0.1186, walls=("z_lo", "z_hi"),
                          cylinder=(128.0, 20.0, 20.0), R=30.0, W=5.0,
                          centre=(160, 128, 80), U=(0.0, 0.0, -0.04), G_ads=0.273, steps=15000)


def random_fields(shape, seed, rho_lo=0.02, rho_hi=0.4, u_amp=0.02):
    """Uniform random density in [rho_lo, rho_hi) and velocity components in
    [-u_amp, u_amp), float64, from numpy's PCG64 with the given seed."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(rho_lo, rho_hi, shape)
    u = rng.uniform(-u_amp, u_amp, (3,) + tuple(shape))
    return rho, u


def random_factors(Q, shape, seed, amp=0.05):
    """Multiplicative perturbations 1 + amp U(-1, 1) for Q populations per node."""
    rng = np.random.default_rng(seed + 7919)
    return 1.0 + amp * rng.uniform(-1.0, 1.0, (Q,) + tuple(shape))


def serving_trace(n_requests=256, rate_per_s=4.0, seed=2306, L_lo=64, L_hi=192,
                  steps_lo=2000, steps_hi=8000):
    """Poisson arrivals of droplet-impact requests: cubic box L log-uniform in
    [L_lo, L_hi], contact angle in [60, 160] degrees, impact speed in [0.02, 0.06],
    radius L/6, steps uniform in [steps_lo, steps_hi]."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, n_requests)
    t = np.cumsum(gaps) - gaps[0]
    L = np.rint(np.exp(rng.uniform(np.log(L_lo), np.log(L_hi), n_requests))).astype(int)
    theta = rng.uniform(60.0, 160.0, n_requests)
    U = rng.uniform(0.02, 0.06, n_requests)
    steps = rng.integers(steps_lo, steps_hi + 1, n_requests)
    return [dict(id=i, t_arrival=float(t[i]), L=int(L[i]), theta=float(theta[i]),
                 U=float(U[i]), R=float(L[i]) / 6.0, steps=int(steps[i]))
            for i in range(n_requests)]
