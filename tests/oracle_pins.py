"""Pin checks of the oracle step, written as functions that return an error measure so the
planted-mistake tests can run them against a deliberately broken oracle.

Each check compares the oracle with something the paper or the mathematics fixes:
closed-form textbook BGK, exact conservation laws, polynomial exactness of the force
stencil, the velocity-space (dense Lambda) form of the same collision, and fixed points.
"""
import numpy as np

from oracle import eos, lbm
from oracle.lattice import lattice


def _fake_macro(P, rng, n=6):
    """Random post-streaming populations on an n^3 periodic box and their macroscopic
    fields, with non-trivial forces."""
    lat = P.lat
    f = lat.omega.reshape(-1, 1, 1, 1) * rng.uniform(0.2, 0.5, (1, n, n, n)) \
        * (1 + 0.2 * rng.uniform(-1, 1, (lat.Q, n, n, n)))
    solid = np.zeros((n, n, n), dtype=bool)
    return f, solid


def conservation_error(Q=19, seed=0):
    """Collision conserves mass exactly and adds exactly F to the momentum, for arbitrary
    relaxation rates (Eq. (8) with Eqs. (14)-(15) and (B1))."""
    rng = np.random.default_rng(seed)
    P = lbm.Params(Q=Q, nx=6, ny=6, nz=6, eos=eos.CarnahanStarling(0.5, 4, 1, 0.6),
                   sigma=0.11, kappa=0.4, nu_l=0.07, s0=0.7, s1=1.6, s2b=0.8, s3=1.4,
                   s3b=0.9, s4=1.1, s4b=1.3, s5=0.95, s6=1.7)
    f, solid = _fake_macro(P, rng)
    mac = lbm.macroscopic(f, P, solid)
    fs = lbm.collide(f, P, mac)
    lat = P.lat
    e = lat.e.T.astype(float)
    dm = np.abs(fs.sum(0) - f.sum(0)).max()
    j0 = np.tensordot(e, f, axes=(1, 0))
    j1 = np.tensordot(e, fs, axes=(1, 0))
    dj = np.abs(j1 - j0 - mac["F"]).max()
    return max(dm, dj)


def srt_bgk_error(Q=27, seed=1):
    """With all rates equal and sigma = kappa = 0 the collision is BGK with Guo forcing
    (Sec. II B): f* = f - s (f - f^eq) + (1 - s/2) F_i, f^eq of Eq. (5), F_i of Eq. (6).
    For D3Q19 only moments 0..15 of the two forms coincide; those are compared."""
    rng = np.random.default_rng(seed)
    s = 1.37
    P = lbm.Params(Q=Q, nx=6, ny=6, nz=6, eos=eos.CarnahanStarling(0.5, 4, 1, 0.6),
                   sigma=0.0, kappa=0.0, nu_l=(1 / s - 0.5) / 3, s0=s, s1=s, s2b=s, s3=s,
                   s3b=s, s4=s, s4b=s, s5=s, s6=s)
    f, solid = _fake_macro(P, rng)
    mac = lbm.macroscopic(f, P, solid)
    fs = lbm.collide(f, P, mac)
    lat = P.lat
    err = 0.0
    idx = [(1, 2, 3), (0, 4, 5), (5, 0, 2)]
    for (z, y, x) in idx:
        fn = f[:, z, y, x]
        u = mac["u"][:, z, y, x]
        F = mac["F"][:, z, y, x]
        rho = fn.sum()
        bgk = fn - s * (fn - lat.feq_hermite(rho, u)) + (1 - s / 2) * lat.guo_force(u, F)
        got = fs[:, z, y, x]
        if Q == 27:
            err = max(err, np.abs(got - bgk).max())
        else:
            err = max(err, np.abs((lat.M @ got)[:16] - (lat.M @ bgk)[:16]).max())
    return err


def dense_lambda_error(Q=19, seed=2):
    """The moment-space collision (Eq. (8)) equals the velocity-space form of Eq. (7) with
    Lambda = M^-1 S M, on an 8^3 box with walls, a cylinder and wetting."""
    rng = np.random.default_rng(seed)
    P = lbm.Params(Q=Q, nx=8, ny=8, nz=8, eos=eos.CarnahanStarling(0.5, 4, 1, 0.6),
                   sigma=0.1, kappa=0.3, G_ads=0.1, nu_l=0.05,
                   walls={"z_lo": True, "z_hi": True}, cylinder=(3.0, 1.0, 1.5))
    solid = lbm.solid_mask(P)
    rho = rng.uniform(0.01, 0.45, P.shape)
    u = rng.uniform(-0.03, 0.03, (3,) + P.shape)
    f = lbm.equilibrium_populations(P, rho, u, solid)
    f = f * (1 + 0.05 * rng.uniform(-1, 1, f.shape))
    a = lbm.step(f, P, solid)
    b = lbm.step(f, P, solid, dense_lambda=True)
    return np.abs(a - b).max()


def stencil_polynomial_error(Q=19):
    """Taylor forms of Eq. (B4): for psi quadratic, Q_ab = (kappa G/12) psi (lap psi d_ab +
    2 d_a d_b psi); for psi cubic, F_int = -G psi (grad psi + (1/6) grad lap psi). These
    hold exactly for polynomials of those degrees (fourth-order isotropy of w)."""
    P = lbm.Params(Q=Q, nx=12, ny=12, nz=12, eos=eos.CarnahanStarling(0.5, 4, 1, 0.6),
                   G=-1.0, kappa=0.7)
    z, y, x = np.meshgrid(*(np.arange(12.0),) * 3, indexing="ij")
    solid = np.zeros(P.shape, dtype=bool)
    inner = (slice(2, 10),) * 3
    err = 0.0
    # quadratic psi: H symmetric, g, c
    H = np.array([[0.02, 0.005, -0.003], [0.005, -0.01, 0.004], [-0.003, 0.004, 0.015]])
    g = np.array([0.01, -0.02, 0.03])
    X = np.stack([x, y, z])
    psi = 1.0 + np.einsum("a...,a->...", X, g) + 0.5 * np.einsum("a...,ab,b...->...", X, H, X)
    _, _, Qab, _ = lbm.forces(psi, solid, P)
    lap = np.trace(H)
    names = {"xx": (0, 0), "yy": (1, 1), "zz": (2, 2), "xy": (0, 1), "xz": (0, 2), "yz": (1, 2)}
    for k, (a, b) in names.items():
        want = P.kappa * P.G / 12.0 * psi * (lap * (a == b) + 2 * H[a, b])
        err = max(err, np.abs(Qab[k][inner] - want[inner]).max())
    # cubic psi = 1 + g.x + c3 x^3 + c4 x y z + c5 z^2 y
    c3, c4, c5 = 1e-4, 2e-4, -1.5e-4
    psi = 1.0 + g[0] * x + g[1] * y + g[2] * z + c3 * x ** 3 + c4 * x * y * z + c5 * z * z * y
    grad = np.stack([g[0] + 3 * c3 * x ** 2 + c4 * y * z,
                     g[1] + c4 * x * z + c5 * z * z,
                     g[2] + c4 * x * y + 2 * c5 * z * y])
    # lap psi = 6 c3 x + 2 c5 y ; grad lap = (6 c3, 2 c5, 0)
    glap = np.stack([np.full_like(x, 6 * c3), np.full_like(x, 2 * c5), np.zeros_like(x)])
    F_int, _, _, _ = lbm.forces(psi, solid, P)
    want = -P.G * psi * (grad + glap / 6.0)
    err = max(err, np.abs(F_int[(slice(None),) + inner] - want[(slice(None),) + inner]).max())
    return err


def fixed_point_error(Q=19):
    """A uniform state is a fixed point of the whole step: m = m^eq and no force. At rest
    and with a constant velocity in a periodic box."""
    P = lbm.Params(Q=Q, nx=5, ny=4, nz=6, eos=eos.CarnahanStarling(0.5, 4, 1, 0.6),
                   sigma=0.1, kappa=0.5, nu_l=0.08)
    err = 0.0
    for U in ((0.0, 0.0, 0.0), (0.03, -0.02, 0.01)):
        rho = np.full(P.shape, 0.37)
        u = np.array([np.full(P.shape, c) for c in U])
        f = lbm.equilibrium_populations(P, rho, u)
        g = lbm.run(f, P, 3)
        err = max(err, np.abs(g - f).max())
    return err


def neutral_wall_error(Q=19):
    """With G_ads = 0 a uniform fluid next to a wall feels no force (the solid-neighbour
    reading of psi), and it stays at rest."""
    P = lbm.Params(Q=Q, nx=4, ny=4, nz=7, eos=eos.CarnahanStarling(0.5, 4, 1, 0.6),
                   sigma=0.1, kappa=0.3, nu_l=0.08, walls={"z_lo": True, "z_hi": True})
    solid = lbm.solid_mask(P)
    rho = np.full(P.shape, 0.3)
    u = np.zeros((3,) + P.shape)
    f = lbm.equilibrium_populations(P, rho, u, solid)
    g = lbm.run(f, P, 3, solid)
    return np.abs(g - f).max()


def periodic_momentum_drift(Q=19, steps=20):
    """Total mass and momentum of a fully periodic box are constant: the pairwise
    interaction force of Eq. (16) sums to zero over the box (antisymmetry)."""
    P = lbm.Params(Q=Q, nx=10, ny=9, nz=8, eos=eos.CarnahanStarling(0.5, 4, 1, 0.7),
                   sigma=0.1, kappa=0.4, nu_l=0.1)
    rng = np.random.default_rng(5)
    rho = rng.uniform(0.02, 0.35, P.shape)
    u = rng.uniform(-0.02, 0.02, (3,) + P.shape)
    f = lbm.equilibrium_populations(P, rho, u)
    t0 = lbm.totals(f, P)
    f = lbm.run(f, P, steps)
    t1 = lbm.totals(f, P)
    return max(abs(t1[0] - t0[0]) / t0[0], np.abs(t1[1:4] - t0[1:4]).max())


def wall_mass_drift(Q=19, steps=20):
    """Halfway bounce-back conserves mass exactly with walls, a cylinder and wetting."""
    P = lbm.Params(Q=Q, nx=10, ny=9, nz=10, eos=eos.CarnahanStarling(0.5, 4, 1, 0.7),
                   sigma=0.1, kappa=0.2, G_ads=0.15, nu_l=0.1,
                   walls={"z_lo": True, "z_hi": True, "y_lo": True}, cylinder=(4.0, 2.0, 2.0))
    solid = lbm.solid_mask(P)
    rng = np.random.default_rng(6)
    rho = rng.uniform(0.02, 0.35, P.shape)
    u = rng.uniform(-0.02, 0.02, (3,) + P.shape)
    f = lbm.equilibrium_populations(P, rho, u, solid)
    m0 = lbm.totals(f, P, solid)[0]
    f = lbm.run(f, P, steps, solid)
    return abs(lbm.totals(f, P, solid)[0] - m0) / m0


def planar_coexistence(Q=19, steps=4000):
    """Flat liquid slab with the piecewise EOS of Sec. III A (G = -1, sigma = 0.1): returns
    the simulated (rho_v, rho_l); the paper reports they reproduce 0.001 and 1 (Fig. 1)."""
    n = 200
    P = lbm.Params(Q=Q, nx=1, ny=1, nz=n, eos=eos.Piecewise.paper_default(), G=-1.0,
                   sigma=0.1, kappa=0.0, nu_l=0.1)
    zz = np.arange(n)
    rho = 0.5 * 1.001 + 0.5 * 0.999 * np.tanh(2.0 * np.minimum(zz - 50, 150 - zz) / 5.0)
    rho = rho.reshape(n, 1, 1)
    f = lbm.equilibrium_populations(P, rho, np.zeros((3, n, 1, 1)))
    f = lbm.run(f, P, steps)
    r = f.sum(0)[:, 0, 0]
    return r[0], r[n // 2]


def laplace_cylinders(kappa, n=40, steps=1500, radii=(7, 10, 13)):
    """Quasi-2D Laplace test (nz = 1, a liquid cylinder along z): returns the least-squares
    slope and intercept of dp = p_in - p_out against 1/R. In two dimensions Laplace's law
    reads dp = gamma / R, so the slope is the surface tension."""
    cs = eos.CarnahanStarling(0.5, 4.0, 1.0, 0.7)
    rv, rl = eos.maxwell_densities(cs, 1e-9, 0.7)
    dps = []
    for R in radii:
        P = lbm.Params(Q=19, nx=n, ny=n, nz=1, eos=cs, G=-1.0, sigma=0.1, kappa=kappa,
                       nu_l=0.1)
        rho, u = lbm.droplet_fields(P, n / 2 - 0.5, n / 2 - 0.5, 0.0, R, 5.0, rl, rv)
        f = lbm.run(lbm.equilibrium_populations(P, rho, u), P, steps)
        _, _, p, _ = lbm.moments(f, P)
        dps.append(p[0, n // 2, n // 2] - p[0, 0, 0])
    A = np.vstack([1.0 / np.array(radii, float), np.ones(len(radii))]).T
    (slope, icpt), res, _, _ = np.linalg.lstsq(A, np.array(dps), rcond=None)
    r2 = 1.0 - res[0] / np.sum((np.array(dps) - np.mean(dps)) ** 2) if len(res) else 1.0
    return slope, icpt, r2
