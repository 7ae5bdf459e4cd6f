"""Linear (von Neumann) stability of the time step around a uniform state.

TEST INFRASTRUCTURE: an analysis built from the oracle's moment-space pieces (M, M^-1, the
equilibrium moments of Eq. (14)/(C5), the forcing moments of Eq. (15)/(C6), the rates of
Eq. (12)/(C3)). It answers whether a small perturbation of a uniform fluid (density rho0,
velocity u0) grows under the step of Sec. II A with the force of Eq. (16) and the source
terms of Eq. (B1).

Linearisation. Around a uniform state psi is uniform, so F = 0 there; a density
perturbation drho(x) changes psi by psi'(rho0) drho and
  dF(x)    = -G psi0 psi' sum_i w_i drho(x + e_i) e_i                      (Eq. (16))
  dQ_ab(x) = kappa (G/2) psi0 psi' sum_i w_i (drho(x + e_i) - drho(x)) e_ia e_ib   (Eq. (B2))
while |F_int|^2/psi^2 of Eq. (B1) is quadratic and drops out. With u = (j + F/2)/rho
(Eq. (10)), the collision of Eq. (8) and the pull f_i(x, t+1) = f*_i(x - e_i, t), a Fourier
mode exp(i k.x) of the populations is advanced by the Q x Q matrix
  A(k) = E(k)* M^-1 [ (I - S) M + S dm^eq/df + (I - S/2) dF~'/df ],   E(k) = diag(exp(i k.e_i))
whose spectral radius, maximised over k, is the growth factor per step. The derivatives of
m^eq with respect to (rho, u) are taken by central differences, exact for these polynomials
(degree <= 2 in each variable); F~ is bilinear in (F, u) and F = 0 at the base state, so
dF~ = F~(dF, u0).
"""
import numpy as np

from oracle.lattice import CS2, lattice

PAPER_RATES = dict(s2b=0.6, s3=1.2, s3b=0.6, s4=1.2, s4b=1.2, s5=1.2, s6=1.2)


def rate_vector(Q, nu, rates):
    """Diagonal of S for kinematic viscosity nu (s_nu from nu = c_s^2 (1/s_nu - 1/2))."""
    s_nu = 1.0 / (nu / CS2 + 0.5)
    r = dict(PAPER_RATES, **rates)
    return lattice(Q).relaxation_rates(1.0, 1.0, s_nu, r["s2b"], r["s3"], r["s3b"], r["s4"],
                                       r["s4b"], r["s5"], r["s6"])


def _meq_jacobian(lat, rho0, u0, h=1e-3):
    x0 = np.array([rho0, *u0], dtype=np.float64)
    J = np.zeros((lat.Q, 4))
    for a in range(4):
        xp, xm = x0.copy(), x0.copy()
        xp[a] += h
        xm[a] -= h
        J[:, a] = (lat.meq(*xp) - lat.meq(*xm)) / (2.0 * h)
    return J


def step_matrices(Q, ks, S, rho0=1.0, u0=(0.0, 0.0, 0.0), g_psi_dpsi=0.0, kappa=0.0):
    """A(k) for every wave vector in ks (K, 3): array (K, Q, Q). g_psi_dpsi = G psi0 psi'(rho0)
    (0 where psi does not depend on rho, e.g. the liquid branch of the piecewise EOS)."""
    lat = lattice(Q)
    e = lat.e.astype(np.float64)
    w = lat.w
    u0 = np.asarray(u0, dtype=np.float64)
    ks = np.atleast_2d(np.asarray(ks, dtype=np.float64))
    ph = np.exp(1j * ks @ e.T)                                     # (K, Q): exp(i k.e_i)
    g = -g_psi_dpsi * np.einsum("kq,qa->ka", ph * w, e)            # dF = g drho, (K, 3)
    qf = kappa * 0.5 * g_psi_dpsi
    pairs = dict(xx=(0, 0), yy=(1, 1), zz=(2, 2), xy=(0, 1), xz=(0, 2), yz=(1, 2))
    q = {n: qf * np.einsum("kq,q->k", (ph - 1.0) * w, e[:, a] * e[:, b]) for n, (a, b) in pairs.items()}
    tau_nu, tau_e = 1.0 / S[4] - 0.5, 1.0 / S[7] - 0.5
    b = np.zeros((len(ks), Q), dtype=complex)                     # Eq. (B1) Q_ab terms per drho
    b[:, 4] = -q["xy"] / tau_nu
    b[:, 5] = -q["xz"] / tau_nu
    b[:, 6] = -q["yz"] / tau_nu
    b[:, 7] = 4.0 * (q["xx"] + q["yy"] + q["zz"]) / (5.0 * tau_e)
    b[:, 8] = -(q["xx"] - q["yy"]) / tau_nu
    b[:, 9] = -(q["xx"] - q["zz"]) / tau_nu
    # dF~/dF at u0 (Q x 3): F~ is linear in F
    PhiF = np.stack([lat.forcing_moments(*np.eye(3)[a], *u0) for a in range(3)], axis=1)
    J = _meq_jacobian(lat, rho0, u0)
    ones = np.ones(Q)
    # du = (E^T df + (g/2 - u0) drho) / rho0  ->  (K, 3, Q)
    Du = (e.T[None, :, :] + (0.5 * g - u0)[:, :, None] * ones[None, None, :]) / rho0
    dmeq = J[:, :1][None] * ones[None, None, :] + np.einsum("qa,kaj->kqj", J[:, 1:], Du)
    forcing = (np.einsum("qa,ka->kq", PhiF, g) + b)[:, :, None] * ones[None, None, :]
    inner = ((1.0 - S)[:, None] * lat.M)[None] + S[None, :, None] * dmeq \
        + (1.0 - 0.5 * S)[None, :, None] * forcing
    return np.conj(ph)[:, :, None] * np.einsum("ij,kjl->kil", lat.Minv, inner)


def k_grid(n):
    """Wave vectors 2 pi (a, b, c) / n of an n^3 periodic box."""
    k1 = 2.0 * np.pi * np.arange(n) / n
    return np.stack(np.meshgrid(k1, k1, k1, indexing="ij"), -1).reshape(-1, 3)


def max_growth(Q, nu, rates=None, n=12, **kw):
    """Largest |eigenvalue| of A(k) over the wave vectors of an n^3 box, and where."""
    S = rate_vector(Q, nu, rates or {})
    ks = k_grid(n)
    A = step_matrices(Q, ks, S, **kw)
    rad = np.abs(np.linalg.eigvals(A)).max(axis=1)
    i = int(np.argmax(rad))
    return float(rad[i]), ks[i]
