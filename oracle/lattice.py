"""Lattice tables and the moment-space pieces of the non-orthogonal MRT-LBM.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Everything here is built from the paper's definitions, not from pre-computed tables:

* velocities        Sec. II A, Eq. (1) (D3Q27); Appendix C, Eq. (C1): D3Q19 = first 19
* weights           Sec. II A under Eq. (5) (D3Q27). The D3Q19 weights are not printed;
                    the reading used is omega = 1/3, 1/18, 1/36 (|e|^2 = 0, 1, 2), which is
                    what M^-1 m^eq(rho=1, u=0) of the printed D3Q19 model reproduces.
* raw moments       Sec. II A, Eq. (2): k_mnp = <f_i | e_ix^m e_iy^n e_iz^p>
* moment set        Sec. II B, Eq. (11) (27 moments); Appendix C, Eq. (C2) (19 moments)
* M                 row k of M holds the coefficients of moment k over the populations
* M^-1              exact rational inverse (Gauss-Jordan over fractions)
* S                 Sec. II B, Eq. (12); Appendix C, Eq. (C3)
* m^eq              Sec. II B, Eq. (14); Appendix C, Eq. (C5)
* F~                Sec. II B, Eq. (15); Appendix C, Eq. (C6)
* f^eq, Guo F_i     Sec. II A, Eqs. (5) and (6) (used only as cross-checks)
"""
from fractions import Fraction

import numpy as np

CS2 = 1.0 / 3.0  # lattice sound speed squared, c_s = 1/sqrt(3) (Sec. II A)

# Eq. (1): the D3Q27 velocities in the paper's order.
_EX27 = [0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1]
_EY27 = [0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, 1, -1, -1, 1, 1, -1, -1]
_EZ27 = [0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, 1, 1, -1, -1, -1, -1]

# Eq. (11): each moment as a linear combination of raw moments k_mnp, {(m,n,p): coeff}.
_MOMENTS27 = [
    {(0, 0, 0): 1},                                   # m0  k000
    {(1, 0, 0): 1}, {(0, 1, 0): 1}, {(0, 0, 1): 1},   # m1-3
    {(1, 1, 0): 1}, {(1, 0, 1): 1}, {(0, 1, 1): 1},   # m4-6
    {(2, 0, 0): 1, (0, 2, 0): 1, (0, 0, 2): 1},       # m7  k200+k020+k002
    {(2, 0, 0): 1, (0, 2, 0): -1},                    # m8  k200-k020
    {(2, 0, 0): 1, (0, 0, 2): -1},                    # m9  k200-k002
    {(1, 2, 0): 1}, {(1, 0, 2): 1}, {(2, 1, 0): 1},   # m10-12
    {(2, 0, 1): 1}, {(0, 1, 2): 1}, {(0, 2, 1): 1},   # m13-15
    {(1, 1, 1): 1},                                   # m16
    {(2, 2, 0): 1}, {(2, 0, 2): 1}, {(0, 2, 2): 1},   # m17-19
    {(2, 1, 1): 1}, {(1, 2, 1): 1}, {(1, 1, 2): 1},   # m20-22
    {(1, 2, 2): 1}, {(2, 1, 2): 1}, {(2, 2, 1): 1},   # m23-25
    {(2, 2, 2): 1},                                   # m26
]
# Eq. (C2): the D3Q19 moment set is m0..m15 of Eq. (11) followed by k220, k202, k022.
_Q19_FROM_Q27 = list(range(16)) + [17, 18, 19]


class Lattice:
    """One velocity set (Q = 19 or 27) with its moment-space matrices, all float64."""

    def __init__(self, Q):
        if Q not in (19, 27):
            raise ValueError("Q must be 19 or 27")
        self.Q = Q
        self.e = np.array([_EX27[:Q], _EY27[:Q], _EZ27[:Q]], dtype=np.int64).T  # (Q, 3)
        self.opp = np.array([self._opposite(i) for i in range(Q)])
        self.moment_defs = (_MOMENTS27 if Q == 27
                            else [_MOMENTS27[k] for k in _Q19_FROM_Q27])
        norm2 = (self.e ** 2).sum(1)
        if Q == 27:
            table = {0: Fraction(8, 27), 1: Fraction(2, 27), 2: Fraction(1, 54), 3: Fraction(1, 216)}
        else:
            table = {0: Fraction(1, 3), 1: Fraction(1, 18), 2: Fraction(1, 36)}
        self.omega_frac = [table[int(n)] for n in norm2]
        self.omega = np.array([float(x) for x in self.omega_frac])
        # Normalised weights of the interaction force, w = omega / c_s^2 (Eq. (16)).
        self.w = self.omega / CS2
        self.M_frac = self._build_M()
        self.Minv_frac = invert_exact(self.M_frac)
        self.M = np.array([[float(x) for x in row] for row in self.M_frac])
        self.Minv = np.array([[float(x) for x in row] for row in self.Minv_frac])

    def _opposite(self, i):
        target = [-c for c in self.e[i]]
        for j in range(self.Q):
            if list(self.e[j]) == target:
                return j
        raise AssertionError("velocity set is not symmetric")

    def _build_M(self):
        """M[k][i] = sum over (m,n,p) of coeff * e_ix^m e_iy^n e_iz^p  (Eq. (2) with Eq. (11))."""
        M = []
        for mdef in self.moment_defs:
            row = []
            for i in range(self.Q):
                ex, ey, ez = (int(c) for c in self.e[i])
                row.append(Fraction(sum(c * ex ** m * ey ** n * ez ** p
                                        for (m, n, p), c in mdef.items())))
            M.append(row)
        return M

    # ---- relaxation matrix -------------------------------------------------------------
    def relaxation_rates(self, s0, s1, s_nu, s2b, s3, s3b, s4, s4b, s5, s6):
        """Diagonal of S: Eq. (12) for D3Q27, Eq. (C3) for D3Q19 (s2 is s_nu)."""
        if self.Q == 27:
            return np.array([s0, s1, s1, s1, s_nu, s_nu, s_nu, s2b, s_nu, s_nu]
                            + [s3] * 6 + [s3b] + [s4] * 3 + [s4b] * 3 + [s5] * 3 + [s6],
                            dtype=np.float64)
        return np.array([s0, s1, s1, s1, s_nu, s_nu, s_nu, s2b, s_nu, s_nu]
                        + [s3] * 6 + [s4] * 3, dtype=np.float64)

    # ---- equilibrium moments and forcing moments --------------------------------------
    def meq(self, rho, ux, uy, uz):
        """Equilibrium moments: Eq. (14) for D3Q27, Eq. (C5) for D3Q19. Returns (Q, ...)."""
        c2 = CS2
        u2 = ux * ux + uy * uy + uz * uz
        m27 = [
            rho,
            rho * ux, rho * uy, rho * uz,
            rho * ux * uy, rho * ux * uz, rho * uy * uz,
            rho * (1.0 + u2),
            rho * (ux * ux - uy * uy),
            rho * (ux * ux - uz * uz),
            rho * c2 * ux, rho * c2 * ux, rho * c2 * uy,
            rho * c2 * uz, rho * c2 * uy, rho * c2 * uz,
            0.0 * rho,
            rho * c2 * (c2 + ux * ux + uy * uy),
            rho * c2 * (c2 + ux * ux + uz * uz),
            rho * c2 * (c2 + uy * uy + uz * uz),
            rho * c2 * uy * uz, rho * c2 * ux * uz, rho * c2 * ux * uy,
            rho * c2 * c2 * ux, rho * c2 * c2 * uy, rho * c2 * c2 * uz,
            rho * c2 * c2 * u2 + rho * c2 * c2 * c2,
        ]
        sel = range(27) if self.Q == 27 else _Q19_FROM_Q27
        return np.array([np.broadcast_to(m27[k], np.shape(rho)) for k in sel], dtype=np.float64)

    def forcing_moments(self, Fx, Fy, Fz, ux, uy, uz):
        """Forcing term in moment space F~: Eq. (15) for D3Q27, Eq. (C6) for D3Q19."""
        c2 = CS2
        Fu = Fx * ux + Fy * uy + Fz * uz
        zero = 0.0 * Fx
        F27 = [
            zero,
            Fx, Fy, Fz,
            Fx * uy + Fy * ux, Fx * uz + Fz * ux, Fy * uz + Fz * uy,
            2.0 * Fu,
            2.0 * (Fx * ux - Fy * uy),
            2.0 * (Fx * ux - Fz * uz),
            Fx * c2, Fx * c2, Fy * c2, Fz * c2, Fy * c2, Fz * c2,
            zero,
            2.0 * c2 * (Fx * ux + Fy * uy),
            2.0 * c2 * (Fx * ux + Fz * uz),
            2.0 * c2 * (Fy * uy + Fz * uz),
            c2 * (Fy * uz + Fz * uy), c2 * (Fx * uz + Fz * ux), c2 * (Fx * uy + Fy * ux),
            c2 * c2 * Fx, c2 * c2 * Fy, c2 * c2 * Fz,
            2.0 * c2 * c2 * Fu,
        ]
        sel = range(27) if self.Q == 27 else _Q19_FROM_Q27
        return np.array([np.broadcast_to(F27[k], np.shape(Fx)) for k in sel], dtype=np.float64)

    # ---- velocity-space forms, for cross-checks only -----------------------------------
    def feq_hermite(self, rho, u):
        """Low-Mach equilibrium of Eq. (5), f_i^eq for one node, velocity u (3,)."""
        u = np.asarray(u, dtype=np.float64)
        out = np.empty(self.Q)
        for i in range(self.Q):
            e = self.e[i].astype(np.float64)
            eu = e @ u
            uu_ee = eu * eu - CS2 * (u @ u)  # uu:(e e - c_s^2 I)
            out[i] = rho * self.omega[i] * (1.0 + eu / CS2 + uu_ee / (2.0 * CS2 * CS2))
        return out

    def guo_force(self, u, F):
        """Forcing term of Eq. (6), F_i = omega [ (e - u)/c_s^2 + (u.e) e / c_s^4 ] . F."""
        u = np.asarray(u, dtype=np.float64)
        F = np.asarray(F, dtype=np.float64)
        out = np.empty(self.Q)
        for i in range(self.Q):
            e = self.e[i].astype(np.float64)
            out[i] = self.omega[i] * (((e - u) / CS2 + (u @ e) * e / (CS2 * CS2)) @ F)
        return out


def invert_exact(A):
    """Inverse of a square matrix of Fractions by Gauss-Jordan elimination with pivoting."""
    n = len(A)
    aug = [list(map(Fraction, row)) + [Fraction(int(i == j)) for j in range(n)]
           for i, row in enumerate(A)]
    for col in range(n):
        piv = next((r for r in range(col, n) if aug[r][col] != 0), None)
        if piv is None:
            raise ValueError("matrix is singular")
        aug[col], aug[piv] = aug[piv], aug[col]
        p = aug[col][col]
        aug[col] = [x / p for x in aug[col]]
        for r in range(n):
            if r != col and aug[r][col] != 0:
                fac = aug[r][col]
                aug[r] = [x - fac * y for x, y in zip(aug[r], aug[col])]
    return [row[n:] for row in aug]


_CACHE = {}


def lattice(Q):
    """Cached Lattice(Q)."""
    if Q not in _CACHE:
        _CACHE[Q] = Lattice(Q)
    return _CACHE[Q]
