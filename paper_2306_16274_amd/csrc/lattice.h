// Device-side lattice description and per-node arithmetic of the non-orthogonal MRT-LBM
// with the pseudopotential multiphase model (Fei et al., arXiv 2306.16274).
//
// The transforms are written out from the structure of the moment set rather than as
// dense matrices: populations are grouped into the rest node, the six axis links, the
// twelve edge links (three planes of four) and, for D3Q27, the eight corners. Inside a
// group the moments are sums and differences of the members (a 2x2 or 2x2x2 Hadamard
// pattern), so m = M f costs the 139 (D3Q19) / 339 (D3Q27) signed additions of the
// printed M minus the shared partial sums, and f = M^-1 m follows by undoing the group
// sums (Table I counts 101 / 226 nonzeros in M^-1; denominators 2, 3, 4, 8).
//
// All moments are carried as deviations from the rest state rho_ref * M w, where w are
// the lattice weights: populations are stored as d_i = f_i - w_i rho_ref, and since
// M w = m^eq(rho = 1, u = 0) (1 in m0 and m7, c_s^4 in the k220-type moments, c_s^6 in
// k222, 0 elsewhere) only those entries of the equilibrium change. With rho_ref = 0 this
// is the plain scheme.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbmk {

// Velocities in the order of Eq. (1); D3Q19 uses the first 19 (Eq. (C1)).
__host__ __device__ constexpr int vel_x(int i) {
    constexpr int v[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0,
                           1, -1, 1, -1, 1, -1, 1, -1};
    return v[i];
}
__host__ __device__ constexpr int vel_y(int i) {
    constexpr int v[27] = {0, 0, 0, 1, -1, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 1, -1, 1, -1,
                           1, 1, -1, -1, 1, 1, -1, -1};
    return v[i];
}
__host__ __device__ constexpr int vel_z(int i) {
    constexpr int v[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, 1, -1, -1, 1, 1, -1, -1,
                           1, 1, 1, 1, -1, -1, -1, -1};
    return v[i];
}
__host__ __device__ constexpr int opposite(int i) {
    int j = 0;
    for (int k = 0; k < 27; ++k)
        if (vel_x(k) == -vel_x(i) && vel_y(k) == -vel_y(i) && vel_z(k) == -vel_z(i)) j = k;
    return j;
}
__host__ __device__ constexpr int norm2(int i) {
    return vel_x(i) * vel_x(i) + vel_y(i) * vel_y(i) + vel_z(i) * vel_z(i);
}
// Lattice weights omega: D3Q27 as listed under Eq. (5); D3Q19 1/3, 1/18, 1/36.
template <int Q>
__host__ __device__ constexpr double omega(int i) {
    return Q == 19 ? (norm2(i) == 0 ? 1.0 / 3.0 : norm2(i) == 1 ? 1.0 / 18.0 : 1.0 / 36.0)
                   : (norm2(i) == 0 ? 8.0 / 27.0
                      : norm2(i) == 1 ? 2.0 / 27.0
                      : norm2(i) == 2 ? 1.0 / 54.0
                                      : 1.0 / 216.0);
}
// Normalised weights of the interaction force, w = omega / c_s^2 (Eq. (16)).
template <int Q>
__host__ __device__ constexpr double wforce(int i) { return 3.0 * omega<Q>(i); }

enum { EOS_CS = 0, EOS_PIECEWISE = 1 };
// psi taken at a solid neighbour in F_int and Q_ab (the paper leaves it open): the node's
// own psi, the w-weighted mean over its fluid neighbours, or zero.
// WALL_PSI_MIRROR: psi(x + e') with e' = e_i less every component along which the axis
// neighbour of x is solid (for a flat wall the mirror image of x + e_i across the wall
// plane of halfway bounce-back); psi of the node where e' = 0 or x + e' is solid.
enum { WALL_PSI_NODE = 0, WALL_PSI_FLUID_MEAN = 1, WALL_PSI_ZERO = 2, WALL_PSI_MIRROR = 3 };

// Index of the lattice velocity (ex, ey, ez) in the order of Eq. (1) (-1 if none).
__host__ __device__ constexpr int vel_index(int ex, int ey, int ez) {
    for (int k = 0; k < 27; ++k)
        if (vel_x(k) == ex && vel_y(k) == ey && vel_z(k) == ez) return k;
    return -1;
}

// Reciprocal and square root: in float32 the hardware instructions (v_rcp_f32,
// v_sqrt_f32, about 1 ulp); in float64 the correctly rounded operations.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float sqrt_r(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_r(double x) { return sqrt(x); }

// Physical constants of one lattice, in the arithmetic type R.
template <typename R>
struct Phys {
    R rho_ref;
    R G, two_over_G;          // interaction strength and 2/G for psi
    R sigma, kappa, G_ads;
    int eos;
    R cs_a, cs_b, cs_RT;      // Carnahan-Starling a, b and R*T
    R pw_tv, pw_tm, pw_tl, pw_r1, pw_r2, pw_p1, pw_p2;  // piecewise slopes, knees, p at knees
    R s_nu, s_e, s3, s3b, s4, s4b, s5, s6;
    int var_nu;               // density-dependent viscosity, Eq. (24)
    R nu_v, dnu_drho, rho_v;  // nu = nu_v + dnu_drho (rho - rho_v)
    R bfx, bfy, bfz;          // body force
    int wall_psi;             // WALL_PSI_*
};

// Square-root pseudopotential of Sec. II C, psi = sqrt(2 (p_EOS - rho c_s^2) / G), c = 1,
// clamped at 0 outside the phase diagram.
template <typename R>
__device__ __forceinline__ R pseudopotential(R rho, const Phys<R>& P) {
    R p;
    if (P.eos == EOS_CS) {
        const R eta = P.cs_b * rho * R(0.25);
        const R om = R(1) - eta;
        p = rho * P.cs_RT * (R(1) + eta + eta * eta - eta * eta * eta) * recip(om * om * om) -
            P.cs_a * rho * rho;
    } else {
        p = rho <= P.pw_r1 ? rho * P.pw_tv
            : rho <= P.pw_r2 ? P.pw_p1 + (rho - P.pw_r1) * P.pw_tm
                             : P.pw_p2 + (rho - P.pw_r2) * P.pw_tl;
    }
    const R arg = P.two_over_G * (p - rho * R(1.0 / 3.0));
    return arg > R(0) ? sqrt_r(arg) : R(0);
}

// Force terms at one node from psi at the node and its Q-1 neighbours.
template <typename R>
struct NodeForce {
    R Fx, Fy, Fz;             // total force F_int + F_ads + body force
    R phi;                    // |F_int|^2 / psi^2 = G^2 |sum_i w_i psi(x+e_i) e_i|^2
    R Qxx, Qyy, Qzz, Qxy, Qxz, Qyz;   // Q_ab of Eq. (B2)
};

// psi_nb[i] = psi(x + e_i) for i >= 1, negative where x + e_i is solid. A solid neighbour
// counts in the wetting sum and takes, in F_int and Q_ab, psi of the node itself
// (WALL_PSI_NODE: its terms vanish), the w-weighted mean psi of the fluid neighbours or 0:
// the main loop sums the fluid neighbours only, and for the two other readings a second
// pass adds (psi_wall - psi0) times the solid neighbours' first and second moments of w e.
// SOLIDS = false: the lattice has no solid node (psi_nb is never negative), so the solid
// tests and the wetting sums drop out at compile time; the arithmetic of every remaining
// term is unchanged, so both forms give bitwise equal results on such a lattice.
// WITH_Q = false: kappa = 0, so Q_ab of Eq. (B2) vanishes identically and its sums are
// skipped (Q_ab = +0; the kappa-scaled products would be signed zeros).
template <int Q, typename R, bool SOLIDS, bool WITH_Q>
__device__ __forceinline__ NodeForce<R> node_force_sums(R psi0, const R* psi_nb, const Phys<R>& P) {
    R ax = 0, ay = 0, az = 0;                 // sum w (psi_nb - psi0) e
    R qxx = 0, qyy = 0, qzz = 0, qxy = 0, qxz = 0, qyz = 0;
    R sx = 0, sy = 0, sz = 0;                 // sum w s(x+e) e
#pragma unroll
    for (int i = 1; i < Q; ++i) {
        const R w = R(wforce<Q>(i));
        const bool solid = SOLIDS && psi_nb[i] < R(0);
        const R d = solid ? R(0) : psi_nb[i] - psi0;
        const int ex = vel_x(i), ey = vel_y(i), ez = vel_z(i);
        const R wd = w * d;
        if (ex) ax += ex > 0 ? wd : -wd;
        if (ey) ay += ey > 0 ? wd : -wd;
        if (ez) az += ez > 0 ? wd : -wd;
        if (WITH_Q) {
            if (ex) qxx += wd;
            if (ey) qyy += wd;
            if (ez) qzz += wd;
            if (ex && ey) qxy += ex * ey > 0 ? wd : -wd;
            if (ex && ez) qxz += ex * ez > 0 ? wd : -wd;
            if (ey && ez) qyz += ey * ez > 0 ? wd : -wd;
        }
        const R ws = solid ? w : R(0);
        if (ex) sx += ex > 0 ? ws : -ws;
        if (ey) sy += ey > 0 ? ws : -ws;
        if (ez) sz += ez > 0 ? ws : -ws;
    }
    if (SOLIDS && P.wall_psi == WALL_PSI_MIRROR) {
        // solidity of the six axis neighbours decides which components of a solid link to
        // drop; the image's psi is chosen by selects among the compile-time candidates
        const bool sol[3][2] = {{psi_nb[2] < R(0), psi_nb[1] < R(0)},
                                {psi_nb[4] < R(0), psi_nb[3] < R(0)},
                                {psi_nb[6] < R(0), psi_nb[5] < R(0)}};
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            if (!(psi_nb[i] < R(0))) continue;
            const int e[3] = {vel_x(i), vel_y(i), vel_z(i)};
            bool keep[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) keep[a] = e[a] != 0 && !sol[a][e[a] > 0];
            R pm = psi0;
#pragma unroll
            for (int mask = 1; mask < 8; ++mask) {
                // candidate e' keeps the components in mask (only those e has)
                const int cx = (mask & 1) ? e[0] : 0, cy = (mask & 2) ? e[1] : 0,
                          cz = (mask & 4) ? e[2] : 0;
                if (((mask & 1) && !e[0]) || ((mask & 2) && !e[1]) || ((mask & 4) && !e[2]))
                    continue;
                const int j = vel_index(cx, cy, cz);
                if (j < 1 || j >= Q) continue;
                const bool pick = keep[0] == ((mask & 1) != 0) && keep[1] == ((mask & 2) != 0) &&
                                  keep[2] == ((mask & 4) != 0);
                if (pick && !(psi_nb[j] < R(0))) pm = psi_nb[j];
            }
            const R w = R(wforce<Q>(i));
            const R wd = w * (pm - psi0);
            if (e[0]) ax += e[0] > 0 ? wd : -wd;
            if (e[1]) ay += e[1] > 0 ? wd : -wd;
            if (e[2]) az += e[2] > 0 ? wd : -wd;
            if (WITH_Q) {
                if (e[0]) qxx += wd;
                if (e[1]) qyy += wd;
                if (e[2]) qzz += wd;
                if (e[0] && e[1]) qxy += e[0] * e[1] > 0 ? wd : -wd;
                if (e[0] && e[2]) qxz += e[0] * e[2] > 0 ? wd : -wd;
                if (e[1] && e[2]) qyz += e[1] * e[2] > 0 ? wd : -wd;
            }
        }
    }
    if (SOLIDS && (P.wall_psi == WALL_PSI_FLUID_MEAN || P.wall_psi == WALL_PSI_ZERO)) {
        R wf = 0, pf = 0;                     // sum over fluid neighbours of w, w (psi - psi0)
        R txx = 0, tyy = 0, tzz = 0, txy = 0, txz = 0, tyz = 0;   // solid: sum w e_a e_b
#pragma unroll
        for (int i = 1; i < Q; ++i) {
            const R w = R(wforce<Q>(i));
            const bool solid = psi_nb[i] < R(0);
            const int ex = vel_x(i), ey = vel_y(i), ez = vel_z(i);
            if (!solid) { wf += w; pf += w * (psi_nb[i] - psi0); }
            if (WITH_Q && solid) {
                if (ex) txx += w;
                if (ey) tyy += w;
                if (ez) tzz += w;
                if (ex && ey) txy += ex * ey > 0 ? w : -w;
                if (ex && ez) txz += ex * ez > 0 ? w : -w;
                if (ey && ez) tyz += ey * ez > 0 ? w : -w;
            }
        }
        const R dm = P.wall_psi == WALL_PSI_ZERO ? -psi0 : (wf > R(0) ? pf / wf : R(0));
        ax += dm * sx; ay += dm * sy; az += dm * sz;
        if (WITH_Q) {
            qxx += dm * txx; qyy += dm * tyy; qzz += dm * tzz;
            qxy += dm * txy; qxz += dm * txz; qyz += dm * tyz;
        }
    }
    NodeForce<R> nf;
    // Eq. (16): F_int = -G psi sum w psi(x+e) e; sum w e = 0 lets psi(x+e) become the
    // difference psi(x+e) - psi(x), which is better conditioned.
    const R gp = -P.G * psi0;
    const R ga = -P.G_ads * psi0 * psi0;      // Eq. (22)
    nf.Fx = gp * ax + ga * sx + P.bfx;
    nf.Fy = gp * ay + ga * sy + P.bfy;
    nf.Fz = gp * az + ga * sz + P.bfz;
    nf.phi = P.G * P.G * (ax * ax + ay * ay + az * az);
    if (WITH_Q) {
        const R kq = P.kappa * P.G * R(0.5) * psi0;   // Eq. (B2)
        nf.Qxx = kq * qxx; nf.Qyy = kq * qyy; nf.Qzz = kq * qzz;
        nf.Qxy = kq * qxy; nf.Qxz = kq * qxz; nf.Qyz = kq * qyz;
    } else {
        nf.Qxx = nf.Qyy = nf.Qzz = nf.Qxy = nf.Qxz = nf.Qyz = R(0);
    }
    return nf;
}
// kappa is uniform over the launch, so the branch between the two forms is a scalar one.
// Only lattices without solid nodes take it: with the solid tests in the loop, two copies
// of it cost registers (walled and cylinder lattices ran 7-57 % slower).
template <int Q, typename R, bool SOLIDS = true>
__device__ __forceinline__ NodeForce<R> node_force(R psi0, const R* psi_nb, const Phys<R>& P) {
    if (SOLIDS || P.kappa != R(0)) return node_force_sums<Q, R, SOLIDS, true>(psi0, psi_nb, P);
    return node_force_sums<Q, R, false, false>(psi0, psi_nb, P);
}

// Raw moments k_mnp of the deviations (Eq. (2)); names follow the exponents.
template <typename R>
struct Raw {
    R k000, k100, k010, k001, k110, k101, k011, k200, k020, k002;
    R k120, k102, k210, k201, k012, k021, k220, k202, k022;
    R k111, k211, k121, k112, k122, k212, k221, k222;   // D3Q27 only
};

template <int Q, typename R>
__device__ __forceinline__ Raw<R> forward(const R* d) {
    Raw<R> k;
    const R x1 = d[1] + d[2], x1d = d[1] - d[2];
    const R y1 = d[3] + d[4], y1d = d[3] - d[4];
    const R z1 = d[5] + d[6], z1d = d[5] - d[6];
    // xy links 7(+,+) 8(-,+) 9(+,-) 10(-,-)
    const R xy_p = d[7] + d[9], xy_m = d[8] + d[10];
    const R xy0 = xy_p + xy_m, xy_x = xy_p - xy_m;
    const R xy_y = (d[7] + d[8]) - (d[9] + d[10]);
    const R xy_xy = (d[7] - d[8]) - (d[9] - d[10]);
    // xz links 11(+,+) 12(-,+) 13(+,-) 14(-,-)
    const R xz_p = d[11] + d[13], xz_m = d[12] + d[14];
    const R xz0 = xz_p + xz_m, xz_x = xz_p - xz_m;
    const R xz_z = (d[11] + d[12]) - (d[13] + d[14]);
    const R xz_xz = (d[11] - d[12]) - (d[13] - d[14]);
    // yz links 15(+,+) 16(-,+) 17(+,-) 18(-,-)
    const R yz_p = d[15] + d[17], yz_m = d[16] + d[18];
    const R yz0 = yz_p + yz_m, yz_y = yz_p - yz_m;
    const R yz_z = (d[15] + d[16]) - (d[17] + d[18]);
    const R yz_yz = (d[15] - d[16]) - (d[17] - d[18]);
    k.k000 = d[0] + x1 + y1 + z1 + xy0 + xz0 + yz0;
    k.k100 = x1d + xy_x + xz_x;
    k.k010 = y1d + xy_y + yz_y;
    k.k001 = z1d + xz_z + yz_z;
    k.k110 = xy_xy; k.k101 = xz_xz; k.k011 = yz_yz;
    k.k200 = x1 + xy0 + xz0;
    k.k020 = y1 + xy0 + yz0;
    k.k002 = z1 + xz0 + yz0;
    k.k120 = xy_x; k.k102 = xz_x; k.k210 = xy_y; k.k201 = xz_z; k.k012 = yz_y; k.k021 = yz_z;
    k.k220 = xy0; k.k202 = xz0; k.k022 = yz0;
    if constexpr (Q == 27) {
        // corners 19(+,+,+) 20(-,+,+) 21(+,-,+) 22(-,-,+) 23(+,+,-) 24(-,+,-) 25(+,-,-) 26(-,-,-)
        const R p0 = d[19] + d[20], q0 = d[19] - d[20];
        const R p1 = d[21] + d[22], q1 = d[21] - d[22];
        const R p2 = d[23] + d[24], q2 = d[23] - d[24];
        const R p3 = d[25] + d[26], q3 = d[25] - d[26];
        const R r0 = p0 + p1, r1 = p0 - p1, r2 = p2 + p3, r3 = p2 - p3;
        const R t0 = q0 + q1, t1 = q0 - q1, t2 = q2 + q3, t3 = q2 - q3;
        const R C0 = r0 + r2, Cz = r0 - r2, Cy = r1 + r3, Cyz = r1 - r3;
        const R Cx = t0 + t2, Cxz = t0 - t2, Cxy = t1 + t3, Cxyz = t1 - t3;
        k.k000 += C0; k.k100 += Cx; k.k010 += Cy; k.k001 += Cz;
        k.k110 += Cxy; k.k101 += Cxz; k.k011 += Cyz;
        k.k200 += C0; k.k020 += C0; k.k002 += C0;
        k.k120 += Cx; k.k102 += Cx; k.k210 += Cy; k.k201 += Cz; k.k012 += Cy; k.k021 += Cz;
        k.k220 += C0; k.k202 += C0; k.k022 += C0;
        k.k111 = Cxyz; k.k211 = Cyz; k.k121 = Cxz; k.k112 = Cxy;
        k.k122 = Cx; k.k212 = Cy; k.k221 = Cz; k.k222 = C0;
    }
    return k;
}

// f = M^-1 m, written by undoing the group sums of forward().
template <int Q, typename R>
__device__ __forceinline__ void backward(const Raw<R>& k, R* d) {
    R c220 = k.k220, c202 = k.k202, c022 = k.k022;
    R c120 = k.k120, c102 = k.k102, c210 = k.k210, c201 = k.k201, c012 = k.k012, c021 = k.k021;
    R c110 = k.k110, c101 = k.k101, c011 = k.k011;
    R ax = k.k100 - k.k120 - k.k102, ay = k.k010 - k.k210 - k.k012, az = k.k001 - k.k201 - k.k021;
    R sx = k.k200 - k.k220 - k.k202, sy = k.k020 - k.k220 - k.k022, sz = k.k002 - k.k202 - k.k022;
    R rest = k.k000 - (k.k200 + k.k020 + k.k002) + k.k220 + k.k202 + k.k022;
    if constexpr (Q == 27) {
        // remove the corner share from the edge and axis sums, then the corners themselves
        c220 -= k.k222; c202 -= k.k222; c022 -= k.k222;
        c120 -= k.k122; c102 -= k.k122; c210 -= k.k212; c201 -= k.k221;
        c012 -= k.k212; c021 -= k.k221;
        c110 -= k.k112; c101 -= k.k121; c011 -= k.k211;
        ax += k.k122; ay += k.k212; az += k.k221;
        sx += k.k222; sy += k.k222; sz += k.k222;
        rest -= k.k222;
        const R C0 = k.k222, Cx = k.k122, Cy = k.k212, Cz = k.k221;
        const R Cxy = k.k112, Cxz = k.k121, Cyz = k.k211, Cxyz = k.k111;
        // inverse 2x2x2 Hadamard
        const R r0 = C0 + Cz, r2 = C0 - Cz, r1 = Cy + Cyz, r3 = Cy - Cyz;
        const R t0 = Cx + Cxz, t2 = Cx - Cxz, t1 = Cxy + Cxyz, t3 = Cxy - Cxyz;
        const R p0 = r0 + r1, p1 = r0 - r1, p2 = r2 + r3, p3 = r2 - r3;
        const R q0 = t0 + t1, q1 = t0 - t1, q2 = t2 + t3, q3 = t2 - t3;
        const R e8 = R(0.125);
        d[19] = e8 * (p0 + q0); d[20] = e8 * (p0 - q0);
        d[21] = e8 * (p1 + q1); d[22] = e8 * (p1 - q1);
        d[23] = e8 * (p2 + q2); d[24] = e8 * (p2 - q2);
        d[25] = e8 * (p3 + q3); d[26] = e8 * (p3 - q3);
    }
    const R q = R(0.25), h = R(0.5);
    d[7] = q * ((c220 + c110) + (c120 + c210));
    d[8] = q * ((c220 - c110) - (c120 - c210));
    d[9] = q * ((c220 - c110) + (c120 - c210));
    d[10] = q * ((c220 + c110) - (c120 + c210));
    d[11] = q * ((c202 + c101) + (c102 + c201));
    d[12] = q * ((c202 - c101) - (c102 - c201));
    d[13] = q * ((c202 - c101) + (c102 - c201));
    d[14] = q * ((c202 + c101) - (c102 + c201));
    d[15] = q * ((c022 + c011) + (c012 + c021));
    d[16] = q * ((c022 - c011) - (c012 - c021));
    d[17] = q * ((c022 - c011) + (c012 - c021));
    d[18] = q * ((c022 + c011) - (c012 + c021));
    d[1] = h * (sx + ax); d[2] = h * (sx - ax);
    d[3] = h * (sy + ay); d[4] = h * (sy - ay);
    d[5] = h * (sz + az); d[6] = h * (sz - az);
    d[0] = rest;
}

// Moment-space collision of Eq. (8), m* = m - S (m - m^eq) + (I - S/2) F~', with m^eq of
// Eq. (14)/(C5) and F~' of Eq. (15)/(C6) modified by Eq. (B1). The (I - S/2) factor on the
// sigma and Q terms of Eq. (B1) cancels their 1/(1/s - 1/2) to a plain factor s. Mass and
// momentum rows are written in their exact post-collision form (rho and j + F), which is
// what Eq. (8) gives for any s0, s1. In-place on d (deviations); returns rho.
template <int Q, typename R>
__device__ __forceinline__ R collide(R* d, const NodeForce<R>& nf, const Phys<R>& P) {
    const Raw<R> k = forward<Q, R>(d);
    const R rho = P.rho_ref + k.k000;
    const R inv_rho = recip(rho);
    const R Fx = nf.Fx, Fy = nf.Fy, Fz = nf.Fz;
    const R ux = (k.k100 + R(0.5) * Fx) * inv_rho;
    const R uy = (k.k010 + R(0.5) * Fy) * inv_rho;
    const R uz = (k.k001 + R(0.5) * Fz) * inv_rho;
    const R uxx = ux * ux, uyy = uy * uy, uzz = uz * uz;
    const R c2 = R(1.0 / 3.0), c4 = R(1.0 / 9.0);

    R s_nu = P.s_nu;
    if (P.var_nu) {   // Eq. (24) with nu = (1/s_nu - 1/2)/3
        const R nu = P.nu_v + P.dnu_drho * (rho - P.rho_v);
        s_nu = recip(R(3) * nu + R(0.5));
    }
    const R sn = s_nu, hn = R(1) - R(0.5) * sn;
    const R se = P.s_e, he = R(1) - R(0.5) * se;
    const R s3 = P.s3, h3 = R(1) - R(0.5) * s3;
    const R s4 = P.s4, h4 = R(1) - R(0.5) * s4;

    Raw<R> o;
    o.k000 = k.k000;
    o.k100 = k.k100 + Fx;
    o.k010 = k.k010 + Fy;
    o.k001 = k.k001 + Fz;
    // viscous stress: m4..m6, m8, m9 (rate s_nu); m7 (rate s_e = s_2b)
    o.k110 = k.k110 - sn * (k.k110 - rho * ux * uy) + hn * (Fx * uy + Fy * ux) - sn * nf.Qxy;
    o.k101 = k.k101 - sn * (k.k101 - rho * ux * uz) + hn * (Fx * uz + Fz * ux) - sn * nf.Qxz;
    o.k011 = k.k011 - sn * (k.k011 - rho * uy * uz) + hn * (Fy * uz + Fz * uy) - sn * nf.Qyz;
    const R m7 = k.k200 + k.k020 + k.k002;
    const R m8 = k.k200 - k.k020;
    const R m9 = k.k200 - k.k002;
    const R Fu = Fx * ux + Fy * uy + Fz * uz;
    const R m7s = m7 - se * (m7 - (k.k000 + rho * (uxx + uyy + uzz))) + he * (R(2) * Fu) +
                  se * (R(6) * P.sigma * nf.phi + R(0.8) * (nf.Qxx + nf.Qyy + nf.Qzz));
    const R m8s = m8 - sn * (m8 - rho * (uxx - uyy)) + hn * (R(2) * (Fx * ux - Fy * uy)) -
                  sn * (nf.Qxx - nf.Qyy);
    const R m9s = m9 - sn * (m9 - rho * (uxx - uzz)) + hn * (R(2) * (Fx * ux - Fz * uz)) -
                  sn * (nf.Qxx - nf.Qzz);
    const R third = R(1.0 / 3.0);
    o.k200 = third * (m7s + m8s + m9s);
    o.k020 = third * (m7s - R(2) * m8s + m9s);
    o.k002 = third * (m7s + m8s - R(2) * m9s);
    // third order (rate s3): m^eq = rho c_s^2 u_a, F~ = c_s^2 F_a
    const R rc2 = rho * c2;
    o.k120 = k.k120 - s3 * (k.k120 - rc2 * ux) + h3 * c2 * Fx;
    o.k102 = k.k102 - s3 * (k.k102 - rc2 * ux) + h3 * c2 * Fx;
    o.k210 = k.k210 - s3 * (k.k210 - rc2 * uy) + h3 * c2 * Fy;
    o.k201 = k.k201 - s3 * (k.k201 - rc2 * uz) + h3 * c2 * Fz;
    o.k012 = k.k012 - s3 * (k.k012 - rc2 * uy) + h3 * c2 * Fy;
    o.k021 = k.k021 - s3 * (k.k021 - rc2 * uz) + h3 * c2 * Fz;
    // fourth order k220-type (rate s4): deviation m^eq = c_s^4 drho + rho c_s^2 (u_a^2+u_b^2)
    const R c4d = c4 * k.k000;
    const R tc2 = R(2) * c2;
    o.k220 = k.k220 - s4 * (k.k220 - (c4d + rc2 * (uxx + uyy))) + h4 * tc2 * (Fx * ux + Fy * uy);
    o.k202 = k.k202 - s4 * (k.k202 - (c4d + rc2 * (uxx + uzz))) + h4 * tc2 * (Fx * ux + Fz * uz);
    o.k022 = k.k022 - s4 * (k.k022 - (c4d + rc2 * (uyy + uzz))) + h4 * tc2 * (Fy * uy + Fz * uz);
    if constexpr (Q == 27) {
        const R s3b = P.s3b, s4b = P.s4b, h4b = R(1) - R(0.5) * s4b;
        const R s5 = P.s5, h5 = R(1) - R(0.5) * s5;
        const R s6 = P.s6, h6 = R(1) - R(0.5) * s6;
        o.k111 = k.k111 - s3b * k.k111;
        o.k211 = k.k211 - s4b * (k.k211 - rc2 * uy * uz) + h4b * c2 * (Fy * uz + Fz * uy);
        o.k121 = k.k121 - s4b * (k.k121 - rc2 * ux * uz) + h4b * c2 * (Fx * uz + Fz * ux);
        o.k112 = k.k112 - s4b * (k.k112 - rc2 * ux * uy) + h4b * c2 * (Fx * uy + Fy * ux);
        const R rc4 = rho * c4;
        o.k122 = k.k122 - s5 * (k.k122 - rc4 * ux) + h5 * c4 * Fx;
        o.k212 = k.k212 - s5 * (k.k212 - rc4 * uy) + h5 * c4 * Fy;
        o.k221 = k.k221 - s5 * (k.k221 - rc4 * uz) + h5 * c4 * Fz;
        const R c6 = R(1.0 / 27.0);
        o.k222 = k.k222 - s6 * (k.k222 - (c6 * k.k000 + rc4 * (uxx + uyy + uzz))) +
                 h6 * (R(2) * c4 * Fu);
    }
    backward<Q, R>(o, d);
    return rho;
}

// Equilibrium deviations d_i = (M^-1 m^eq(rho, u))_i - w_i rho_ref (initial state).
template <int Q, typename R>
__device__ __forceinline__ void equilibrium(R rho, R ux, R uy, R uz, R rho_ref, R* d) {
    const R c2 = R(1.0 / 3.0), c4 = R(1.0 / 9.0);
    const R drho = rho - rho_ref;
    const R uxx = ux * ux, uyy = uy * uy, uzz = uz * uz;
    const R rc2 = rho * c2;
    Raw<R> o;
    o.k000 = drho;
    o.k100 = rho * ux; o.k010 = rho * uy; o.k001 = rho * uz;
    o.k110 = rho * ux * uy; o.k101 = rho * ux * uz; o.k011 = rho * uy * uz;
    // m7 = drho + rho u^2, m8 = rho (ux^2 - uy^2), m9 = rho (ux^2 - uz^2)
    const R m7 = drho + rho * (uxx + uyy + uzz);
    const R m8 = rho * (uxx - uyy), m9 = rho * (uxx - uzz);
    const R third = R(1.0 / 3.0);
    o.k200 = third * (m7 + m8 + m9);
    o.k020 = third * (m7 - R(2) * m8 + m9);
    o.k002 = third * (m7 + m8 - R(2) * m9);
    o.k120 = rc2 * ux; o.k102 = rc2 * ux; o.k210 = rc2 * uy;
    o.k201 = rc2 * uz; o.k012 = rc2 * uy; o.k021 = rc2 * uz;
    o.k220 = c4 * drho + rc2 * (uxx + uyy);
    o.k202 = c4 * drho + rc2 * (uxx + uzz);
    o.k022 = c4 * drho + rc2 * (uyy + uzz);
    if constexpr (Q == 27) {
        const R rc4 = rho * c4;
        o.k111 = 0;
        o.k211 = rc2 * uy * uz; o.k121 = rc2 * ux * uz; o.k112 = rc2 * ux * uy;
        o.k122 = rc4 * ux; o.k212 = rc4 * uy; o.k221 = rc4 * uz;
        o.k222 = R(1.0 / 27.0) * drho + rc4 * (uxx + uyy + uzz);
    }
    backward<Q, R>(o, d);
}

}  // namespace lbmk
