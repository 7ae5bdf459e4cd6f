// Fused single-pass time step (gfx950).
//
// The step has a global dependency: the force at x needs psi at the neighbours of x, and
// psi(y) needs the populations pulled into y. Instead of a separate density pass (which
// re-reads every population), each workgroup recomputes rho and psi for its tile plus a
// one-node halo and keeps them in LDS:
//
//   * a workgroup owns a TX x TY tile of (x, y) columns and marches along z over a chunk
//     of planes [z0, z1); thread (lx, ly) owns column (x0+lx, y0+ly);
//   * for the plane ahead (z+1) every thread pulls the Q populations of its own node
//     into registers (they are collided one iteration later) and writes psi(rho) to an
//     LDS ring of 4 planes; the first H threads also pull the populations of the
//     2(TX+TY)+4 halo nodes of that plane, only to form their psi;
//   * after one barrier the plane z is collided from registers with psi(z-1..z+1) read
//     from LDS, and the post-collision populations are stored (SoA, coalesced);
//   * halo pulls touch rows that the neighbouring tiles pull at about the same time:
//     tiles are mapped to XCDs in contiguous ranges (workgroup b runs on XCD b mod 8),
//     so neighbouring tiles share an L2 and the halo re-reads stay on chip.
//
// Every LDS cell stands for a node with periodically wrapped coordinates, so tiles that
// cross the domain edge (or are wider than the domain) need no special case: threads
// outside the domain compute psi of the wrapped node but never store.
#pragma once

#include "kernels.h"

namespace lbmk {

// Workgroup b -> tile index such that each XCD (b mod 8) gets a contiguous tile range.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb / 8, r = nb % 8;
    const int xcd = b % 8, k = b / 8;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

// Pull the Q populations of node (x, y, z) (coordinates already wrapped) and return their
// sum (the density deviation). SOLID: bounce back where the source is solid.
template <int Q, typename T, typename R, bool SOLID, bool KEEP>
__device__ __forceinline__ R pull_node(const T* __restrict__ f, const uint8_t* __restrict__ solid,
                                       const Grid& g, int x, int y, int z, R* keep) {
    int nb[Q];
    neighbour_index<Q>(g, x, y, z, nb);
    const int n = nb[0];
    R s = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int o = opposite(i);
        long long idx = (long long)i * g.stride + nb[o];
        if (SOLID && i != 0 && solid[nb[o]]) idx = (long long)o * g.stride + n;
        const R v = load_as<T, R>(f + idx);
        if (KEEP) keep[i] = v;
        s += v;
    }
    return s;
}

template <int Q, typename T, bool SOLID, int TX, int TY>
__global__ __launch_bounds__(TX * TY) void k_step_fused(const T* __restrict__ fin,
                                                       T* __restrict__ fout,
                                                       const uint8_t* __restrict__ solid,
                                                       Grid g, Phys<typename Arith<T>::type> P,
                                                       int ntx, int nty, int zc) {
    using R = typename Arith<T>::type;
    constexpr int LX = TX + 2, LY = TY + 2;
    constexpr int H = 2 * (TX + TY) + 4;
    static_assert(H <= TX * TY, "halo larger than the workgroup");
    __shared__ R ring[4][LY][LX];

    int t = xcd_tile(blockIdx.x, gridDim.x);
    const int ix = t % ntx; t /= ntx;
    const int iy = t % nty;
    const int iz = t / nty;
    const int x0 = ix * TX, y0 = iy * TY, z0 = iz * zc;
    const int z1 = min(z0 + zc, g.nz);
    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int x = x0 + lx, y = y0 + ly;
    const bool active = x < g.nx && y < g.ny;
    auto wrapc = [](int c, int n) { c %= n; return c < 0 ? c + n : c; };
    const int xw = wrapc(x, g.nx), yw = wrapc(y, g.ny);

    // halo cell of this thread (if any), as LDS coordinates (hx, hy) in [-1, T]
    int hx = 0, hy = 0;
    const bool has_halo = tid < H;
    if (has_halo) {
        if (tid < LX) { hx = tid - 1; hy = -1; }
        else if (tid < 2 * LX) { hx = tid - LX - 1; hy = TY; }
        else if (tid < 2 * LX + TY) { hx = -1; hy = tid - 2 * LX; }
        else { hx = TX; hy = tid - 2 * LX - TY; }
    }
    const int hxw = wrapc(x0 + hx, g.nx), hyw = wrapc(y0 + hy, g.ny);

    auto psi_of = [&](R drho) { return pseudopotential<R>(P.rho_ref + drho, P); };
    auto plane_psi = [&](int zp, int slot, R* keep) {
        // own node (populations kept when keep != nullptr)
        const int zw = wrapc(zp, g.nz);
        R v;
        if (SOLID && solid[xw + g.nx * (yw + g.ny * zw)]) v = R(-1);
        else if (keep) v = psi_of(pull_node<Q, T, R, SOLID, true>(fin, solid, g, xw, yw, zw, keep));
        else v = psi_of(pull_node<Q, T, R, SOLID, false>(fin, solid, g, xw, yw, zw, nullptr));
        ring[slot][ly + 1][lx + 1] = v;
        if (has_halo) {
            R hv;
            if (SOLID && solid[hxw + g.nx * (hyw + g.ny * zw)]) hv = R(-1);
            else hv = psi_of(pull_node<Q, T, R, SOLID, false>(fin, solid, g, hxw, hyw, zw, nullptr));
            ring[slot][hy + 1][hx + 1] = hv;
        }
    };

    R cur[Q], nxt[Q];
    plane_psi(z0 - 1, 0, nullptr);
    plane_psi(z0, 1, cur);

    for (int z = z0; z < z1; ++z) {
        const int k = z - z0;
        plane_psi(z + 1, (k + 2) & 3, nxt);
        __syncthreads();
        const int s0 = k & 3, s1 = (k + 1) & 3, s2 = (k + 2) & 3;
        const R psi0 = ring[s1][ly + 1][lx + 1];
        if (active && !(psi0 < R(0))) {
            R pn[Q];
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                const int ez = vel_z(j);
                const int sl = ez < 0 ? s0 : (ez > 0 ? s2 : s1);
                pn[j] = ring[sl][ly + 1 + vel_y(j)][lx + 1 + vel_x(j)];
            }
            const NodeForce<R> nf = node_force<Q, R>(psi0, pn, P);
            collide<Q, R>(cur, nf, P);
            const long long n = x + (long long)g.nx * (y + (long long)g.ny * z);
#pragma unroll
            for (int i = 0; i < Q; ++i) store_as<T, R>(fout + (long long)i * g.stride + n, cur[i]);
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) cur[i] = nxt[i];
    }
}

}  // namespace lbmk
