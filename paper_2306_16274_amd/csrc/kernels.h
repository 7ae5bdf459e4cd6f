// HIP kernels of the two-pass time step, the diagnostics and the initialisation (gfx950).
// Storage layout and the pull convention: common.h.
//
// Two-pass step:
//   k_density_psi  gather -> rho -> psi(rho); psi < 0 marks solid nodes
//   k_collide      gather + psi of the 26-neighbourhood -> forces -> collision -> store
#pragma once

#include "common.h"

namespace lbmk {

template <int Q, typename T, bool SOLID>
__global__ __launch_bounds__(256) void k_density_psi(const T* __restrict__ f,
                                                     const uint8_t* __restrict__ solid,
                                                     typename Arith<T>::type* __restrict__ psi,
                                                     Grid g, Phys<typename Arith<T>::type> P) {
    using R = typename Arith<T>::type;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const int n = x + g.nx * (y + g.ny * z);
    if (SOLID && solid[n]) { psi[n] = R(-1); return; }
    int nb[Q];
    neighbour_index<Q>(g, x, y, z, nb);
    bool snb[Q];
#pragma unroll
    for (int j = 0; j < Q; ++j) snb[j] = SOLID ? solid[nb[j]] != 0 : false;
    R d[Q];
    gather<Q, T, R>(f, g.stride, n, nb, snb, d);
    R s = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) s += d[i];
    psi[n] = pseudopotential<R>(P.rho_ref + s, P);
}

template <int Q, typename T>
__global__ __launch_bounds__(256) void k_collide(const T* __restrict__ fin, T* __restrict__ fout,
                                                 const typename Arith<T>::type* __restrict__ psi,
                                                 Grid g, Phys<typename Arith<T>::type> P) {
    using R = typename Arith<T>::type;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const int n = x + g.nx * (y + g.ny * z);
    const R psi0 = psi[n];
    if (psi0 < R(0)) return;                       // solid node: nothing stored
    int nb[Q];
    neighbour_index<Q>(g, x, y, z, nb);
    R pn[Q];
    bool snb[Q];
#pragma unroll
    for (int j = 1; j < Q; ++j) { pn[j] = psi[nb[j]]; snb[j] = pn[j] < R(0); }
    pn[0] = psi0; snb[0] = false;
    R d[Q];
    gather<Q, T, R>(fin, g.stride, n, nb, snb, d);
    const NodeForce<R> nf = node_force<Q, R>(psi0, pn, P);
    collide<Q, R>(d, nf, P);
#pragma unroll
    for (int i = 0; i < Q; ++i) store_as<T, R>(fout + (long long)i * g.stride + n, d[i]);
}

// Macroscopic quantities of one fluid node (x, y, z) at the current time, in float64:
// rho, j = sum f e + F/2 (Eq. (10)) and u = j / rho; needs psi of the node's neighbourhood.
struct NodeMoments { double rho, jx, jy, jz, ux, uy, uz; };
template <int Q, typename T>
__device__ __forceinline__ NodeMoments node_moments(const T* __restrict__ fin,
                                                    const typename Arith<T>::type* __restrict__ psi,
                                                    const Grid& g, const Phys<typename Arith<T>::type>& P,
                                                    int x, int y, int z, int n) {
    using R = typename Arith<T>::type;
    int nb[Q];
    neighbour_index<Q>(g, x, y, z, nb);
    R pn[Q];
    bool snb[Q];
#pragma unroll
    for (int j = 1; j < Q; ++j) { pn[j] = psi[nb[j]]; snb[j] = pn[j] < R(0); }
    pn[0] = psi[n]; snb[0] = false;
    R d[Q];
    gather<Q, T, R>(fin, g.stride, n, nb, snb, d);
    const NodeForce<R> nf = node_force<Q, R>(pn[0], pn, P);
    const Raw<R> k = forward<Q, R>(d);
    NodeMoments m;
    m.rho = (double)P.rho_ref + (double)k.k000;
    m.jx = (double)k.k100 + 0.5 * (double)nf.Fx;
    m.jy = (double)k.k010 + 0.5 * (double)nf.Fy;
    m.jz = (double)k.k001 + 0.5 * (double)nf.Fz;
    m.ux = m.jx / m.rho; m.uy = m.jy / m.rho; m.uz = m.jz / m.rho;
    return m;
}

// Sum of acc[0..C-1] over a 256-thread block (wavefront shuffles, then one value per
// wavefront through LDS, in a fixed order); thread 0..C-1 writes out[c].
template <int C>
__device__ __forceinline__ void block_sums_to(double* acc, double* __restrict__ out) {
    __shared__ double red[C][8];
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int c = 0; c < C; ++c) {
        double v = acc[c];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[c][wave] = v;
    }
    __syncthreads();
    if (tid < C) {
        const int nw = (blockDim.x * blockDim.y + 63) / 64;
        double s = 0;
        for (int w = 0; w < nw; ++w) s += red[tid][w];
        out[tid] = s;
    }
}

// Macroscopic fields at the current time: rho, u (with F/2), p = rho/3 + G psi^2/2, and
// per-block partial sums of rho, rho u, rho |u|^2 / 2 for the totals.
template <int Q, typename T>
__global__ __launch_bounds__(256) void k_moments(const T* __restrict__ fin,
                                                 const typename Arith<T>::type* __restrict__ psi,
                                                 double* __restrict__ rho_out,
                                                 double* __restrict__ u_out,
                                                 double* __restrict__ p_out,
                                                 double* __restrict__ partial,
                                                 Grid g, Phys<typename Arith<T>::type> P) {
    using R = typename Arith<T>::type;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    const long long N = (long long)g.nx * g.ny * g.nz;
    double acc[5] = {0, 0, 0, 0, 0};
    if (x < g.nx && y < g.ny) {
        const int n = x + g.nx * (y + g.ny * z);
        const R psi0 = psi[n];
        if (psi0 < R(0)) {
            rho_out[n] = 0; p_out[n] = 0;
            u_out[n] = 0; u_out[N + n] = 0; u_out[2 * N + n] = 0;
        } else {
            const NodeMoments m = node_moments<Q, T>(fin, psi, g, P, x, y, z, n);
            rho_out[n] = m.rho;
            u_out[n] = m.ux; u_out[N + n] = m.uy; u_out[2 * N + n] = m.uz;
            const double ps = (double)psi0;
            p_out[n] = m.rho / 3.0 + 0.5 * (double)P.G * ps * ps;
            acc[0] = m.rho; acc[1] = m.jx; acc[2] = m.jy; acc[3] = m.jz;
            acc[4] = 0.5 * (m.jx * m.ux + m.jy * m.uy + m.jz * m.uz);
        }
    }
    const long long b = blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z);
    block_sums_to<5>(acc, partial + b * 5);
}

// Per-block partial sums of the five totals of k_moments (rho, rho u, rho |u|^2 / 2 over
// fluid nodes) with no field output: a 1-D grid of gridDim.x blocks of 256 threads that
// strides over the nodes in index order, so any lattice fits a fixed number of partials
// (partial[5 b .. 5 b + 4] for block b).
template <int Q, typename T>
__global__ __launch_bounds__(256) void k_totals(const T* __restrict__ fin,
                                                const typename Arith<T>::type* __restrict__ psi,
                                                double* __restrict__ partial, Grid g,
                                                Phys<typename Arith<T>::type> P) {
    using R = typename Arith<T>::type;
    const long long N = (long long)g.nx * g.ny * g.nz;
    const long long nxy = (long long)g.nx * g.ny;
    double acc[5] = {0, 0, 0, 0, 0};
    for (long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x; n < N;
         n += (long long)gridDim.x * blockDim.x) {
        if (psi[n] < R(0)) continue;
        const int z = (int)(n / nxy), r = (int)(n - (long long)z * nxy);
        const int y = r / g.nx, x = r - y * g.nx;
        const NodeMoments m = node_moments<Q, T>(fin, psi, g, P, x, y, z, (int)n);
        acc[0] += m.rho; acc[1] += m.jx; acc[2] += m.jy; acc[3] += m.jz;
        acc[4] += 0.5 * (m.jx * m.ux + m.jy * m.uy + m.jz * m.uz);
    }
    block_sums_to<5>(acc, partial + (long long)blockIdx.x * 5);
}

// Store f_bar(x) (float64, Q planes of N) into the pull layout: population i of node x
// goes to the slot it will be pulled from, (x - e_i, i), or to (x, opp(i)) when x - e_i is
// solid. Values are stored as deviations from w_i rho_ref.
template <int Q, typename T>
__global__ __launch_bounds__(256) void k_scatter(const double* __restrict__ fsrc, T* __restrict__ f,
                                                 const uint8_t* __restrict__ solid, Grid g,
                                                 double rho_ref) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const long long N = (long long)g.nx * g.ny * g.nz;
    const int n = x + g.nx * (y + g.ny * z);
    if (solid[n]) return;
    int nb[Q];
    neighbour_index<Q>(g, x, y, z, nb);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int o = opposite(i);
        const double v = fsrc[(long long)i * N + n] - omega<Q>(i) * rho_ref;
        const long long idx = solid[nb[o]] ? (long long)o * g.stride + n
                                           : (long long)i * g.stride + nb[o];
        f[idx] = static_cast<T>(v);
    }
}

// Read f_bar(x) back (float64, Q planes of N), 0 at solid nodes.
template <int Q, typename T>
__global__ __launch_bounds__(256) void k_gather_out(const T* __restrict__ f, double* __restrict__ fdst,
                                                    const uint8_t* __restrict__ solid, Grid g,
                                                    double rho_ref) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const long long N = (long long)g.nx * g.ny * g.nz;
    const int n = x + g.nx * (y + g.ny * z);
    if (solid[n]) {
        for (int i = 0; i < Q; ++i) fdst[(long long)i * N + n] = 0.0;
        return;
    }
    int nb[Q];
    neighbour_index<Q>(g, x, y, z, nb);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int o = opposite(i);
        const long long idx = solid[nb[o]] ? (long long)o * g.stride + n
                                           : (long long)i * g.stride + nb[o];
        fdst[(long long)i * N + n] = static_cast<double>(f[idx]) + omega<Q>(i) * rho_ref;
    }
}

// f_bar = M^-1 m^eq(rho, u) from float64 fields (u may be null), written in the pull
// layout like k_scatter.
template <int Q, typename T>
__global__ __launch_bounds__(256) void k_init_fields(const double* __restrict__ rho0,
                                                     const double* __restrict__ u0,
                                                     T* __restrict__ f,
                                                     const uint8_t* __restrict__ solid, Grid g,
                                                     Phys<typename Arith<T>::type> P) {
    using R = typename Arith<T>::type;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    const long long N = (long long)g.nx * g.ny * g.nz;
    const int n = x + g.nx * (y + g.ny * z);
    if (solid[n]) return;
    R d[Q];
    const R ux = u0 ? (R)u0[n] : R(0), uy = u0 ? (R)u0[N + n] : R(0), uz = u0 ? (R)u0[2 * N + n] : R(0);
    equilibrium<Q, R>((R)rho0[n], ux, uy, uz, P.rho_ref, d);
    int nb[Q];
    neighbour_index<Q>(g, x, y, z, nb);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int o = opposite(i);
        const long long idx = solid[nb[o]] ? (long long)o * g.stride + n
                                           : (long long)i * g.stride + nb[o];
        f[idx] = static_cast<T>(d[i]);
    }
}

// Liquid diagnostics of the current state (Sec. IV A spreading diameter, Sec. IV B
// contact time and liquid volume). Per block: the number of liquid fluid nodes
// (rho > threshold), of those the ones with a solid node at x + k e_i for some lattice
// velocity e_i and 1 <= k <= reach (in contact with a wall or the cylinder), and the liquid
// volume fraction sum clamp((rho - rho_v)/(rho_l - rho_v), 0, 1).
// rho is formed exactly as k_moments forms it (float64 sum of rho_ref and the zeroth
// moment), so a threshold applied to the density field lbm_moments returns makes the same
// decisions. Needs psi of the current state (solid marker) from k_density_psi.
template <int Q, typename T>
__global__ __launch_bounds__(256) void k_liquid_stats(const T* __restrict__ fin,
                                                      const typename Arith<T>::type* __restrict__ psi,
                                                      double* __restrict__ partial, Grid g,
                                                      typename Arith<T>::type rho_ref,
                                                      double threshold, double rho_v, double rho_l,
                                                      int reach) {
    using R = typename Arith<T>::type;
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    double acc[3] = {0, 0, 0};
    if (x < g.nx && y < g.ny) {
        const int n = x + g.nx * (y + g.ny * z);
        if (psi[n] >= R(0)) {
            int nb[Q];
            neighbour_index<Q>(g, x, y, z, nb);
            bool snb[Q];
            bool touches = false;
#pragma unroll
            for (int j = 1; j < Q; ++j) { snb[j] = psi[nb[j]] < R(0); touches |= snb[j]; }
            snb[0] = false;
            R d[Q];
            gather<Q, T, R>(fin, g.stride, n, nb, snb, d);
            const double rho = (double)rho_ref + (double)forward<Q, R>(d).k000;
            if (rho > threshold) {
                for (int k = 2; k <= reach && !touches; ++k)
#pragma unroll
                    for (int j = 1; j < Q; ++j) {
                        int c[3] = {x + k * vel_x(j), y + k * vel_y(j), z + k * vel_z(j)};
                        const int n3[3] = {g.nx, g.ny, g.nz};
#pragma unroll
                        for (int a = 0; a < 3; ++a) c[a] = ((c[a] % n3[a]) + n3[a]) % n3[a];
                        touches |= psi[c[0] + g.nx * (c[1] + g.ny * c[2])] < R(0);
                    }
                acc[0] = 1.0;
                acc[1] = touches ? 1.0 : 0.0;
            }
            acc[2] = fmin(fmax((rho - rho_v) / (rho_l - rho_v), 0.0), 1.0);
        }
    }
    __shared__ double red[3][8];
    const int tid = threadIdx.x + blockDim.x * threadIdx.y;
    const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double v = acc[c];
        for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
        if (lane == 0) red[c][wave] = v;
    }
    __syncthreads();
    if (tid < 3) {
        const int nw = (blockDim.x * blockDim.y + 63) / 64;
        double s = 0;
        for (int w = 0; w < nw; ++w) s += red[tid][w];
        const long long b = blockIdx.x + (long long)gridDim.x * (blockIdx.y + (long long)gridDim.y * blockIdx.z);
        partial[b * 3 + tid] = s;
    }
}

// Fixed-order sums of rows of C values: block k adds rows [k rows_per_group, (k+1)
// rows_per_group) of `in` into out[k C .. k C + C - 1] (one block of 256 threads per group).
template <int C>
__global__ __launch_bounds__(256) void k_sum_rows(const double* __restrict__ in,
                                                  long long rows_per_group, double* __restrict__ out) {
    __shared__ double red[C][256];
    const double* base = in + (long long)blockIdx.x * rows_per_group * C;
    double acc[C];
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = 0.0;
    for (long long r = threadIdx.x; r < rows_per_group; r += blockDim.x)
#pragma unroll
        for (int c = 0; c < C; ++c) acc[c] += base[r * C + c];
#pragma unroll
    for (int c = 0; c < C; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int c = 0; c < C; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < C) out[(long long)blockIdx.x * C + threadIdx.x] = red[threadIdx.x][0];
}

// Link words of the fused step on the solid mask: bit 0 = node n is solid, bit i (1..Q-1)
// = its neighbour x - e_i (periodically wrapped, as the fused kernels wrap) is solid.
template <int Q>
__global__ __launch_bounds__(256) void k_build_links(uint32_t* __restrict__ links,
                                                     const uint8_t* __restrict__ solid, Grid g) {
    const int x = blockIdx.x * blockDim.x + threadIdx.x;
    const int y = blockIdx.y * blockDim.y + threadIdx.y;
    const int z = blockIdx.z;
    if (x >= g.nx || y >= g.ny) return;
    auto wrap = [](int c, int n) { return c < 0 ? c + n : (c >= n ? c - n : c); };
    const long long n = x + (long long)g.nx * (y + (long long)g.ny * z);
    uint32_t w = solid[n] ? 1u : 0u;
    for (int i = 1; i < Q; ++i) {
        const int xs = wrap(x - vel_x(i), g.nx), ys = wrap(y - vel_y(i), g.ny), zs = wrap(z - vel_z(i), g.nz);
        if (solid[xs + (long long)g.nx * (ys + (long long)g.ny * zs)]) w |= 1u << i;
    }
    links[n] = w;
}

}  // namespace lbmk
