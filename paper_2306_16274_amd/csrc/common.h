// Device helpers shared by every kernel: storage/arithmetic types, the domain grid, the
// periodic neighbour indices and the pull of a node's populations (gfx950).
//
// Population storage is SoA: plane i of the buffer holds population i of every node
// (index n = x + nx (y + ny z)), planes `stride` elements apart. The stored state is the
// post-collision f_bar* of the previous step; a step pulls f_bar_i(x) = f_bar*_i(x - e_i)
// (Eq. (9) read backwards), or, when x - e_i is solid, the halfway bounce-back value
// f_bar*_opp(i)(x).
#pragma once

#include "lattice.h"

namespace lbmk {

template <typename T> struct Arith { using type = float; };
template <> struct Arith<double> { using type = double; };

template <typename T, typename R>
__device__ __forceinline__ R load_as(const T* p) { return static_cast<R>(*p); }
template <typename T, typename R>
__device__ __forceinline__ void store_as(T* p, R v) { *p = static_cast<T>(v); }

struct Grid {
    int nx, ny, nz;
    int walls;                // solid layers: bit 2a = axis a low face, bit 2a+1 = high face
    long long stride;         // elements between population planes
    int sf0, sf1;             // fused step: planes [sf0, sf1) may run the solid-free form
};

// Indices of x + e_j for all j (periodic wrap on every axis).
template <int Q>
__device__ __forceinline__ void neighbour_index(const Grid& g, int x, int y, int z, int* nb) {
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? g.ny - 1 : y - 1, yp = y == g.ny - 1 ? 0 : y + 1;
    const int zm = z == 0 ? g.nz - 1 : z - 1, zp = z == g.nz - 1 ? 0 : z + 1;
    const int nxy = g.nx * g.ny;
    const int ox[3] = {xm, x, xp};
    const int oy[3] = {ym * g.nx, y * g.nx, yp * g.nx};
    const int oz[3] = {zm * nxy, z * nxy, zp * nxy};
#pragma unroll
    for (int j = 0; j < Q; ++j)
        nb[j] = ox[vel_x(j) + 1] + oy[vel_y(j) + 1] + oz[vel_z(j) + 1];
}

// Pull the Q populations of node n, with bounce-back where the source is solid.
template <int Q, typename T, typename R>
__device__ __forceinline__ void gather(const T* __restrict__ f, long long stride, int n,
                                       const int* nb, const bool* solid_nb, R* d) {
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        const int o = opposite(i);
        // source x - e_i = x + e_o
        const long long idx = solid_nb[o] ? (long long)o * stride + n
                                          : (long long)i * stride + nb[o];
        d[i] = load_as<T, R>(f + idx);
    }
}

}  // namespace lbmk
