// Fused single-pass time step (gfx950).
//
// The step has a global dependency: the force at x needs psi at the neighbours of x, and
// psi(y) needs the populations pulled into y. Instead of a separate density pass (which
// re-reads every population), each workgroup recomputes rho and psi for its tile plus a
// one-node halo and keeps them in LDS:
//
//   * a workgroup owns a TX x TY tile of (x, y) columns and marches along z over a chunk
//     of planes [z0, z1); thread (lx, ly) owns column (x0+lx, y0+ly);
//   * psi of the planes around z lives in an LDS ring of four planes (tile plus halo);
//     one barrier per plane. At plane z a thread pulls the populations of its own node
//     of plane z+1 into registers and writes its psi, then (after the barrier) collides
//     plane z from the registers filled one iteration earlier, with psi(z-1..z+1) from
//     LDS, and stores it;
//   * the first H threads also pull the populations of the halo nodes of plane z+1,
//     only to form their psi (H = 2(TX+TY)+4 for a tile, 2 TX for full rows). Those rows
//     are pulled by the neighbouring tiles at about the same time: tiles are mapped to
//     XCDs in contiguous ranges (workgroup b runs on XCD b mod 8), so neighbouring tiles
//     share an L2 and the halo re-reads stay on chip;
//   * with a cylinder, solidity comes from one 32-bit link word per node (bit 0: the node,
//     bit i: its neighbour x - e_i), not from a byte load per population; on a lattice
//     without solid nodes the force sums drop their solid tests and wetting sums at compile
//     time, and at kappa = 0 also the Q_ab sums (a scalar branch per launch);
//   * addresses are 32-bit byte offsets from the buffer base below 4 GiB of populations,
//     64-bit offsets (plain 64x4 / 64x8 tiles only) from there on, with the in-plane
//     offsets of the 3x3 column neighbourhood computed once per thread.
//
// Every LDS cell stands for a node with periodically wrapped coordinates, so tiles that
// cross the domain edge (or are wider than the domain) need no special case: threads
// outside the domain compute psi of the wrapped node but never store.
#pragma once

#include <type_traits>

#include "common.h"

namespace lbmk {

// Cache hints of the fused step (bit flags, uniform per launch):
//   kHintNtStore      populations written by a step are stored with the nontemporal hint
//                     (not read again within the step, so they need not displace the halo
//                     rows other tiles are about to pull);
//   kHintNtInterior   prefetching tiles load the own pulls of their interior rows (read by
//                     no other tile) with the nontemporal hint.
// The store hint is a template parameter of the kernels (the host picks the instantiation):
// a run-time branch between a plain and a nontemporal store of the same value to the same
// address is merged by the compiler into one plain store, and two inlined copies of a tile
// would double its LDS and spill.
constexpr int kHintNtStore = 1, kHintNtInterior = 2;

// Launch configurations of the fused step: tile width and height, whether the tile spans
// the whole x row (then nx must equal tx), and pf: the next planes are prefetched into LDS
// (k_step_fused_pf; 2- or 4-byte storage, and the populations of a tile plus its halo rows
// must fit in LDS). Full rows of 256, 320 and 384 nodes; 64x8 (4-byte storage) or 64x4
// tiles serve other widths (32x8 tiles remain as configuration 0).
// Full-row tiles cut z into chunks sized for whole rounds of one workgroup per CU (each holds
// a CU alone: LDS or VGPRs), so every workgroup marches as far as possible and the two
// lead-in planes of a chunk are paid rarely; small tiles march through 16-plane chunks. Both
// map tiles to XCDs in contiguous ranges.
struct FusedCfg { int tx, ty; bool fullx, pf; };
constexpr FusedCfg kFusedCfgs[] = {{32, 8, false, false}, {256, 2, true, false},
                                   {256, 4, true, false}, {256, 4, true, true},
                                   {256, 2, true, true},  {320, 2, true, false},
                                   {320, 2, true, true},  {384, 2, true, false},
                                   {384, 2, true, true},  {64, 4, false, false},
                                   {64, 8, false, false}};
constexpr int kNumFusedCfgs = sizeof(kFusedCfgs) / sizeof(kFusedCfgs[0]);
constexpr int kFusedZcTiled = 16, kFusedZcMin = 8;

// LDS bytes of a prefetching tile: psi ring, own-plane and halo population buffers.
constexpr int fused_pf_lds_bytes(int Q, int tx, int ty, bool fullx = true) {
    return fullx ? 4 * (4 * (ty + 2) * tx + Q * tx * ty + Q * 2 * tx)
                 : 4 * (4 * (ty + 2) * (tx + 2) + Q * tx * ty + Q * (2 * (tx + ty) + 4));
}
constexpr int kLdsBytesPerCU = 160 * 1024;
// LDS bytes of an FP64 full-row tile with own-population prefetch: psi ring (8-byte) and the
// two dword slot arrays of the own buffer.
constexpr int fused_pf64_lds_bytes(int Q, int tx, int ty) {
    return 4 * (ty + 2) * tx * 8 + 2 * Q * tx * ty * 4;
}

// Planes per z-chunk for full-row tiles: nz is cut into n chunks, n minimising
// rounds(n) x (planes per chunk + 2 lead-in planes), where a round is one workgroup on each
// of the cus CUs; e.g. 64 planes for 256x4 and 128 for 256x2 tiles at 256^3 (one round),
// 48 for 384x2 tiles at 384^2 x 192 (three rounds of 256 over 192 tiles x 4 chunks), 8 for
// a 256 x 256 x 32 slab (one GPU's share of 256^3 on eight: 70 us per step with 8-plane
// chunks, 100 us with 16, 173 us with 32).
// Measured at 256^3, ms per step, 128- vs 64-plane chunks with 256x2 tiles: D3Q19 FP64 1.20
// vs 1.24, D3Q27 FP32 0.756 vs 0.816, D3Q27 FP64 2.29 vs 2.34, D3Q27 FP16 0.602 vs 0.638.
constexpr int default_fused_zc(const FusedCfg& c, long long tiles, int nz, int cus) {
    if (!c.fullx) return kFusedZcTiled;
    const int nmax = nz / kFusedZcMin < 1 ? 1 : (nz / kFusedZcMin > 64 ? 64 : nz / kFusedZcMin);
    int best_zc = nz;
    long long best = -1;
    for (int n = 1; n <= nmax; ++n) {
        const int zc = (nz + n - 1) / n;
        const long long chunks = (nz + zc - 1) / zc;
        const long long rounds = (tiles * chunks + cus - 1) / cus;
        const long long cost = rounds * (zc + 2);
        if (best < 0 || cost < best) { best = cost; best_zc = zc; }
    }
    return best_zc;
}
constexpr int default_fused_remap(const FusedCfg&) { return 1; }
// Cache hints (measured at 256^3, ms per step, plain stores vs nontemporal stores): full-row
// prefetching 256x4 tiles, D3Q19 FP32 0.526 vs 0.486 (0.482 with nontemporal interior loads
// too), FP16 0.323 vs 0.302; FP64 own-population prefetch 256x2, D3Q27 2.30 vs 2.11; plain
// 256x2 tiles, D3Q27 FP16 0.607 vs 0.585. Plain stores elsewhere: prefetching 256x2 tiles,
// D3Q27 FP32 0.761 vs 0.830; plain 256x2, D3Q19 FP64 1.19 vs 1.21; 32x8 tiles (300^2 x 250)
// 1.30 vs 1.69 D3Q19 FP32, 1.86 vs 2.40 D3Q27 FP32, 2.08 vs 2.28 D3Q19 FP64 (a nontemporal
// store of a partly written cache line costs more than a cached one).
constexpr int default_fused_hints(const FusedCfg& c, int elem_bytes) {
    if (!c.fullx) return 0;
    if (c.pf && elem_bytes == 4) return c.ty == 4 ? kHintNtStore | kHintNtInterior : 0;
    return (elem_bytes == 2 || (c.pf && elem_bytes == 8)) ? kHintNtStore : 0;
}

// Default configuration for a 256-wide domain (measured at 256^3, ms per step; the
// comparisons made with 64-plane chunks are marked "64"):
//   4-byte storage: prefetching 256x4 tiles where they fit in LDS (D3Q19: 0.506 vs 0.536
//     plain), else prefetching 256x2 tiles (D3Q27: 0.76-0.78; 64: 0.800 vs 0.926 plain
//     256x2, 1.142 plain 256x4, which spills);
//   8-byte storage: plain 256x2 tiles for D3Q19 (1.19-1.22 vs 1.26-1.28 with the
//     own-population prefetch of k_step_fused_pf64; 256x4 spills), prefetching 256x2 for
//     D3Q27 (2.29-2.33; 64: 2.36 vs 2.56 plain, 4.10 plain 256x4);
//   2-byte storage: prefetching 256x4 for D3Q19 (0.320 vs 0.342 plain), plain 256x2 for
//     D3Q27 (0.602-0.609 vs 0.645 prefetching; 64: 0.92 plain 256x4).
// Other widths (GLUPS; 32x8 / 64x4 / 64x8 / 128x4 tiles): 300^2 x 250 D3Q19 FP32 17.4 / 21.8 /
// 23.3 / 22.5, D3Q27 FP32 13.0 / 14.7 / 14.9 / 13.7, D3Q27 FP16 19.5 / 23.1 / 20.5 / 19.3,
// D3Q27 FP32 with walls 12.7 / 13.8 / 14.5 / 13.9; 200^3 D3Q19 FP32 17.4 / 18.7 / 18.2 / 20.0;
// FP64 384^2 x 160 D3Q19 12.3 / 12.9 / 12.9 / 12.5, 320 x 256 x 192 D3Q27 cylinder 6.0 / 6.4 /
// 6.2 / 5.6: 64x8 for 4-byte storage, 64x4 otherwise.
// 320- and 384-wide domains (GLUPS; 2-row full-row tiles vs 32x8 tiles): D3Q19 prefetching
// (FP32 384^2 x 192 30.0 vs 22.0, 27.3 plain; 320 x 256 x 192 28.6 vs 22.2; FP16 384^2 x 192
// 43-45 vs 30.7), D3Q27 plain (320 x 256 x 192 FP32 19.3 vs 15.5, 19.3 prefetching, which
// spills; FP16 28.1 vs 21.5); FP64 takes 64x4 tiles (32x8: 12.3-12.7 vs 9.4 at 384^2 x 160,
// 6.7-7.1 vs 5.4-5.6 for D3Q27 at 320 x 256 x 192: 640 or 768 threads leave too few VGPRs).
// D3Q27 on a solid mask at width 320 (the cylinder workload, 320 x 256 x 192, walls and a
// cylinder with wetting): prefetching 320x2 tiles, FP32 0.90 vs 0.98 ms plain, FP16 0.80 vs
// 0.78 with the solid-free segments (1.02 vs 1.22-1.26 and 0.92 vs 0.99-1.03 without them);
// the masked form holds 161 VGPRs without spills, between plain walls it spills.
constexpr int default_fused_cfg_index(int nx, int elem_bytes, int Q, bool mask = false) {
    return (nx == 320 || nx == 384)
               ? (elem_bytes == 8 ? 9
                  : Q == 19 && fused_pf_lds_bytes(Q, nx, 2) <= kLdsBytesPerCU ? (nx == 320 ? 6 : 8)
                  : nx == 320 ? (mask && fused_pf_lds_bytes(Q, nx, 2) <= kLdsBytesPerCU ? 6 : 5)
                  : 7)
         : nx != 256 ? (elem_bytes == 4 ? 10 : 9)
         : elem_bytes == 8 ? (Q == 27 && fused_pf64_lds_bytes(Q, 256, 2) <= kLdsBytesPerCU ? 4 : 1)
         : elem_bytes == 4 ? (fused_pf_lds_bytes(Q, 256, 4) <= kLdsBytesPerCU ? 3
                              : fused_pf_lds_bytes(Q, 256, 2) <= kLdsBytesPerCU ? 4 : 1)
         : (Q == 19 && fused_pf_lds_bytes(Q, 256, 4) <= kLdsBytesPerCU ? 3 : 1);
}

// Workgroup b -> tile index such that each XCD (b mod 8) gets a contiguous tile range.
__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int q = nb / 8, r = nb % 8;
    const int xcd = b % 8, k = b / 8;
    return xcd * q + (xcd < r ? xcd : r) + k;
}

// Byte offsets from the buffer base: 32-bit (buffers below 4 GiB, the scalar base plus a
// 32-bit vector offset) or 64-bit (larger buffers, the plain small-tile kernel only).
template <bool WIDE> struct OffSel { using type = unsigned; };
template <> struct OffSel<true> { using type = size_t; };

template <typename T, typename Off>
__device__ __forceinline__ T ld_off(const T* __restrict__ base, Off byte_off) {
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byte_off);
}
template <typename T, typename Off>
__device__ __forceinline__ void st_off(T* __restrict__ base, Off byte_off, T v) {
    *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off) = v;
}
// Streaming store (nontemporal hint).
template <typename T, typename Off>
__device__ __forceinline__ void st_off_nt(T* __restrict__ base, Off byte_off, T v) {
    __builtin_nontemporal_store(v, reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byte_off));
}

// How a kernel learns which nodes are solid: none (fully periodic), wall layers only
// (decided from the coordinates, no memory traffic), or the link words built from the
// solid mask (cylinder).
enum { GEOM_NONE = 0, GEOM_WALLS = 1, GEOM_MASK = 2 };

// Wall solidity of the coordinates c-1, c, c+1 (wrapped) along one axis, as bits 0..2.
__device__ __forceinline__ unsigned wall_bits(int c, int n, int walls, int axis) {
    const bool lo = (walls >> (2 * axis)) & 1, hi = (walls >> (2 * axis + 1)) & 1;
    unsigned b = 0;
#pragma unroll
    for (int d = -1; d <= 1; ++d) {
        int cc = c + d;
        cc = cc < 0 ? cc + n : (cc >= n ? cc - n : cc);
        if ((lo && cc == 0) || (hi && cc == n - 1)) b |= 1u << (d + 1);
    }
    return b;
}
struct WallBits { unsigned wx, wy, wz; };

// Element index of the pull source x - e_i of population i for a column whose 3x3
// in-plane neighbour indices are xy[(dy+1)*3 + dx+1] and whose plane indices are
// zo[dz+1]; with bounce-back from the node itself when the source is solid. lk: the node's
// link word (GEOM_MASK; bit i set when x - e_i is solid).
template <int Q, int GEOM>
__device__ __forceinline__ void pull_source(int i, const int* xy, const int* zo, unsigned lk,
                                            const WallBits& wb, int& e, int& pop) {
    const int ex = vel_x(i), ey = vel_y(i), ez = vel_z(i);
    e = xy[(1 - ey) * 3 + (1 - ex)] + zo[1 - ez];
    pop = i;
    bool s = false;
    if (GEOM == GEOM_MASK && i != 0) s = (lk >> i) & 1u;
    if (GEOM == GEOM_WALLS && i != 0)
        s = ((wb.wx >> (1 - ex)) | (wb.wy >> (1 - ey)) | (wb.wz >> (1 - ez))) & 1u;
    if (s) { e = xy[4] + zo[1]; pop = opposite(i); }
}

// Link word of node n for the solid mask (bit 0: the node is solid; bit i: its neighbour
// x - e_i is solid), 0 without a mask: one 4-byte load replaces a byte load per population.
template <int GEOM>
__device__ __forceinline__ unsigned link_word(const uint32_t* __restrict__ links, int n) {
    if constexpr (GEOM == GEOM_MASK) return links[n];
    return 0u;
}

template <int GEOM>
__device__ __forceinline__ bool node_solid(const uint32_t* __restrict__ links, int n,
                                           const WallBits& wb) {
    if (GEOM == GEOM_MASK) return links[n] & 1u;
    if (GEOM == GEOM_WALLS) return ((wb.wx | wb.wy | wb.wz) >> 1) & 1u;
    return false;
}

// Issue the Q loads of a column's node (values land in v[]).
template <int Q, typename T, typename R, int GEOM, typename Off = unsigned>
__device__ __forceinline__ void pull_loads(const T* __restrict__ f, const uint32_t* __restrict__ links,
                                           const int* xy, const int* zo, const WallBits& wb,
                                           Off pst, R* v) {
    const unsigned lk = link_word<GEOM>(links, xy[4] + zo[1]);
#pragma unroll
    for (int i = 0; i < Q; ++i) {
        int e, pop;
        pull_source<Q, GEOM>(i, xy, zo, lk, wb, e, pop);
        v[i] = static_cast<R>(ld_off(f, (Off)e * (Off)sizeof(T) + (Off)pop * pst));
    }
}

template <int Q, typename R>
__device__ __forceinline__ R sum_q(const R* v) {
    R s = 0;
#pragma unroll
    for (int i = 0; i < Q; ++i) s += v[i];
    return s;
}

// LDS of one tile shape, shared by the geometry forms of that shape: a kernel that runs the
// solid-free form of its tile on some planes (fused_segments) then holds one copy of the
// tile's buffers, not one per form.
template <typename R, int LY, int LX>
struct RingLds { R ring[4][LY][LX]; };
template <typename R, int LY, int LX>
__device__ __forceinline__ RingLds<R, LY, LX>& ring_lds() {
    __shared__ RingLds<R, LY, LX> s;
    return s;
}
template <typename S, int Q, int LY, int LX, int NT, int H>
struct PfLds {
    float ring[4][LY][LX];
    S own[Q][NT];
    S halo[Q][H];
};
template <typename S, int Q, int LY, int LX, int NT, int H>
__device__ __forceinline__ PfLds<S, Q, LY, LX, NT, H>& pf_lds() {
    __shared__ PfLds<S, Q, LY, LX, NT, H> s;
    return s;
}

// Solid-free form. A walled or cylinder lattice runs the general form of its tile, with
// bounce-back in the pulls, solid tests and wetting sums over the neighbours and the mirror
// reading of psi at solid ones. Only planes within two of a solid node need it: a plane z
// whose planes z - 2 .. z + 2 hold no solid node pulls without bounce-back, reads the psi of
// fluid nodes only (its own and, through its ring, planes z - 1 .. z + 1, each from pulls
// within one more plane) and has no solid or wetting terms, so the form of the tile for a
// lattice without solid nodes gives its nodes the same values (up to the sign of exact
// zeros). The host gives the longest run of such planes as [g.sf0, g.sf1); a workgroup splits
// its chunk into a general and a solid-free segment, each marched like a chunk of its own
// (with its two lead-in planes), a barrier between them so that the ring and the prefetch
// buffers are free again. 2- and 4-byte storage only; FP64 tiles always take the general
// form.
template <typename T, int GEOM, typename F>
__device__ __forceinline__ void fused_segments(const Grid& g, int z0, int z1, F&& run) {
    if constexpr (GEOM == GEOM_NONE || sizeof(T) == 8) {
        run(std::integral_constant<int, GEOM>{}, z0, z1);
    } else {
        // one general segment and one solid-free segment at most, one call site each (a
        // chunk that would need general segments on both sides runs wholly in the general
        // form): segments are independent, so the general one runs first
        int glo = z0, ghi = z1, flo = z1, fhi = z1;
        const int a = max(z0, g.sf0), b = min(z1, g.sf1);
        if (a < b && (a == z0 || b == z1)) {
            flo = a;
            fhi = b;
            glo = a == z0 ? b : z0;
            ghi = a == z0 ? z1 : a;
        }
        if (glo < ghi) run(std::integral_constant<int, GEOM>{}, glo, ghi);
        if (flo < fhi) {
            if (glo < ghi) __syncthreads();
            run(std::integral_constant<int, GEOM_NONE>{}, flo, fhi);
        }
    }
}

// FULLX: the tile spans the whole x extent (TX == nx); x wraps inside the tile and the
// halo is just the rows y0-1 and y0+TY (H = 2 TX, one halo node per thread when TY = 2).
// Planes z0 .. z1 - 1 of tile (column) t of a domain with ntx x nty tiles per plane, in the
// geometry form GEOM.
template <int Q, typename T, int GEOM, int TX, int TY, bool FULLX, bool NTS, bool WIDE = false>
__device__ __forceinline__ void fused_tile_seg(const T* __restrict__ fin, T* __restrict__ fout,
                                               const uint32_t* __restrict__ links, const Grid& g,
                                               const Phys<typename Arith<T>::type>& P,
                                               int t, int ntx, int nty, int z0, int z1, int hints) {
    using R = typename Arith<T>::type;
    constexpr int LX = FULLX ? TX : TX + 2, LY = TY + 2;
    constexpr int OX = FULLX ? 0 : 1;                 // LDS column of tile column 0
    constexpr int H = FULLX ? 2 * TX : 2 * (TX + TY) + 4;
    static_assert(H <= TX * TY, "halo larger than the workgroup");
    auto& ring = ring_lds<R, LY, LX>().ring;

    const int ix = t % ntx; t /= ntx;
    const int iy = t % nty;
    const int x0 = ix * TX, y0 = iy * TY;
    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int x = x0 + lx, y = y0 + ly;
    const bool active = x < g.nx && y < g.ny;
    auto wrapc = [](int c, int n) { c %= n; return c < 0 ? c + n : c; };
    const int nxy = g.nx * g.ny;
    using Off = typename OffSel<WIDE>::type;
    const Off pst = (Off)g.stride * (Off)sizeof(T);   // plane stride, bytes

    // halo cell of this thread (if any), as tile coordinates (hx, hy)
    int hx = 0, hy = 0;
    const bool has_halo = tid < H;
    if (has_halo) {
        if (FULLX) { hx = tid % TX; hy = tid < TX ? -1 : TY; }
        else if (tid < LX) { hx = tid - 1; hy = -1; }
        else if (tid < 2 * LX) { hx = tid - LX - 1; hy = TY; }
        else if (tid < 2 * LX + TY) { hx = -1; hy = tid - 2 * LX; }
        else { hx = TX; hy = tid - 2 * LX - TY; }
    }
    // in-plane indices of the 3x3 neighbourhood of the own column and of the halo column
    int oxy[9], hxy[9];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            oxy[(dy + 1) * 3 + dx + 1] = wrapc(x + dx, g.nx) + wrapc(y + dy, g.ny) * g.nx;
            hxy[(dy + 1) * 3 + dx + 1] =
                wrapc(x0 + hx + dx, g.nx) + wrapc(y0 + hy + dy, g.ny) * g.nx;
        }
    auto zoffs = [&](int zp, int* zo) {
        zo[0] = wrapc(zp - 1, g.nz) * nxy;
        zo[1] = wrapc(zp, g.nz) * nxy;
        zo[2] = wrapc(zp + 1, g.nz) * nxy;
    };
    // wall solidity of the own and the halo column (x, y fixed; z per plane)
    WallBits wo{0u, 0u, 0u}, wh{0u, 0u, 0u};
    if (GEOM == GEOM_WALLS) {
        wo.wx = wall_bits(wrapc(x, g.nx), g.nx, g.walls, 0);
        wo.wy = wall_bits(wrapc(y, g.ny), g.ny, g.walls, 1);
        wh.wx = wall_bits(wrapc(x0 + hx, g.nx), g.nx, g.walls, 0);
        wh.wy = wall_bits(wrapc(y0 + hy, g.ny), g.ny, g.walls, 1);
    }
    auto zbits = [&](int zp) {
        return GEOM == GEOM_WALLS ? wall_bits(wrapc(zp, g.nz), g.nz, g.walls, 2) : 0u;
    };
    auto psi_of = [&](R drho) { return pseudopotential<R>(P.rho_ref + drho, P); };
    // psi of the halo node of plane zp into ring slot
    auto halo_psi = [&](int zp, int slot) {
        if (!has_halo) return;
        int zo[3];
        zoffs(zp, zo);
        const WallBits wb{wh.wx, wh.wy, zbits(zp)};
        R hv;
        if (node_solid<GEOM>(links, hxy[4] + zo[1], wb)) hv = R(-1);
        else {
            R v[Q];
            pull_loads<Q, T, R, GEOM, Off>(fin, links, hxy, zo, wb, pst, v);
            hv = psi_of(sum_q<Q, R>(v));
        }
        ring[slot][hy + 1][hx + OX] = hv;
    };
    // own node of plane zp: loads into v, psi into ring slot
    auto own_psi = [&](int zp, int slot, R* v) {
        int zo[3];
        zoffs(zp, zo);
        const WallBits wb{wo.wx, wo.wy, zbits(zp)};
        const bool s = node_solid<GEOM>(links, oxy[4] + zo[1], wb);
        pull_loads<Q, T, R, GEOM, Off>(fin, links, oxy, zo, wb, pst, v);
        ring[slot][ly + 1][lx + OX] = s ? R(-1) : psi_of(sum_q<Q, R>(v));
    };
    // LDS column of tile column lx + dx
    auto col = [&](int dx) {
        if (!FULLX) return lx + 1 + dx;
        const int c = lx + dx;
        return c < 0 ? c + TX : (c >= TX ? c - TX : c);
    };
    auto collide_store = [&](R* c, int z, int s0, int s1, int s2) {
        const R psi0 = ring[s1][ly + 1][lx + OX];
        if (active && !(psi0 < R(0))) {
            R pn[Q];
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                const int ez = vel_z(j);
                const int sl = ez < 0 ? s0 : (ez > 0 ? s2 : s1);
                pn[j] = ring[sl][ly + 1 + vel_y(j)][col(vel_x(j))];
            }
            const NodeForce<R> nf = node_force<Q, R, GEOM != GEOM_NONE>(psi0, pn, P);
            collide<Q, R>(c, nf, P);
            const Off nb = (Off)(oxy[4] + z * nxy) * (Off)sizeof(T);
            if constexpr (NTS) {
#pragma unroll
                for (int i = 0; i < Q; ++i) st_off_nt(fout, nb + (Off)i * pst, static_cast<T>(c[i]));
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) st_off(fout, nb + (Off)i * pst, static_cast<T>(c[i]));
            }
        }
    };

    R cur[Q], nxt[Q];
    own_psi(z0 - 1, 0, nxt);
    halo_psi(z0 - 1, 0);
    own_psi(z0, 1, cur);
    halo_psi(z0, 1);
    for (int z = z0; z < z1; ++z) {
        const int k = z - z0;
        own_psi(z + 1, (k + 2) & 3, nxt);
        halo_psi(z + 1, (k + 2) & 3);
        __syncthreads();
        collide_store(cur, z, k & 3, (k + 1) & 3, (k + 2) & 3);
#pragma unroll
        for (int i = 0; i < Q; ++i) cur[i] = nxt[i];
    }
}

// One tile (workgroup) of the fused step: tile index t of a domain with ntx x nty tiles
// per plane and z-chunks of zc planes. Shared by the single-domain kernel and the
// multi-domain (batched) kernel.
template <int Q, typename T, int GEOM, int TX, int TY, bool FULLX, bool NTS, bool WIDE = false>
__device__ __forceinline__ void fused_tile(const T* __restrict__ fin, T* __restrict__ fout,
                                           const uint32_t* __restrict__ links, const Grid& g,
                                           const Phys<typename Arith<T>::type>& P,
                                           int t, int ntx, int nty, int zc, int hints) {
    const int z0 = t / (ntx * nty) * zc, z1 = min(z0 + zc, g.nz);
    fused_segments<T, GEOM>(g, z0, z1, [&](auto form, int a, int b) {
        fused_tile_seg<Q, T, decltype(form)::value, TX, TY, FULLX, NTS, WIDE>(fin, fout, links, g,
                                                                             P, t, ntx, nty, a, b,
                                                                             hints);
    });
}

#define LBM_LDS_PTR(p) ((__attribute__((address_space(3))) void*)(p))

// Wait until every vector memory operation of this wavefront has completed (vmcnt(0); the
// expcnt and lgkmcnt fields at their maxima, i.e. not waited for).
__device__ __forceinline__ void wait_vector_memory() { __builtin_amdgcn_s_waitcnt(0x0F70); }
// Wait until at most N vector memory operations of this wavefront are outstanding (vmcnt(N):
// bits 3:0 and 15:14 of the immediate). Vector memory operations complete in issue order,
// loads into VGPRs or LDS and stores alike (the compiler's own waits for a load followed by
// a store count on this too), so when the last N issued were stores this waits for
// everything issued before them and lets the stores drain.
template <int N>
__device__ __forceinline__ void wait_vector_memory_but() {
    static_assert(N >= 0 && N < 64, "vmcnt is a 6-bit field");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}
// Workgroup barrier for LDS traffic only: every wavefront's LDS accesses complete, then
// s_barrier. Unlike __syncthreads it does not wait for outstanding vector memory operations
// (the asynchronous LDS loads in flight are read back only by the lanes that issued them,
// after their own vmcnt wait). The memory clobber keeps the compiler from moving memory
// accesses across it.
__device__ __forceinline__ void barrier_lds() {
    asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");
}
// Wait until every LDS access of this wavefront has completed (lgkmcnt(0); vmcnt and expcnt
// at their maxima): LDS cells just read may then be overwritten by an asynchronous load.
__device__ __forceinline__ void wait_lds() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// One full-row tile of the fused step with the populations of the plane ahead streamed from
// HBM straight into LDS (global_load_lds: no VGPRs held while in flight). With one
// 1024-thread workgroup per CU the plain tile alternates a load phase and an arithmetic
// phase; here the loads of plane z+2 are in flight while plane z is collided:
//   wait for plane z+1 -> psi of the halo node from its LDS buffer -> refill that buffer
//   with plane z+2 -> own populations of z+1 from LDS into registers, psi -> refill -> LDS
//   barrier -> psi(z-1..z+1) of the neighbourhood from the ring -> collide and store z.
// Each lane reads back only the LDS cells its own loads wrote, so the prefetch buffers need
// no barrier, and the barrier waits for LDS accesses only (a __syncthreads would also wait
// for the loads in flight); the ring slot written at plane z+1 was last read at plane z-1,
// one barrier earlier. The arithmetic per node is the one of fused_tile (same functions,
// same order), so both give bitwise identical results.
// Asynchronous load of one element per lane from global memory into LDS (the lane's element
// lands at dst + 4 * lane); AUX selects the cache policy (0 default, 2 nontemporal).
// (The builtin takes its size and policy as literal constants, hence one specialization each.)
// The LDS destination is a wave-uniform byte address (it goes to M0): callers form it with
// scalar arithmetic from lds_addr(), so no per-load readfirstlane is needed.
#define LBM_LDS_AT(a) ((__attribute__((address_space(3))) void*)(a))
template <int SIZE, int AUX> __device__ __forceinline__ void lds_dma(const char* src, uint32_t dst);
template <> __device__ __forceinline__ void lds_dma<4, 0>(const char* src, uint32_t dst) {
    __builtin_amdgcn_global_load_lds(src, LBM_LDS_AT(dst), 4, 0, 0);
}
template <> __device__ __forceinline__ void lds_dma<4, 2>(const char* src, uint32_t dst) {
    __builtin_amdgcn_global_load_lds(src, LBM_LDS_AT(dst), 4, 0, 2);
}
template <> __device__ __forceinline__ void lds_dma<2, 0>(const char* src, uint32_t dst) {
    __builtin_amdgcn_global_load_lds(src, LBM_LDS_AT(dst), 2, 0, 0);
}
template <> __device__ __forceinline__ void lds_dma<2, 2>(const char* src, uint32_t dst) {
    __builtin_amdgcn_global_load_lds(src, LBM_LDS_AT(dst), 2, 0, 2);
}
// Wave-uniform LDS byte address of a shared object (as a scalar).
__device__ __forceinline__ uint32_t lds_addr(const void* p) {
    return __builtin_amdgcn_readfirstlane((uint32_t)(size_t)LBM_LDS_PTR(p));
}

// Prefetch slots: the LDS DMA writes each lane's element into a dword of its own (a 2-byte
// element zero-extended into the low half), so 2-byte storage uses 4-byte slots.
template <typename T> struct PfSlot { using type = T; };
template <> struct PfSlot<_Float16> { using type = uint32_t; };
template <typename T, typename R>
__device__ __forceinline__ R pf_value(typename PfSlot<T>::type v) { return static_cast<R>(v); }
template <>
__device__ __forceinline__ float pf_value<_Float16, float>(uint32_t v) {
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(v)));
}

template <int Q, typename T, int GEOM, int TX, int TY, bool FULLX, bool NTS>
__device__ __forceinline__ void fused_tile_pf_seg(const T* __restrict__ fin, T* __restrict__ fout,
                                                  const uint32_t* __restrict__ links, const Grid& g,
                                                  const Phys<float>& P, int t, int ntx, int nty,
                                                  int z0, int z1, int hints) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 2, "the LDS prefetch moves 2- or 4-byte elements");
    using R = float;
    using S = typename PfSlot<T>::type;
    constexpr int NT = TX * TY;
    constexpr int LX = FULLX ? TX : TX + 2;
    constexpr int OX = FULLX ? 0 : 1;                 // LDS column of tile column 0
    constexpr int H = FULLX ? 2 * TX : 2 * (TX + TY) + 4;
    static_assert(H <= NT && (!FULLX || TX % 64 == 0),
                  "halo larger than the tile, or full rows not whole wavefronts");
    static_assert(fused_pf_lds_bytes(Q, TX, TY, FULLX) <= kLdsBytesPerCU, "tile does not fit in LDS");
    // the halo buffer holds H cells; the DMA of the last, partly used wavefront writes only
    // its active lanes
    auto& lds = pf_lds<S, Q, TY + 2, LX, NT, H>();
    auto& ring = lds.ring;
    auto& pf_own = lds.own;
    auto& pf_halo = lds.halo;
    // this wavefront's slots of population 0 in the two buffers (scalars)
    const uint32_t own_lds = lds_addr(&pf_own[0][(threadIdx.x >> 6) * 64]);
    const uint32_t halo_lds = lds_addr(&pf_halo[0][(threadIdx.x >> 6) * 64]);

    const int ix = t % ntx; t /= ntx;
    const int iy = t % nty;
    const int x0 = ix * TX, y0 = iy * TY;
    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int x = x0 + lx, y = y0 + ly;
    const bool active = x < g.nx && y < g.ny;
    auto wrapc = [](int c, int n) { c %= n; return c < 0 ? c + n : c; };
    const int nxy = g.nx * g.ny;
    const unsigned pst = (unsigned)g.stride * (unsigned)sizeof(T);

    // halo cell of this thread (if any), as tile coordinates (hx, hy)
    int hx = 0, hy = 0;
    const bool has_halo = tid < H;
    if (has_halo) {
        if (FULLX) { hx = tid % TX; hy = tid < TX ? -1 : TY; }
        else if (tid < LX) { hx = tid - 1; hy = -1; }
        else if (tid < 2 * LX) { hx = tid - LX - 1; hy = TY; }
        else if (tid < 2 * LX + TY) { hx = -1; hy = tid - 2 * LX; }
        else { hx = TX; hy = tid - 2 * LX - TY; }
    }
    int oxy[9], hxy[9];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            oxy[(dy + 1) * 3 + dx + 1] = wrapc(x + dx, g.nx) + wrapc(y + dy, g.ny) * g.nx;
            hxy[(dy + 1) * 3 + dx + 1] =
                wrapc(x0 + hx + dx, g.nx) + wrapc(y0 + hy + dy, g.ny) * g.nx;
        }
    auto zoffs = [&](int zp, int* zo) {
        zo[0] = wrapc(zp - 1, g.nz) * nxy;
        zo[1] = wrapc(zp, g.nz) * nxy;
        zo[2] = wrapc(zp + 1, g.nz) * nxy;
    };
    WallBits wo{0u, 0u, 0u}, wh{0u, 0u, 0u};
    if (GEOM == GEOM_WALLS) {
        wo.wx = wall_bits(wrapc(x, g.nx), g.nx, g.walls, 0);
        wo.wy = wall_bits(wrapc(y, g.ny), g.ny, g.walls, 1);
        wh.wx = wall_bits(wrapc(x0 + hx, g.nx), g.nx, g.walls, 0);
        wh.wy = wall_bits(wrapc(y0 + hy, g.ny), g.ny, g.walls, 1);
    }
    auto zbits = [&](int zp) {
        return GEOM == GEOM_WALLS ? wall_bits(wrapc(zp, g.nz), g.nz, g.walls, 2) : 0u;
    };
    auto psi_of = [&](R drho) { return pseudopotential<R>(P.rho_ref + drho, P); };
    // LDS column of tile column lx + dx
    auto col = [&](int dx) {
        if (!FULLX) return lx + 1 + dx;
        const int c = lx + dx;
        return c < 0 ? c + TX : (c >= TX ? c - TX : c);
    };

    // synchronous pulls (first two planes of the chunk)
    auto own_psi = [&](int zp, int slot, R* v) {
        int zo[3];
        zoffs(zp, zo);
        const WallBits wb{wo.wx, wo.wy, zbits(zp)};
        const bool s = node_solid<GEOM>(links, oxy[4] + zo[1], wb);
        pull_loads<Q, T, R, GEOM>(fin, links, oxy, zo, wb, pst, v);
        ring[slot][ly + 1][lx + OX] = s ? R(-1) : psi_of(sum_q<Q, R>(v));
    };
    auto halo_psi = [&](int zp, int slot) {
        if (!has_halo) return;
        int zo[3];
        zoffs(zp, zo);
        const WallBits wb{wh.wx, wh.wy, zbits(zp)};
        R hv;
        if (node_solid<GEOM>(links, hxy[4] + zo[1], wb)) hv = R(-1);
        else {
            R v[Q];
            pull_loads<Q, T, R, GEOM>(fin, links, hxy, zo, wb, pst, v);
            hv = psi_of(sum_q<Q, R>(v));
        }
        ring[slot][hy + 1][hx + OX] = hv;
    };
    // asynchronous pulls of plane zp into the LDS buffers (own node, halo node)
    // Own pulls of the interior rows of a full-row tile are read by no other tile
    // (kHintNtInterior). A wavefront covers part of one row (TX is a multiple of 64), so
    // the choice is uniform.
    const bool interior_row = FULLX && (hints & kHintNtInterior) && ly != 0 && ly != TY - 1;
    auto prefetch_own = [&](int zp) {
        int zo[3];
        zoffs(zp, zo);
        const WallBits wb{wo.wx, wo.wy, zbits(zp)};
        const unsigned lk = link_word<GEOM>(links, oxy[4] + zo[1]);
        if (interior_row) {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                int e, pop;
                pull_source<Q, GEOM>(i, oxy, zo, lk, wb, e, pop);
                lds_dma<(int)sizeof(T), 2>(
                    reinterpret_cast<const char*>(fin) + ((unsigned)e * (unsigned)sizeof(T) + (unsigned)pop * pst),
                    own_lds + (uint32_t)(i * NT * sizeof(S)));
            }
        } else {
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                int e, pop;
                pull_source<Q, GEOM>(i, oxy, zo, lk, wb, e, pop);
                lds_dma<(int)sizeof(T), 0>(
                    reinterpret_cast<const char*>(fin) + ((unsigned)e * (unsigned)sizeof(T) + (unsigned)pop * pst),
                    own_lds + (uint32_t)(i * NT * sizeof(S)));
            }
        }
    };
    auto prefetch_halo = [&](int zp) {
        if (!has_halo) return;
        int zo[3];
        zoffs(zp, zo);
        const WallBits hb{wh.wx, wh.wy, zbits(zp)};
        const unsigned lk = link_word<GEOM>(links, hxy[4] + zo[1]);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int e, pop;
            pull_source<Q, GEOM>(i, hxy, zo, lk, hb, e, pop);
            lds_dma<(int)sizeof(T), 0>(
                reinterpret_cast<const char*>(fin) + ((unsigned)e * (unsigned)sizeof(T) + (unsigned)pop * pst),
                halo_lds + (uint32_t)(i * H * sizeof(S)));
        }
    };
    // plane zp from the LDS buffers: psi of the halo node; own populations into v and psi
    auto take_halo = [&](int zp, int slot) {
        if (!has_halo) return;
        int zo[3];
        zoffs(zp, zo);
        const WallBits hb{wh.wx, wh.wy, zbits(zp)};
        R hv;
        if (node_solid<GEOM>(links, hxy[4] + zo[1], hb)) hv = R(-1);
        else {
            R s = 0;
#pragma unroll
            for (int i = 0; i < Q; ++i) s += pf_value<T, R>(pf_halo[i][tid]);
            hv = psi_of(s);
        }
        ring[slot][hy + 1][hx + OX] = hv;
    };
    auto take_own = [&](int zp, int slot, R* v) {
        int zo[3];
        zoffs(zp, zo);
        const WallBits wb{wo.wx, wo.wy, zbits(zp)};
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = pf_value<T, R>(pf_own[i][tid]);
        ring[slot][ly + 1][lx + OX] =
            node_solid<GEOM>(links, oxy[4] + zo[1], wb) ? R(-1) : psi_of(sum_q<Q, R>(v));
    };

    R cur[Q], nxt[Q];
    own_psi(z0 - 1, 0, nxt);
    halo_psi(z0 - 1, 0);
    own_psi(z0, 1, cur);
    halo_psi(z0, 1);
    prefetch_halo(z0 + 1);
    prefetch_own(z0 + 1);
    // true when this wavefront's last vector memory operations were the Q stores of the
    // previous plane (some lane stored, so all Q store instructions were issued): the wait
    // for the prefetched plane then leaves those stores in flight
    bool stored = false;
    for (int z = z0; z < z1; ++z) {
        const int k = z - z0;
        const int s0 = k & 3, s1 = (k + 1) & 3, s2 = (k + 2) & 3;
        const bool more = z + 1 < z1;
        if (stored) wait_vector_memory_but<Q>();
        else wait_vector_memory();
        // each buffer is refilled with plane z+2 as soon as its plane z+1 has been read
        take_halo(z + 1, s2);
        wait_lds();
        if (more) prefetch_halo(z + 2);
        take_own(z + 1, s2, nxt);
        wait_lds();
        if (more) prefetch_own(z + 2);
        barrier_lds();
        const R psi0 = ring[s1][ly + 1][lx + OX];
        const bool fluid_node = active && !(psi0 < R(0));
        stored = __any(fluid_node);
        if (fluid_node) {
            R pn[Q];
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                const int ez = vel_z(j);
                const int sl = ez < 0 ? s0 : (ez > 0 ? s2 : s1);
                pn[j] = ring[sl][ly + 1 + vel_y(j)][col(vel_x(j))];
            }
            const NodeForce<R> nf = node_force<Q, R, GEOM != GEOM_NONE>(psi0, pn, P);
            collide<Q, R>(cur, nf, P);
            const unsigned nb = (unsigned)(oxy[4] + z * nxy) * (unsigned)sizeof(T);
            if constexpr (NTS) {
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    st_off_nt(fout, nb + (unsigned)i * pst, static_cast<T>(cur[i]));
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) st_off(fout, nb + (unsigned)i * pst, static_cast<T>(cur[i]));
            }
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) cur[i] = nxt[i];
    }
}

// One prefetching tile of the fused step (tile index t, z-chunks of zc planes), its chunk
// split into geometry forms by fused_segments.
template <int Q, typename T, int GEOM, int TX, int TY, bool FULLX, bool NTS>
__device__ __forceinline__ void fused_tile_pf(const T* __restrict__ fin, T* __restrict__ fout,
                                              const uint32_t* __restrict__ links, const Grid& g,
                                              const Phys<float>& P, int t, int ntx, int nty,
                                              int zc, int hints) {
    const int z0 = t / (ntx * nty) * zc, z1 = min(z0 + zc, g.nz);
    fused_segments<T, GEOM>(g, z0, z1, [&](auto form, int a, int b) {
        fused_tile_pf_seg<Q, T, decltype(form)::value, TX, TY, FULLX, NTS>(fin, fout, links, g, P, t,
                                                                          ntx, nty, a, b, hints);
    });
}

// FP64 full-row tile with the own populations of plane z+2 prefetched into LDS (each double
// as two dword DMAs into a low and a high slot array). The halo rows are pulled
// synchronously, before the prefetch is issued: vector memory completes in order, so waiting
// for the halo loads after the prefetch would also wait for the prefetch. The own buffer
// (77.8 KB at 256x2, D3Q19) and the psi ring (32 KB) fit in LDS; a halo buffer would not.
// Arithmetic per node as in fused_tile (bitwise identical results).
template <int Q, int GEOM, int TX, int TY, bool NTS>
__device__ __forceinline__ void fused_tile_pf64(const double* __restrict__ fin,
                                                double* __restrict__ fout,
                                                const uint32_t* __restrict__ links, const Grid& g,
                                                const Phys<double>& P, int t, int nty, int zc,
                                                int hints) {
    using R = double;
    using T = double;
    constexpr int NT = TX * TY, H = 2 * TX;
    static_assert(H <= NT && TX % 64 == 0, "full rows must be whole wavefronts");
    static_assert(fused_pf64_lds_bytes(Q, TX, TY) <= kLdsBytesPerCU, "tile does not fit in LDS");
    __shared__ R ring[4][TY + 2][TX];
    __shared__ uint32_t pf_lo[Q][NT];
    __shared__ uint32_t pf_hi[Q][NT];
    const uint32_t lo_lds = lds_addr(&pf_lo[0][(threadIdx.x >> 6) * 64]);
    const uint32_t hi_lds = lds_addr(&pf_hi[0][(threadIdx.x >> 6) * 64]);

    const int iy = t % nty;
    const int iz = t / nty;
    const int y0 = iy * TY, z0 = iz * zc;
    const int z1 = min(z0 + zc, g.nz);
    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int x = lx, y = y0 + ly;
    const bool active = y < g.ny;
    auto wrapc = [](int c, int n) { c %= n; return c < 0 ? c + n : c; };
    const int nxy = g.nx * g.ny;
    const unsigned pst = (unsigned)g.stride * (unsigned)sizeof(T);
    const bool has_halo = tid < H;
    const int hx = tid % TX, hy = tid < TX ? -1 : TY;
    int oxy[9], hxy[9];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            oxy[(dy + 1) * 3 + dx + 1] = wrapc(x + dx, g.nx) + wrapc(y + dy, g.ny) * g.nx;
            hxy[(dy + 1) * 3 + dx + 1] = wrapc(hx + dx, g.nx) + wrapc(y0 + hy + dy, g.ny) * g.nx;
        }
    auto zoffs = [&](int zp, int* zo) {
        zo[0] = wrapc(zp - 1, g.nz) * nxy;
        zo[1] = wrapc(zp, g.nz) * nxy;
        zo[2] = wrapc(zp + 1, g.nz) * nxy;
    };
    WallBits wo{0u, 0u, 0u}, wh{0u, 0u, 0u};
    if (GEOM == GEOM_WALLS) {
        wo.wx = wall_bits(x, g.nx, g.walls, 0);
        wo.wy = wall_bits(wrapc(y, g.ny), g.ny, g.walls, 1);
        wh.wx = wall_bits(hx, g.nx, g.walls, 0);
        wh.wy = wall_bits(wrapc(y0 + hy, g.ny), g.ny, g.walls, 1);
    }
    auto zbits = [&](int zp) {
        return GEOM == GEOM_WALLS ? wall_bits(wrapc(zp, g.nz), g.nz, g.walls, 2) : 0u;
    };
    auto psi_of = [&](R drho) { return pseudopotential<R>(P.rho_ref + drho, P); };
    auto col = [&](int dx) {
        const int c = lx + dx;
        return c < 0 ? c + TX : (c >= TX ? c - TX : c);
    };
    auto own_psi = [&](int zp, int slot, R* v) {
        int zo[3];
        zoffs(zp, zo);
        const WallBits wb{wo.wx, wo.wy, zbits(zp)};
        const bool s = node_solid<GEOM>(links, oxy[4] + zo[1], wb);
        pull_loads<Q, T, R, GEOM>(fin, links, oxy, zo, wb, pst, v);
        ring[slot][ly + 1][lx] = s ? R(-1) : psi_of(sum_q<Q, R>(v));
    };
    auto halo_psi = [&](int zp, int slot) {
        if (!has_halo) return;
        int zo[3];
        zoffs(zp, zo);
        const WallBits wb{wh.wx, wh.wy, zbits(zp)};
        R hv;
        if (node_solid<GEOM>(links, hxy[4] + zo[1], wb)) hv = R(-1);
        else {
            R v[Q];
            pull_loads<Q, T, R, GEOM>(fin, links, hxy, zo, wb, pst, v);
            hv = psi_of(sum_q<Q, R>(v));
        }
        ring[slot][hy + 1][hx] = hv;
    };
    auto prefetch_own = [&](int zp) {
        int zo[3];
        zoffs(zp, zo);
        const WallBits wb{wo.wx, wo.wy, zbits(zp)};
        const unsigned lk = link_word<GEOM>(links, oxy[4] + zo[1]);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int e, pop;
            pull_source<Q, GEOM>(i, oxy, zo, lk, wb, e, pop);
            const char* src = reinterpret_cast<const char*>(fin) + ((unsigned)e * 8u + (unsigned)pop * pst);
            lds_dma<4, 0>(src, lo_lds + (uint32_t)(i * NT * 4));
            lds_dma<4, 0>(src + 4, hi_lds + (uint32_t)(i * NT * 4));
        }
    };
    auto take_own = [&](int zp, int slot, R* v) {
        int zo[3];
        zoffs(zp, zo);
        const WallBits wb{wo.wx, wo.wy, zbits(zp)};
#pragma unroll
        for (int i = 0; i < Q; ++i)
            v[i] = __builtin_bit_cast(double, ((unsigned long long)pf_hi[i][tid] << 32) | pf_lo[i][tid]);
        ring[slot][ly + 1][lx] =
            node_solid<GEOM>(links, oxy[4] + zo[1], wb) ? R(-1) : psi_of(sum_q<Q, R>(v));
    };

    R cur[Q], nxt[Q];
    own_psi(z0 - 1, 0, nxt);
    halo_psi(z0 - 1, 0);
    own_psi(z0, 1, cur);
    halo_psi(z0, 1);
    prefetch_own(z0 + 1);
    for (int z = z0; z < z1; ++z) {
        const int k = z - z0;
        const int s0 = k & 3, s1 = (k + 1) & 3, s2 = (k + 2) & 3;
        wait_vector_memory();
        take_own(z + 1, s2, nxt);
        halo_psi(z + 1, s2);
        wait_lds();
        if (z + 1 < z1) prefetch_own(z + 2);
        barrier_lds();
        const R psi0 = ring[s1][ly + 1][lx];
        if (active && !(psi0 < R(0))) {
            R pn[Q];
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                const int ez = vel_z(j);
                const int sl = ez < 0 ? s0 : (ez > 0 ? s2 : s1);
                pn[j] = ring[sl][ly + 1 + vel_y(j)][col(vel_x(j))];
            }
            const NodeForce<R> nf = node_force<Q, R, GEOM != GEOM_NONE>(psi0, pn, P);
            collide<Q, R>(cur, nf, P);
            const unsigned nb = (unsigned)(oxy[4] + z * nxy) * (unsigned)sizeof(T);
            if constexpr (NTS) {
#pragma unroll
                for (int i = 0; i < Q; ++i) st_off_nt(fout, nb + (unsigned)i * pst, cur[i]);
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) st_off(fout, nb + (unsigned)i * pst, cur[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) cur[i] = nxt[i];
    }
}

template <int Q, int GEOM, int TX, int TY, bool NTS>
__global__ __launch_bounds__(TX * TY) void k_step_fused_pf64(const double* __restrict__ fin,
                                                            double* __restrict__ fout,
                                                            const uint32_t* __restrict__ links,
                                                            Grid g, Phys<double> P, int zc,
                                                            int remap, int hints) {
    const int t = remap ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    fused_tile_pf64<Q, GEOM, TX, TY, NTS>(fin, fout, links, g, P, t, (g.ny + TY - 1) / TY, zc, hints);
}

template <int Q, typename T, int GEOM, int TX, int TY, bool NTS>
__global__ __launch_bounds__(TX * TY) void k_step_fused_pf(const T* __restrict__ fin,
                                                          T* __restrict__ fout,
                                                          const uint32_t* __restrict__ links,
                                                          Grid g, Phys<float> P, int zc,
                                                          int remap, int hints) {
    const int t = remap ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    fused_tile_pf<Q, T, GEOM, TX, TY, true, NTS>(fin, fout, links, g, P, t, 1,
                                                 (g.ny + TY - 1) / TY, zc, hints);
}

// Single domain. remap != 0: map workgroups to tiles so that each XCD gets a contiguous
// tile range (workgroup b runs on XCD b mod 8).
template <int Q, typename T, int GEOM, int TX, int TY, bool FULLX, bool NTS, bool WIDE = false>
__global__ __launch_bounds__(TX * TY) void k_step_fused(const T* __restrict__ fin,
                                                       T* __restrict__ fout,
                                                       const uint32_t* __restrict__ links,
                                                       Grid g, Phys<typename Arith<T>::type> P,
                                                       int ntx, int nty, int zc, int remap,
                                                       int hints) {
    const int t = remap ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    fused_tile<Q, T, GEOM, TX, TY, FULLX, NTS, WIDE>(fin, fout, links, g, P, t, ntx, nty, zc, hints);
}

// One domain of a batched step: its buffers, geometry, physics and the first workgroup
// of the batched grid that works on it.
template <typename T>
struct DomainDesc {
    const T* fin;
    T* fout;
    const uint32_t* links;     // link words (solid mask only)
    Grid g;
    Phys<typename Arith<T>::type> P;
    int ntx, nty, zc, block0;
    int rows;                  // rows per tile of the row-tile kernel (k_step_fused_batch_rows)
};

// Many independent lattices advanced by one launch: workgroup b (after the XCD-contiguous
// remap when remap != 0) belongs to the last domain whose block0 <= b (binary search over
// the table, uniform per workgroup).
template <int Q, typename T, int GEOM, int TX, int TY, bool NTS>
__global__ __launch_bounds__(TX * TY) void k_step_fused_batch(const DomainDesc<T>* __restrict__ d,
                                                             int ndom, int remap) {
    const int b = remap ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    int lo = 0, hi = ndom - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].block0 <= b) lo = mid; else hi = mid - 1;
    }
    const DomainDesc<T>& D = d[lo];
    fused_tile<Q, T, GEOM, TX, TY, false, NTS>(D.fin, D.fout, D.links, D.g, D.P, b - D.block0,
                                               D.ntx, D.nty, D.zc, 0);
}

// Batched step with prefetching tiles (4-byte storage): as k_step_fused_batch.
template <int Q, typename T, int GEOM, int TX, int TY, bool NTS>
__global__ __launch_bounds__(TX * TY) void k_step_fused_batch_pf(const DomainDesc<T>* __restrict__ d,
                                                                int ndom, int remap) {
    const int b = remap ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    int lo = 0, hi = ndom - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].block0 <= b) lo = mid; else hi = mid - 1;
    }
    const DomainDesc<T>& D = d[lo];
    fused_tile_pf<Q, T, GEOM, TX, TY, false, NTS>(D.fin, D.fout, D.links, D.g, D.P, b - D.block0,
                                                  D.ntx, D.nty, D.zc, 0);
}


// Full-row tiles of run-time width, for a batch of lattices of different widths (4- and
// 2-byte storage). A workgroup of NT threads covers `rows` consecutive rows of a lattice of
// width L = g.nx <= NT / 2 (rows = NT / L, or ny if smaller): lane tid owns node (tid mod L,
// y0 + tid / L) for tid < rows L, each row wrapping inside itself in x as in the full-row
// tiles, so that no x-halo is pulled; lanes beyond rows L own no node. The halo is the rows
// y0 - 1 and y0 + rows (2 L <= NT nodes, one per thread). Own and halo populations of the
// next plane are prefetched into LDS as in fused_tile_pf (without the nontemporal hint for
// interior rows, whose lanes need not fill whole wavefronts here). The psi ring is flat:
// (rows + 2) L <= NT + 2 L <= 2 NT cells per plane. Arithmetic per node as in fused_tile.
template <int Q, typename T, int GEOM, int NT, bool NTS>
__device__ __forceinline__ void fused_tile_rows_seg(const T* __restrict__ fin, T* __restrict__ fout,
                                                    const uint32_t* __restrict__ links, const Grid& g,
                                                    const Phys<float>& P, int t, int rows, int nty,
                                                    int z0, int z1) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 2, "the LDS prefetch moves 2- or 4-byte elements");
    static_assert(NT % 64 == 0, "whole wavefronts");
    using R = float;
    using S = typename PfSlot<T>::type;
    auto& lds = pf_lds<S, Q, 1, 2 * NT, NT, NT>();
    auto& ring_rows = lds.ring;
    auto& pf_own = lds.own;
    auto& pf_halo = lds.halo;
    const uint32_t own_lds = lds_addr(&pf_own[0][(threadIdx.x >> 6) * 64]);
    const uint32_t halo_lds = lds_addr(&pf_halo[0][(threadIdx.x >> 6) * 64]);

    const int L = g.nx;
    const int iy = t % nty;
    const int y0 = iy * rows;
    const int tid = threadIdx.x;
    // lanes without a node take node 0's column and row (valid addresses; never stored, and
    // they write no ring cell)
    const bool own_lane = tid < rows * L;
    const int lx = own_lane ? tid % L : 0, ly = own_lane ? tid / L : 0;
    const int x = lx, y = y0 + ly;
    const bool active = own_lane && y < g.ny;
    auto wrapc = [](int c, int n) { c %= n; return c < 0 ? c + n : c; };
    const int nxy = g.nx * g.ny;
    const unsigned pst = (unsigned)g.stride * (unsigned)sizeof(T);
    const bool has_halo = tid < 2 * L;
    const int hx = has_halo ? tid % L : 0, hy = tid < L ? -1 : rows;
    int oxy[9], hxy[9];
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
        for (int dx = -1; dx <= 1; ++dx) {
            oxy[(dy + 1) * 3 + dx + 1] = wrapc(x + dx, L) + wrapc(y + dy, g.ny) * L;
            hxy[(dy + 1) * 3 + dx + 1] = wrapc(hx + dx, L) + wrapc(y0 + hy + dy, g.ny) * L;
        }
    auto zoffs = [&](int zp, int* zo) {
        zo[0] = wrapc(zp - 1, g.nz) * nxy;
        zo[1] = wrapc(zp, g.nz) * nxy;
        zo[2] = wrapc(zp + 1, g.nz) * nxy;
    };
    WallBits wo{0u, 0u, 0u}, wh{0u, 0u, 0u};
    if (GEOM == GEOM_WALLS) {
        wo.wx = wall_bits(x, L, g.walls, 0);
        wo.wy = wall_bits(wrapc(y, g.ny), g.ny, g.walls, 1);
        wh.wx = wall_bits(hx, L, g.walls, 0);
        wh.wy = wall_bits(wrapc(y0 + hy, g.ny), g.ny, g.walls, 1);
    }
    auto zbits = [&](int zp) {
        return GEOM == GEOM_WALLS ? wall_bits(wrapc(zp, g.nz), g.nz, g.walls, 2) : 0u;
    };
    auto psi_of = [&](R drho) { return pseudopotential<R>(P.rho_ref + drho, P); };
    // ring cell of tile row r (0: halo row y0 - 1) and column c
    auto cell = [&](int r, int c) { return r * L + c; };
    auto col = [&](int dx) {
        const int c = lx + dx;
        return c < 0 ? c + L : (c >= L ? c - L : c);
    };
    // synchronous pulls (first two planes of the chunk)
    auto own_psi = [&](int zp, int slot, R* v) {
        int zo[3];
        zoffs(zp, zo);
        const WallBits wb{wo.wx, wo.wy, zbits(zp)};
        const bool sld = node_solid<GEOM>(links, oxy[4] + zo[1], wb);
        pull_loads<Q, T, R, GEOM>(fin, links, oxy, zo, wb, pst, v);
        if (own_lane) ring_rows[slot][0][cell(ly + 1, lx)] = sld ? R(-1) : psi_of(sum_q<Q, R>(v));
    };
    auto halo_psi = [&](int zp, int slot) {
        if (!has_halo) return;
        int zo[3];
        zoffs(zp, zo);
        const WallBits wb{wh.wx, wh.wy, zbits(zp)};
        R hv;
        if (node_solid<GEOM>(links, hxy[4] + zo[1], wb)) hv = R(-1);
        else {
            R v[Q];
            pull_loads<Q, T, R, GEOM>(fin, links, hxy, zo, wb, pst, v);
            hv = psi_of(sum_q<Q, R>(v));
        }
        ring_rows[slot][0][cell(hy + 1, hx)] = hv;
    };
    // asynchronous pulls of plane zp into the LDS buffers (lanes with a node / a halo node)
    auto prefetch_own = [&](int zp) {
        if (!own_lane) return;
        int zo[3];
        zoffs(zp, zo);
        const WallBits wb{wo.wx, wo.wy, zbits(zp)};
        const unsigned lk = link_word<GEOM>(links, oxy[4] + zo[1]);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int e, pop;
            pull_source<Q, GEOM>(i, oxy, zo, lk, wb, e, pop);
            lds_dma<(int)sizeof(T), 0>(
                reinterpret_cast<const char*>(fin) + ((unsigned)e * (unsigned)sizeof(T) + (unsigned)pop * pst),
                own_lds + (uint32_t)(i * NT * sizeof(S)));
        }
    };
    auto prefetch_halo = [&](int zp) {
        if (!has_halo) return;
        int zo[3];
        zoffs(zp, zo);
        const WallBits hb{wh.wx, wh.wy, zbits(zp)};
        const unsigned lk = link_word<GEOM>(links, hxy[4] + zo[1]);
#pragma unroll
        for (int i = 0; i < Q; ++i) {
            int e, pop;
            pull_source<Q, GEOM>(i, hxy, zo, lk, hb, e, pop);
            lds_dma<(int)sizeof(T), 0>(
                reinterpret_cast<const char*>(fin) + ((unsigned)e * (unsigned)sizeof(T) + (unsigned)pop * pst),
                halo_lds + (uint32_t)(i * NT * sizeof(S)));
        }
    };
    auto take_halo = [&](int zp, int slot) {
        if (!has_halo) return;
        int zo[3];
        zoffs(zp, zo);
        const WallBits hb{wh.wx, wh.wy, zbits(zp)};
        R hv;
        if (node_solid<GEOM>(links, hxy[4] + zo[1], hb)) hv = R(-1);
        else {
            R sum = 0;
#pragma unroll
            for (int i = 0; i < Q; ++i) sum += pf_value<T, R>(pf_halo[i][tid]);
            hv = psi_of(sum);
        }
        ring_rows[slot][0][cell(hy + 1, hx)] = hv;
    };
    auto take_own = [&](int zp, int slot, R* v) {
        if (!own_lane) return;
        int zo[3];
        zoffs(zp, zo);
        const WallBits wb{wo.wx, wo.wy, zbits(zp)};
#pragma unroll
        for (int i = 0; i < Q; ++i) v[i] = pf_value<T, R>(pf_own[i][tid]);
        ring_rows[slot][0][cell(ly + 1, lx)] =
            node_solid<GEOM>(links, oxy[4] + zo[1], wb) ? R(-1) : psi_of(sum_q<Q, R>(v));
    };

    R cur[Q], nxt[Q];
    own_psi(z0 - 1, 0, nxt);
    halo_psi(z0 - 1, 0);
    own_psi(z0, 1, cur);
    halo_psi(z0, 1);
    prefetch_halo(z0 + 1);
    prefetch_own(z0 + 1);
    // as in fused_tile_pf: after the Q stores of the previous plane, the wait for the
    // prefetched plane leaves those stores in flight
    bool stored = false;
    for (int z = z0; z < z1; ++z) {
        const int k = z - z0;
        const int s0 = k & 3, s1 = (k + 1) & 3, s2 = (k + 2) & 3;
        const bool more = z + 1 < z1;
        if (stored) wait_vector_memory_but<Q>();
        else wait_vector_memory();
        take_halo(z + 1, s2);
        wait_lds();
        if (more) prefetch_halo(z + 2);
        take_own(z + 1, s2, nxt);
        wait_lds();
        if (more) prefetch_own(z + 2);
        barrier_lds();
        const R psi0 = ring_rows[s1][0][cell(ly + 1, lx)];
        const bool fluid_node = active && !(psi0 < R(0));
        stored = __any(fluid_node);
        if (fluid_node) {
            R pn[Q];
#pragma unroll
            for (int j = 0; j < Q; ++j) {
                const int ez = vel_z(j);
                const int sl = ez < 0 ? s0 : (ez > 0 ? s2 : s1);
                pn[j] = ring_rows[sl][0][cell(ly + 1 + vel_y(j), col(vel_x(j)))];
            }
            const NodeForce<R> nf = node_force<Q, R, GEOM != GEOM_NONE>(psi0, pn, P);
            collide<Q, R>(cur, nf, P);
            const unsigned nb = (unsigned)(oxy[4] + z * nxy) * (unsigned)sizeof(T);
            if constexpr (NTS) {
#pragma unroll
                for (int i = 0; i < Q; ++i)
                    st_off_nt(fout, nb + (unsigned)i * pst, static_cast<T>(cur[i]));
            } else {
#pragma unroll
                for (int i = 0; i < Q; ++i) st_off(fout, nb + (unsigned)i * pst, static_cast<T>(cur[i]));
            }
        }
#pragma unroll
        for (int i = 0; i < Q; ++i) cur[i] = nxt[i];
    }
}

// One row tile of the batched step (tile index t, z-chunks of zc planes), its chunk split
// into geometry forms by fused_segments.
template <int Q, typename T, int GEOM, int NT, bool NTS>
__device__ __forceinline__ void fused_tile_rows(const T* __restrict__ fin, T* __restrict__ fout,
                                                const uint32_t* __restrict__ links, const Grid& g,
                                                const Phys<float>& P, int t, int rows, int nty,
                                                int zc) {
    const int z0 = t / nty * zc, z1 = min(z0 + zc, g.nz);
    fused_segments<T, GEOM>(g, z0, z1, [&](auto form, int a, int b) {
        fused_tile_rows_seg<Q, T, decltype(form)::value, NT, NTS>(fin, fout, links, g, P, t, rows,
                                                                 nty, a, b);
    });
}

// Batched step with row tiles of run-time width (fused_tile_rows): as k_step_fused_batch.
template <int Q, typename T, int GEOM, int NT, bool NTS>
__global__ __launch_bounds__(NT) void k_step_fused_batch_rows(const DomainDesc<T>* __restrict__ d,
                                                             int ndom, int remap) {
    const int b = remap ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    int lo = 0, hi = ndom - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d[mid].block0 <= b) lo = mid; else hi = mid - 1;
    }
    const DomainDesc<T>& D = d[lo];
    fused_tile_rows<Q, T, GEOM, NT, NTS>(D.fin, D.fout, D.links, D.g, D.P, b - D.block0, D.rows,
                                         D.nty, D.zc);
}

}  // namespace lbmk
