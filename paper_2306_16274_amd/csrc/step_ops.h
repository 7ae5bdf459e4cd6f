// Step kernels of one (lattice, storage type) pair behind StepOps<Q, T> (ctx.h): the
// fused step in every launch configuration of fused.h, and the two passes of the two-pass
// step (kernels.h). Included only by the step_q*_*.hip units, one instantiation each.
#pragma once

#include "ctx.h"
#include "kernels.h"

template <int Q, typename T>
static void launch_psi(lbm_ctx* c, const void* fin) {
    using R = typename Arith<T>::type;
    const Launch L = node_launch(c);
    const Phys<R>& P = phys_of<R>(c);
    if (c->any_solid)
        hipLaunchKernelGGL((k_density_psi<Q, T, true>), L.grid, L.block, 0, c->stream,
                           (const T*)fin, c->solid, (R*)c->psi, grid_of(c), P);
    else
        hipLaunchKernelGGL((k_density_psi<Q, T, false>), L.grid, L.block, 0, c->stream,
                           (const T*)fin, c->solid, (R*)c->psi, grid_of(c), P);
}

template <int Q, typename T>
static void launch_collide(lbm_ctx* c, const void* fin, void* fout) {
    using R = typename Arith<T>::type;
    const Launch L = node_launch(c);
    const Phys<R>& P = phys_of<R>(c);
    hipLaunchKernelGGL((k_collide<Q, T>), L.grid, L.block, 0, c->stream, (const T*)fin, (T*)fout,
                       (const R*)c->psi, grid_of(c), P);
}


template <typename F>
static void with_geom_nts(const lbm_ctx* c, int hints, F&& f) {
    using std::integral_constant;
    const bool nt = (hints & kHintNtStore) != 0;
    switch (geom_of(c)) {
    case GEOM_NONE:
        if (nt) f(integral_constant<int, GEOM_NONE>{}, integral_constant<bool, true>{});
        else f(integral_constant<int, GEOM_NONE>{}, integral_constant<bool, false>{});
        break;
    case GEOM_WALLS:
        if (nt) f(integral_constant<int, GEOM_WALLS>{}, integral_constant<bool, true>{});
        else f(integral_constant<int, GEOM_WALLS>{}, integral_constant<bool, false>{});
        break;
    default:
        if (nt) f(integral_constant<int, GEOM_MASK>{}, integral_constant<bool, true>{});
        else f(integral_constant<int, GEOM_MASK>{}, integral_constant<bool, false>{});
    }
}

template <int Q, typename T, int TX, int TY, bool FULLX, bool WIDE = false>
static void launch_fused_cfg(lbm_ctx* c, const void* fin, void* fout) {
    using R = typename Arith<T>::type;
    const Phys<R>& P = phys_of<R>(c);
    const int ntx = (c->p.nx + TX - 1) / TX, nty = (c->p.ny + TY - 1) / TY;
    const long long tiles = (long long)ntx * nty;
    int zc, remap, hints;
    fused_chunking(c, zc, remap, hints);
    const int nchunks = (c->p.nz + zc - 1) / zc;
    const dim3 grid((unsigned)(tiles * nchunks)), block(TX * TY);
    // 64-bit offsets are instantiated with plain stores only
    with_geom_nts(c, WIDE ? (hints & ~kHintNtStore) : hints, [&](auto geom, auto nts) {
        if constexpr (!WIDE || !decltype(nts)::value)
            hipLaunchKernelGGL((k_step_fused<Q, T, decltype(geom)::value, TX, TY, FULLX,
                                             decltype(nts)::value, WIDE>),
                               grid, block, 0, c->stream, (const T*)fin, (T*)fout, c->links,
                               grid_of(c), P, ntx, nty, zc, remap, hints);
    });
}

// Full-row tiles with the LDS prefetch: k_step_fused_pf for 2- and 4-byte storage,
// k_step_fused_pf64 (own populations only) for FP64, where the tile buffers fit in LDS; other
// combinations run the plain full-row tiles.
template <int Q, typename T, int TX, int TY>
static void launch_fused_pf(lbm_ctx* c, const void* fin, void* fout) {
    if constexpr (std::is_same<T, double>::value && fused_pf64_lds_bytes(Q, TX, TY) <= kLdsBytesPerCU) {
        const int nty = (c->p.ny + TY - 1) / TY;
        int zc, remap, hints;
        fused_chunking(c, zc, remap, hints);
        const int nchunks = (c->p.nz + zc - 1) / zc;
        const dim3 grid((unsigned)(nty * nchunks)), block(TX * TY);
        const double* f0 = (const double*)fin;
        double* f1 = (double*)fout;
        with_geom_nts(c, hints, [&](auto geom, auto nts) {
            hipLaunchKernelGGL((k_step_fused_pf64<Q, decltype(geom)::value, TX, TY,
                                                  decltype(nts)::value>),
                               grid, block, 0, c->stream, f0, f1, c->links, grid_of(c), c->pd, zc,
                               remap, hints);
        });
    } else if constexpr ((sizeof(T) == 4 || sizeof(T) == 2) && fused_pf_lds_bytes(Q, TX, TY) <= kLdsBytesPerCU) {
        const int nty = (c->p.ny + TY - 1) / TY;
        int zc, remap, hints;
        fused_chunking(c, zc, remap, hints);
        const int nchunks = (c->p.nz + zc - 1) / zc;
        const dim3 grid((unsigned)(nty * nchunks)), block(TX * TY);
        with_geom_nts(c, hints, [&](auto geom, auto nts) {
            hipLaunchKernelGGL((k_step_fused_pf<Q, T, decltype(geom)::value, TX, TY,
                                                decltype(nts)::value>),
                               grid, block, 0, c->stream, (const T*)fin, (T*)fout, c->links,
                               grid_of(c), c->pf, zc, remap, hints);
        });
    } else {
        launch_fused_cfg<Q, T, TX, TY, true>(c, fin, fout);
    }
}

// 320- and 384-wide full rows (2-row tiles) for 2- and 4-byte storage only: FP64 needs more
// VGPRs than 640 or 768 threads leave a lane (12.3 vs 9.4 GLUPS, 32x8 vs 384x2 at 384^2 x 160),
// so FP64 is not instantiated here and never selected (default_fused_cfg).
template <int Q, typename T>
static void launch_fused_wide(lbm_ctx* c, const void* fin, void* fout) {
    if constexpr (sizeof(T) != 8) {
        switch (c->fused_cfg) {
        case 5: launch_fused_cfg<Q, T, 320, 2, true>(c, fin, fout); break;
        case 6: launch_fused_pf<Q, T, 320, 2>(c, fin, fout); break;
        case 7: launch_fused_cfg<Q, T, 384, 2, true>(c, fin, fout); break;
        default: launch_fused_pf<Q, T, 384, 2>(c, fin, fout); break;
        }
    }
}

template <int Q, typename T>
static void launch_fused(lbm_ctx* c, const void* fin, void* fout) {
    if (c->addr64) {                       // population buffer of 4 GiB or more
        if (c->fused_cfg == 9) launch_fused_cfg<Q, T, 64, 4, false, true>(c, fin, fout);
        else launch_fused_cfg<Q, T, 64, 8, false, true>(c, fin, fout);
        return;
    }
    switch (c->fused_cfg) {
    case 1: launch_fused_cfg<Q, T, 256, 2, true>(c, fin, fout); break;
    case 2: launch_fused_cfg<Q, T, 256, 4, true>(c, fin, fout); break;
    case 3: launch_fused_pf<Q, T, 256, 4>(c, fin, fout); break;
    case 4: launch_fused_pf<Q, T, 256, 2>(c, fin, fout); break;
    case 5: case 6: case 7: case 8: launch_fused_wide<Q, T>(c, fin, fout); break;
    case 9: launch_fused_cfg<Q, T, 64, 4, false>(c, fin, fout); break;
    case 10: launch_fused_cfg<Q, T, 64, 8, false>(c, fin, fout); break;
    default: launch_fused_cfg<Q, T, 32, 8, false>(c, fin, fout); break;
    }
}

template <int Q, typename T>
void StepOps<Q, T>::fused(lbm_ctx* c, const void* fin, void* fout) { launch_fused<Q, T>(c, fin, fout); }
template <int Q, typename T>
void StepOps<Q, T>::psi(lbm_ctx* c, const void* fin) { launch_psi<Q, T>(c, fin); }
template <int Q, typename T>
void StepOps<Q, T>::collide(lbm_ctx* c, const void* fin, void* fout) { launch_collide<Q, T>(c, fin, fout); }
