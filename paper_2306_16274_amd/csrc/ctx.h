// Host-side state of one lattice (lbm_ctx) and the helpers shared by the translation units
// of the library: api.hip (the C ABI), batch.hip (batched stepping) and the step_*.hip
// units, each of which instantiates the step kernels of one (lattice, storage type) pair
// (StepOps, defined in step_ops.h) so that the units compile in parallel.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <type_traits>

#include "../../include/lbm.h"
#include "fused.h"

using namespace lbmk;

struct lbm_ctx {
    lbm_params p{};
    int device = 0;
    int Q = 19;
    long long N = 0, stride = 0;
    size_t elem = 4;               // bytes per stored population
    void* f[2] = {nullptr, nullptr};
    int cur = 0;
    void* psi = nullptr;           // float64 (FP64 storage) or float32
    uint8_t* solid = nullptr;
    uint32_t* links = nullptr;     // link words of the fused step (cylinder geometries)
    bool any_solid = false;
    double* mom = nullptr;         // rho, u (3), p: 5 N doubles, allocated on first use
    double* partial = nullptr;     // per-block partial sums (moments and health check)
    long long partial_cap = 0;
    double* dtot = nullptr;        // 8 device doubles: totals (5), health result (2)
    double* hhealth = nullptr;     // pinned: [min rho, non-finite flag]
    hipEvent_t health_ev = nullptr;
    bool health_pending = false;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    bool initialised = false;
    bool failed = false;
    int64_t steps = 0;
    Phys<double> pd{};
    Phys<float> pf{};
    int fused_cfg = 0;             // index into kFusedCfgs
    int cus = 256;                 // compute units of the device
    bool addr64 = false;           // population buffer of 4 GiB or more: 64-bit offsets
    std::string err;
};

// Message of the last failed lbm_create of the calling thread (defined in api.hip).
extern thread_local std::string g_create_error;

inline lbm_status fail(lbm_ctx* c, lbm_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf; else g_create_error = buf;
    return s;
}

#define HIPCHK(c, call)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail((c), e_ == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE,       \
                        "%s failed: %s", #call, hipGetErrorString(e_));                  \
    } while (0)

inline long long plane_stride(long long N) { return (N + 63) / 64 * 64; }

inline size_t storage_bytes(int storage) {
    return storage == LBM_FP64 ? 8 : storage == LBM_FP32 ? 4 : 2;
}

// Device buffers of a context are allocated and freed in stream order on the context's
// stream (hipMallocAsync / hipFreeAsync), so creating or destroying one lattice never
// waits for the work of other lattices.
inline hipError_t dmalloc(hipStream_t s, void** p, size_t bytes) { return hipMallocAsync(p, bytes, s); }
inline void dfree(hipStream_t s, void* p) { if (p) (void)hipFreeAsync(p, s); }

// Physical constants of the context in the arithmetic type R of its storage.
template <typename R>
inline const Phys<R>& phys_of(const lbm_ctx* c) {
    if constexpr (std::is_same<R, double>::value) return c->pd;
    else return c->pf;
}

// Launch shape of the per-node kernels (diagnostics, initialisation, two-pass step).
struct Launch { dim3 grid, block; };
inline Launch node_launch(const lbm_ctx* c) {
    Launch L;
    const int bx = c->p.nx >= 64 ? 64 : (c->p.nx >= 32 ? 32 : 16);
    const int by = 256 / bx;
    L.block = dim3(bx, by, 1);
    L.grid = dim3((c->p.nx + bx - 1) / bx, (c->p.ny + by - 1) / by, c->p.nz);
    return L;
}
inline long long nblocks(const Launch& L) { return (long long)L.grid.x * L.grid.y * L.grid.z; }

inline Grid grid_of(const lbm_ctx* c) {
    Grid g;
    g.nx = c->p.nx; g.ny = c->p.ny; g.nz = c->p.nz; g.stride = c->stride;
    g.walls = 0;
    g.zlo = 0;
    for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 2; ++s)
            if (c->p.bc[a][s] == LBM_BC_WALL) g.walls |= 1 << (2 * a + s);
    return g;
}

// Solid-node source of the fused kernels: none, wall layers from coordinates, or mask.
inline int geom_of(const lbm_ctx* c) {
    if (!c->any_solid) return GEOM_NONE;
    return c->p.cylinder ? GEOM_MASK : GEOM_WALLS;
}

// Population buffers of 4 GiB or more take 64-bit byte offsets, which only the plain 64x4
// and 64x8 tiles are instantiated with (configurations 9 and 10).
inline bool needs_addr64(const lbm_params& p) {
    const long long N = (long long)p.nx * p.ny * p.nz;
    return (double)(p.lattice == 27 ? 27 : 19) * (double)plane_stride(N) *
               (double)storage_bytes(p.storage) >= 4294967296.0;
}

// Launch configuration of the fused step for a lattice of width nx, element size elem and
// lattice Q: the default of fused.h unless LBM_FUSED_CONFIG names a valid one (a full-row
// configuration needs nx equal to its width; FP64 has no 320/384-wide instantiations; with
// 64-bit offsets only configurations 9 and 10 exist).
inline int fused_cfg_for(int nx, int elem, int Q, bool addr64, bool mask = false) {
    if (const char* e = getenv("LBM_FUSED_CONFIG")) {      // tuning override
        const int v = atoi(e);
        if (v >= 0 && v < kNumFusedCfgs && (!kFusedCfgs[v].fullx || nx == kFusedCfgs[v].tx) &&
            !(elem == 8 && kFusedCfgs[v].tx > 256) && (!addr64 || v == 9 || v == 10))
            return v;
    }
    if (addr64) return elem == 4 ? 10 : 9;
    return default_fused_cfg_index(nx, elem, Q, mask);
}

// Whether a configuration's prefetching tile fits in LDS for this lattice and element size
// (the launch falls back to the plain tile of the same shape otherwise).
inline bool fused_prefetch_fits(const FusedCfg& f, int Q, int elem) {
    if (!f.pf || !f.fullx) return false;
    if (elem == 8) return fused_pf64_lds_bytes(Q, f.tx, f.ty) <= kLdsBytesPerCU;
    return fused_pf_lds_bytes(Q, f.tx, f.ty) <= kLdsBytesPerCU;
}

// Solid-free form of the fused tiles (fused.h): z-chunks whose planes z0 - 2 .. z1 + 1 hold
// no solid node run the arithmetic of a lattice without solid nodes (2- and 4-byte storage).
// LBM_SOLID_FREE=0 turns it off (tuning).
inline bool solid_free_enabled() {
    const char* e = getenv("LBM_SOLID_FREE");
    return !e || atoi(e) != 0;
}

// Z-chunk layout of the fused step: chunk 0 holds zlo planes, the others zc, the last the
// rest (zlo == zc: uniform chunks); n chunks.
struct ZChunks { int zlo, zc, n; };
inline ZChunks zchunks_of(int nz, int zlo, int zc) {
    return {zlo, zc, nz <= zlo ? 1 : 1 + (nz - zlo + zc - 1) / zc};
}

// Whether the solid nodes of a lattice are the wall planes z = 0 and/or z = nz - 1 only.
inline bool z_walls_only(const lbm_params& p) {
    if (p.cylinder) return false;
    for (int a = 0; a < 2; ++a)
        if (p.bc[a][0] == LBM_BC_WALL || p.bc[a][1] == LBM_BC_WALL) return false;
    return p.bc[2][0] == LBM_BC_WALL || p.bc[2][1] == LBM_BC_WALL;
}

// Cost of a plane in the general form of a tile relative to the solid-free form, measured on
// lattices between z walls against periodic ones (ms per step): 256x4 prefetching tiles at
// 256^3 FP32 0.74 vs 0.475, FP16 0.62 vs 0.29; 384x2 prefetching tiles at 384^2 x 192 FP32
// 1.02 vs 0.94, FP16 0.95 vs 0.64. 1 where not measured (uniform chunks).
inline double walled_plane_cost(int cfg, int elem) {
    if (cfg == 3) return elem == 2 ? 2.0 : 1.5;
    if (cfg == 8) return elem == 2 ? 1.5 : 1.0;
    return 1.0;
}

// Layout of a single lattice's fused step from its uniform chunk depth zc. With walls along z
// only (2- and 4-byte storage) the walled end chunks, which run the general form, are made
// shorter and the interior ones, which run the solid-free form, longer, with the chunk count
// unchanged, so that the workgroups of the walled and of the interior chunks (on different
// XCDs: tiles are mapped to XCDs in contiguous ranges) have about the same work.
inline ZChunks fused_zchunks(const lbm_params& p, int elem, int cfg, int zc) {
    const ZChunks u = zchunks_of(p.nz, zc, zc);
    if (!solid_free_enabled() || elem == 8 || !z_walls_only(p)) return u;
    const bool lo = p.bc[2][0] == LBM_BC_WALL, hi = p.bc[2][1] == LBM_BC_WALL;
    const int nb = (lo ? 1 : 0) + (hi ? 1 : 0), n = u.n, nz = p.nz;
    const double w = walled_plane_cost(cfg, elem);
    if (n - nb < 1 || w <= 1.0) return u;
    const int i = (int)std::lround(nz / (nb / w + (n - nb)));
    const int b = nz - (n - nb) * i;                       // planes of the walled chunks
    const int blo = nb == 2 ? (b + 1) / 2 : b, bhi = nb == 2 ? b / 2 : b;
    // a walled chunk must hold the wall plane and the two planes next to it, and fit in one
    if (i < 1 || (lo && (blo < 3 || blo > i)) || (hi && (bhi < 3 || bhi > i))) return u;
    const ZChunks z = zchunks_of(nz, lo ? blo : i, i);
    return z.n == n ? z : u;
}

// Layout of a lattice in a batched step (many workgroups per CU, so no balancing): with a
// wall at z = 0 the first chunk holds only the 4 planes next to it.
inline ZChunks batch_zchunks(const lbm_params& p, int zc) {
    if (!solid_free_enabled() || p.storage == LBM_FP64 || !z_walls_only(p) ||
        p.bc[2][0] != LBM_BC_WALL || p.nz < 4 + zc)
        return zchunks_of(p.nz, zc, zc);
    return zchunks_of(p.nz, 4, zc);
}

// Chunks (bit iz, chunks 0..63) of layout zk whose planes z0 - 2 .. z1 + 1 (periodic) hold no
// solid node. Walls along x or y put solid nodes in every plane; a wall along z is the plane 0
// or nz - 1; a cylinder along x fills the planes cyl_z - cyl_r .. cyl_z + cyl_r (taken one
// plane wider either side).
inline uint64_t solid_free_chunks(const lbm_params& p, const ZChunks& zk) {
    if (!solid_free_enabled()) return 0;
    for (int a = 0; a < 2; ++a)
        if (p.bc[a][0] == LBM_BC_WALL || p.bc[a][1] == LBM_BC_WALL) return 0;
    const int nz = p.nz;
    auto solid_plane = [&](int z) {
        z = ((z % nz) + nz) % nz;
        if (p.bc[2][0] == LBM_BC_WALL && z == 0) return true;
        if (p.bc[2][1] == LBM_BC_WALL && z == nz - 1) return true;
        if (p.cylinder && z >= std::floor(p.cyl_z - p.cyl_r) - 1 && z <= std::ceil(p.cyl_z + p.cyl_r) + 1)
            return true;
        return false;
    };
    uint64_t m = 0;
    for (int iz = 0; iz < zk.n && iz < 64; ++iz) {
        const int z0 = iz == 0 ? 0 : zk.zlo + (iz - 1) * zk.zc;
        const int z1 = std::min(zk.zlo + iz * zk.zc, nz);
        bool free = true;
        for (int z = z0 - 2; z <= z1 + 1 && free; ++z) free = !solid_plane(z);
        if (free) m |= 1ull << iz;
    }
    return m;
}

// Planes per z-chunk, tile order and cache hints of a launch (defaults of fused.h, then the
// LBM_FUSED_* tuning overrides), and the workgroup count.
struct FusedPlan { int zc, zlo, remap, hints; long long workgroups; };
inline FusedPlan fused_plan(const lbm_params& p, int elem, int cfg, int cus) {
    const FusedCfg& f = kFusedCfgs[cfg];
    const long long tiles = (long long)((p.nx + f.tx - 1) / f.tx) * ((p.ny + f.ty - 1) / f.ty);
    FusedPlan pl;
    pl.zc = default_fused_zc(f, tiles, p.nz, cus);
    pl.remap = default_fused_remap(f);
    pl.hints = default_fused_hints(f, elem);
    if (const char* e = getenv("LBM_FUSED_HINTS")) pl.hints = atoi(e);         // tuning override
    if (const char* e = getenv("LBM_FUSED_ZC")) pl.zc = std::max(1, atoi(e));   // tuning override
    if (const char* e = getenv("LBM_FUSED_REMAP")) pl.remap = atoi(e) != 0;    // tuning override
    pl.zc = std::min(pl.zc, p.nz);
    const ZChunks zk = fused_zchunks(p, elem, cfg, pl.zc);
    pl.zc = zk.zc;
    pl.zlo = zk.zlo;
    pl.workgroups = tiles * zk.n;
    return pl;
}

inline void fused_chunking(const lbm_ctx* c, int& zc, int& remap, int& hints, int& zlo,
                           int& nchunks) {
    const FusedPlan pl = fused_plan(c->p, (int)c->elem, c->fused_cfg, c->cus);
    zc = pl.zc;
    zlo = pl.zlo;
    nchunks = zchunks_of(c->p.nz, pl.zlo, pl.zc).n;
    remap = pl.remap;
    hints = pl.hints;
}

// Link words of the fused step on a solid mask (stream-ordered after the mask; api.hip).
hipError_t build_links(lbm_ctx* c);

// Enqueue a health check of the current state on the context stream (api.hip); its result
// is read by the context's next lbm_step, lbm_synchronize, lbm_moments or lbm_liquid_stats.
lbm_status enqueue_health(lbm_ctx* c);

// Step kernels of one (lattice, storage type) pair, enqueued on the context stream:
//   fused    one fused time step fin -> fout (the configuration in c->fused_cfg);
//   psi      the density/pseudopotential pass of the two-pass step into c->psi;
//   collide  the collision pass of the two-pass step (needs psi of fin).
// Defined in step_ops.h and instantiated once per pair in step_q*_*.hip.
template <int Q, typename T>
struct StepOps {
    static void fused(lbm_ctx* c, const void* fin, void* fout);
    static void psi(lbm_ctx* c, const void* fin);
    static void collide(lbm_ctx* c, const void* fin, void* fout);
};
extern template struct StepOps<19, double>;
extern template struct StepOps<19, float>;
extern template struct StepOps<19, _Float16>;
extern template struct StepOps<27, double>;
extern template struct StepOps<27, float>;
extern template struct StepOps<27, _Float16>;
