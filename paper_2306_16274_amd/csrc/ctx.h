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
    int sf0 = 0, sf1 = 0;          // planes [sf0, sf1) run the solid-free form (solid_free_range)
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

// Solid-free form of the fused tiles (fused_segments in fused.h), 2- and 4-byte storage:
// planes z whose planes z - 2 .. z + 2 hold no solid node run the arithmetic of a lattice
// without solid nodes. LBM_SOLID_FREE=0 turns it off (tuning).
inline bool solid_free_enabled() {
    const char* e = getenv("LBM_SOLID_FREE");
    return !e || atoi(e) != 0;
}

// The longest run [sf0, sf1) of planes z whose planes z - 2 .. z + 2 hold no solid node
// (sf0 = sf1 = 0 if none). Walls along x or y put solid nodes in every plane; a wall along z
// is the plane 0 or nz - 1; a cylinder along x fills the planes cyl_z - cyl_r .. cyl_z + cyl_r
// (taken one plane wider either side). A lattice without walls or cylinder is periodic in z:
// every plane qualifies.
inline void solid_free_range(const lbm_params& p, int& sf0, int& sf1) {
    sf0 = sf1 = 0;
    if (!solid_free_enabled()) return;
    for (int a = 0; a < 2; ++a)
        if (p.bc[a][0] == LBM_BC_WALL || p.bc[a][1] == LBM_BC_WALL) return;
    const int nz = p.nz;
    auto solid_plane = [&](int z) {
        if (z < 0 || z >= nz) z = ((z % nz) + nz) % nz;
        if (p.bc[2][0] == LBM_BC_WALL && z == 0) return true;
        if (p.bc[2][1] == LBM_BC_WALL && z == nz - 1) return true;
        return p.cylinder != 0 && z >= std::floor(p.cyl_z - p.cyl_r) - 1 &&
               z <= std::ceil(p.cyl_z + p.cyl_r) + 1;
    };
    int run0 = 0;
    for (int z = 0; z <= nz; ++z) {
        bool clear = z < nz;
        for (int d = -2; d <= 2 && clear; ++d) clear = !solid_plane(z + d);
        if (!clear) {
            if (z - run0 > sf1 - sf0) { sf0 = run0; sf1 = z; }
            run0 = z + 1;
        }
    }
}

inline Grid grid_of(const lbm_ctx* c) {
    Grid g;
    g.nx = c->p.nx; g.ny = c->p.ny; g.nz = c->p.nz; g.stride = c->stride;
    g.walls = 0;
    g.sf0 = c->sf0;
    g.sf1 = c->sf1;
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

// Planes per z-chunk, tile order and cache hints of a launch (defaults of fused.h, then the
// LBM_FUSED_* tuning overrides), and the workgroup count.
struct FusedPlan { int zc, remap, hints; long long workgroups; };
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
    pl.workgroups = tiles * ((p.nz + pl.zc - 1) / pl.zc);
    return pl;
}

inline void fused_chunking(const lbm_ctx* c, int& zc, int& remap, int& hints) {
    const FusedPlan pl = fused_plan(c->p, (int)c->elem, c->fused_cfg, c->cus);
    zc = pl.zc;
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
