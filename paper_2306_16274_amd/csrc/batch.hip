// Batched stepping of many lattices (the serving loop's launch path): one launch per time
// step over every member's tiles (row tiles of run-time width, k_step_fused_batch_rows, for
// FP32 members up to 384 wide; else 64x4 tiles, k_step_fused_batch), steps_per_launch
// launches captured once into a HIP graph. C ABI: lbm_batch_* in include/lbm.h.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"

// Tile shapes of the batched kernel (index lbm_batch::tile) and the z-chunk depth.
constexpr int kBatchTiles[2][2] = {{64, 4}, {32, 8}};
constexpr int kBatchZC = 16;
// z-chunk depth of the row tiles: with the solid-free segments 12-plane chunks beat 16 on
// serving mixes (GLUPS, two runs each; 24 mixed sizes 28.0-28.2 vs 27.7-27.8, 8 x 128^3
// 30.2-30.8 vs 30.1-30.5, 32 x 64^3 30.3-30.7 vs 29.8-30.2, 2 x 192^3 31.7-31.9 vs
// 30.3-30.4; 8, 10, 14, 24 and 32 no better overall).
constexpr int kRowsZC = 12;
// Row tiles (k_step_fused_batch_rows): threads per workgroup (12 wavefronts: the walled
// kernel fits the 168 VGPRs that leaves); members up to kRowsNT / 2
// wide, 4-byte storage.
constexpr int kRowsNT = 768;

struct lbm_batch {
    std::vector<lbm_ctx*> ctx;
    int steps_per_launch = 2;
    int storage = LBM_FP32;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* table[2] = {nullptr, nullptr};  // device DomainDesc arrays: even / odd steps
    std::vector<char> host_table[2];      // their sources (alive until the copies are done)
    bool ran = false;
    long long blocks = 0;
    int geom = GEOM_WALLS;                // GEOM_MASK if any member has a cylinder
    int tile = 0;                         // index into kBatchTiles
    bool rows = false;                    // row tiles of run-time width instead
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    std::vector<hipEvent_t> ready;
};

static thread_local std::string g_batch_error;    // per calling thread
static lbm_status batch_fail(lbm_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_batch_error = buf;
    return s;
}
#define BCHK(call) do { hipError_t e_ = (call); if (e_ != hipSuccess)                        \
    return batch_fail(e_ == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "%s failed: %s",  \
                      #call, hipGetErrorString(e_)); } while (0)

template <typename T, int TX, int TY>
static void launch_batch(const lbm_batch* b, hipStream_t s, const void* table, bool pf, bool nt,
                         int remap) {
    const dim3 grid((unsigned)b->blocks), block(TX * TY);
    const DomainDesc<T>* tb = (const DomainDesc<T>*)table;
    const int nd = (int)b->ctx.size();
    auto go = [&](auto geom, auto nts) {
        constexpr int G = decltype(geom)::value;
        constexpr bool N = decltype(nts)::value;
        if constexpr (sizeof(T) == 4) {
            if (pf) {
                hipLaunchKernelGGL((k_step_fused_batch_pf<19, T, G, TX, TY, N>), grid, block, 0, s,
                                   tb, nd, remap);
                return;
            }
        }
        hipLaunchKernelGGL((k_step_fused_batch<19, T, G, TX, TY, N>), grid, block, 0, s, tb, nd, remap);
    };
    using std::integral_constant;
    if (b->geom == GEOM_MASK) {
        if (nt) go(integral_constant<int, GEOM_MASK>{}, integral_constant<bool, true>{});
        else go(integral_constant<int, GEOM_MASK>{}, integral_constant<bool, false>{});
    } else {
        if (nt) go(integral_constant<int, GEOM_WALLS>{}, integral_constant<bool, true>{});
        else go(integral_constant<int, GEOM_WALLS>{}, integral_constant<bool, false>{});
    }
}

template <typename T>
static void launch_batch_rows(const lbm_batch* b, hipStream_t s, const void* table, bool nt,
                              int remap) {
    if constexpr (sizeof(T) == 4) {
        const dim3 grid((unsigned)b->blocks), block(kRowsNT);
        const DomainDesc<T>* tb = (const DomainDesc<T>*)table;
        const int nd = (int)b->ctx.size();
        auto go = [&](auto geom, auto nts) {
            hipLaunchKernelGGL((k_step_fused_batch_rows<19, T, decltype(geom)::value, kRowsNT,
                                                        decltype(nts)::value>),
                               grid, block, 0, s, tb, nd, remap);
        };
        using std::integral_constant;
        if (b->geom == GEOM_MASK) {
            if (nt) go(integral_constant<int, GEOM_MASK>{}, integral_constant<bool, true>{});
            else go(integral_constant<int, GEOM_MASK>{}, integral_constant<bool, false>{});
        } else {
            if (nt) go(integral_constant<int, GEOM_WALLS>{}, integral_constant<bool, true>{});
            else go(integral_constant<int, GEOM_WALLS>{}, integral_constant<bool, false>{});
        }
    }
}

template <typename T>
static lbm_status build_tables(lbm_batch* b) {
    using R = typename Arith<T>::type;
    std::vector<DomainDesc<T>> t[2];
    long long block0 = 0;
    const int TX = kBatchTiles[b->tile][0], TY = kBatchTiles[b->tile][1];
    for (lbm_ctx* c : b->ctx) {
        // row tiles: as many whole rows as the workgroup holds
        const int rows = b->rows ? std::min(kRowsNT / c->p.nx, c->p.ny) : 0;
        const int ntx = b->rows ? 1 : (c->p.nx + TX - 1) / TX;
        const int nty = b->rows ? (c->p.ny + rows - 1) / rows : (c->p.ny + TY - 1) / TY;
        int zc = b->rows ? kRowsZC : kBatchZC;
        if (const char* e = getenv("LBM_BATCH_ZC")) zc = std::max(1, atoi(e));    // tuning override
        zc = std::min(zc, c->p.nz);
        const long long nb = (long long)ntx * nty * ((c->p.nz + zc - 1) / zc);
        const Phys<R>& P = phys_of<R>(c);
        for (int par = 0; par < 2; ++par) {
            DomainDesc<T> d{};
            d.fin = (const T*)c->f[(c->cur + par) & 1];
            d.fout = (T*)c->f[(c->cur + par + 1) & 1];
            d.links = c->links;
            d.g = grid_of(c);
            d.P = P;
            d.ntx = ntx; d.nty = nty; d.zc = zc; d.block0 = (int)block0;
            d.rows = rows;
            t[par].push_back(d);
        }
        block0 += nb;
    }
    if (block0 > 0x7fffffffLL) return batch_fail(LBM_EINVAL, "batch too large");
    b->blocks = block0;
    const size_t bytes = t[0].size() * sizeof(DomainDesc<T>);
    for (int par = 0; par < 2; ++par) {
        b->host_table[par].resize(bytes);
        std::memcpy(b->host_table[par].data(), t[par].data(), bytes);
        BCHK(dmalloc(b->stream, &b->table[par], bytes));
        BCHK(hipMemcpyAsync(b->table[par], b->host_table[par].data(), bytes, hipMemcpyHostToDevice,
                            b->stream));
    }
    // capture steps_per_launch launches, alternating the two tables, on a private stream
    hipStream_t cap = nullptr;
    BCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipError_t ce = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (ce != hipSuccess) { (void)hipStreamDestroy(cap); BCHK(ce); }
    // Plain tiles: on serving mixes of box sizes (rows not 128-byte aligned) they beat the
    // prefetching tiles (19.2 vs 17.9 GLUPS) and 32x8 tiles (16.2); LBM_BATCH_PF=1 selects
    // the prefetching tiles for 4-byte storage (tuning).
    // Nontemporal stores when every member's rows are whole 128-byte lines (serving shapes,
    // GLUPS, nontemporal vs plain: 8x128^3 23.0 vs 22.6, 32x64^3 26.7 vs 26.2, 2x192^3 23.5
    // vs 23.2; 24 mixed sizes, mostly unaligned rows: 18.1 vs 19.1).
    bool pf = false, nt = true;
    for (const lbm_ctx* c : b->ctx) nt = nt && ((long long)c->p.nx * (long long)c->elem) % 128 == 0;
    if (const char* e = getenv("LBM_BATCH_PF")) pf = sizeof(T) == 4 && atoi(e) != 0;
    if (const char* e = getenv("LBM_BATCH_NT")) nt = atoi(e) != 0;              // tuning override
    // XCD-contiguous tile ranges, as for single lattices (GLUPS, on / off: 8x128^3 24.3 / 23.0,
    // 16x96^3 23.3 / 21.3, 32x64^3 27.8 / 26.3, 2x192^3 26.0 / 23.5, 24 mixed 19.9 / 19.1)
    int remap = 1;
    if (const char* e = getenv("LBM_BATCH_REMAP")) remap = atoi(e) != 0;       // tuning override
    for (int s = 0; s < b->steps_per_launch; ++s) {
        if (b->rows)
            launch_batch_rows<T>(b, cap, b->table[s & 1], nt, remap);
        else if (b->tile == 0)
            launch_batch<T, kBatchTiles[0][0], kBatchTiles[0][1]>(b, cap, b->table[s & 1], pf, nt, remap);
        else
            launch_batch<T, kBatchTiles[1][0], kBatchTiles[1][1]>(b, cap, b->table[s & 1], pf, nt, remap);
    }
    ce = hipStreamEndCapture(cap, &b->graph);
    (void)hipStreamDestroy(cap);
    BCHK(ce);
    BCHK(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    return LBM_OK;
}

static void batch_free(lbm_batch* b) {
    if (!b) return;
    // wait for this batch's own replays only (work queued after them keeps running)
    if (b->ran && b->done) (void)hipEventSynchronize(b->done);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->stream)
        for (void* t : b->table) dfree(b->stream, t);
    if (b->done) (void)hipEventDestroy(b->done);
    for (hipEvent_t e : b->ready) if (e) (void)hipEventDestroy(e);
    if (b->own_stream && b->stream) {
        (void)hipStreamSynchronize(b->stream);
        (void)hipStreamDestroy(b->stream);
    }
}

extern "C" lbm_status lbm_batch_create(lbm_ctx* const* ctxs, int32_t n, int32_t steps_per_launch,
                                       void* stream, lbm_batch** out) {
    if (!ctxs || !out || n < 1) return batch_fail(LBM_EINVAL, "need at least one context");
    if (steps_per_launch < 2 || steps_per_launch % 2)
        return batch_fail(LBM_EINVAL, "steps_per_launch must be even and >= 2");
    *out = nullptr;
    const int storage = ctxs[0]->p.storage;
    for (int i = 0; i < n; ++i) {
        const lbm_ctx* c = ctxs[i];
        if (!c) return batch_fail(LBM_EINVAL, "null context");
        if (c->device != ctxs[0]->device) return batch_fail(LBM_EINVAL, "members must share a device");
        if (c->Q != 19) return batch_fail(LBM_EINVAL, "batched stepping supports D3Q19");
        if (c->p.storage != storage || storage == LBM_FP16)
            return batch_fail(LBM_EINVAL, "members must share FP32 or FP64 storage");
        if (!c->initialised || c->failed) return batch_fail(LBM_ESTATE, "member %d not initialised or failed", i);
        if ((double)c->Q * (double)c->stride * (double)c->elem >= 4294967296.0)
            return batch_fail(LBM_EINVAL, "member %d has a population buffer of 4 GiB or more", i);
        for (int j = 0; j < i; ++j)
            if (ctxs[j] == c) return batch_fail(LBM_EINVAL, "context %d appears twice", i);
    }
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return batch_fail(LBM_ENOMEM, "host allocation failed");
    b->ctx.assign(ctxs, ctxs + n);
    b->steps_per_launch = steps_per_launch;
    b->storage = storage;
    for (int i = 0; i < n; ++i)
        if (ctxs[i]->p.cylinder && ctxs[i]->any_solid) b->geom = GEOM_MASK;
    if (const char* e = getenv("LBM_BATCH_TILE")) b->tile = atoi(e) == 1 ? 1 : 0;   // tuning override
    // Row tiles (the default where they apply: 4-byte storage, members at most kRowsNT / 2
    // wide) against the 64x4 tiles, serving physics, GLUPS: 24 mixed sizes 64-192 26.8 vs
    // 19.7, 8 x 128^3 29.0 vs 23.9, 32 x 64^3 28.6-29.0 vs 26.6, 2 x 192^3 27.8 vs 25.3 (no
    // x-halo, whole rows on 128-byte lines where the width allows; 512-thread row tiles
    // lost on 192-wide members, where only two rows fit).
    bool rows_ok = storage == LBM_FP32;
    for (int i = 0; i < n; ++i) rows_ok = rows_ok && ctxs[i]->p.nx <= kRowsNT / 2;
    b->rows = rows_ok;
    if (const char* e = getenv("LBM_BATCH_ROWS")) b->rows = rows_ok && atoi(e) != 0;   // tuning
    auto bail = [&](lbm_status s) { batch_free(b); delete b; return s; };
    hipError_t e = hipSetDevice(ctxs[0]->device);
    if (e == hipSuccess) {
        if (stream) b->stream = (hipStream_t)stream;
        else { e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking); b->own_stream = true; }
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->done, hipEventDisableTiming);
    b->ready.assign(n, nullptr);
    for (int i = 0; e == hipSuccess && i < n; ++i) e = hipEventCreateWithFlags(&b->ready[i], hipEventDisableTiming);
    // a batch on the solid mask reads every member's link words (members without a
    // cylinder get them here, from their wall mask)
    for (int i = 0; e == hipSuccess && b->geom == GEOM_MASK && i < n; ++i) e = build_links(ctxs[i]);
    if (e != hipSuccess) { batch_fail(LBM_EDEVICE, "batch setup failed: %s", hipGetErrorString(e)); return bail(LBM_EDEVICE); }
    lbm_status st = storage == LBM_FP64 ? build_tables<double>(b) : build_tables<float>(b);
    if (st != LBM_OK) return bail(st);
    *out = b;
    return LBM_OK;
}

extern "C" lbm_status lbm_batch_run(lbm_batch* b, int64_t nlaunch) {
    if (!b) return batch_fail(LBM_EINVAL, "null batch");
    if (nlaunch < 0) return batch_fail(LBM_EINVAL, "nlaunch must be >= 0");
    for (lbm_ctx* c : b->ctx)
        if (c->failed) return batch_fail(LBM_ESTATE, "a member failed its health check");
    BCHK(hipSetDevice(b->ctx[0]->device));
    // order after each member's stream, replay, then order each member's stream after us
    for (size_t i = 0; i < b->ctx.size(); ++i) {
        BCHK(hipEventRecord(b->ready[i], b->ctx[i]->stream));
        BCHK(hipStreamWaitEvent(b->stream, b->ready[i], 0));
    }
    for (int64_t k = 0; k < nlaunch; ++k) BCHK(hipGraphLaunch(b->exec, b->stream));
    BCHK(hipEventRecord(b->done, b->stream));
    b->ran = true;
    for (lbm_ctx* c : b->ctx) {
        BCHK(hipStreamWaitEvent(c->stream, b->done, 0));
        c->steps += nlaunch * b->steps_per_launch;      // even count: c->cur unchanged
        // members that ask for health checks get one after this run, on their own stream;
        // a failure is reported by the member's next lbm_step / lbm_synchronize /
        // lbm_moments and makes later lbm_batch_run calls on a batch holding it fail
        if (nlaunch > 0 && c->p.reduce_every > 0) {
            const lbm_status st = enqueue_health(c);
            if (st != LBM_OK) return batch_fail(st, "health check of a member: %s", c->err.c_str());
        }
    }
    return LBM_OK;
}

extern "C" lbm_status lbm_batch_destroy(lbm_batch* b) {
    if (!b) return LBM_OK;
    batch_free(b);
    delete b;
    return LBM_OK;
}

extern "C" const char* lbm_batch_last_error(void) { return g_batch_error.c_str(); }
