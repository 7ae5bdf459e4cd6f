// Host side of the C ABI declared in include/lbm.h: parameter validation, device
// buffers, dispatch over (lattice, storage type) to the step kernels (StepOps, compiled in
// the step_q*_*.hip units), the diagnostics and the host-only coexistence solver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "ctx.h"
#include "kernels.h"
#include "misc_kernels.h"

thread_local std::string g_create_error;   // per calling thread

// ---------------------------------------------------------------------------------------
// Device scratch of lbm_totals_noalloc: the per-block partial sums of its reduction,
// kTotalsBlocks blocks x 5 doubles = 40 KiB in every device's copy of the library, held
// until the process ends. Host code never passes the array's name to a kernel (on the host
// it is only a stand-in for the symbol): the address of each device's copy is looked up
// once per device, with that device current, when the first lattice is created on it
// (ensure_scratch, called from lbm_create), and kept in g_scratch_ptr.
constexpr int kTotalsBlocks = 1024;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double scratch[kTotalsBlocks * 5];
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

static hipError_t ensure_scratch(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    if (g_scratch_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e == hipSuccess) g_scratch_ptr[device] = static_cast<double*>(ptr);
    return e;
}

static double* scratch_of(int device) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}

static int default_fused_cfg(const lbm_ctx* c) {
    return fused_cfg_for(c->p.nx, (int)c->elem, c->Q, c->addr64, c->p.cylinder != 0);
}

// ---------------------------------------------------------------------------------------
// Equations of state on the host (float64), for validation and the coexistence solver.
static double eos_p(const lbm_params& p, double rho) {
    if (p.eos == LBM_EOS_CS) {
        const double T = p.T_over_Tc * 0.3773 * p.cs_a / (p.cs_b * p.cs_R);
        const double eta = p.cs_b * rho / 4.0, om = 1.0 - eta;
        return rho * p.cs_R * T * (1 + eta + eta * eta - eta * eta * eta) / (om * om * om) -
               p.cs_a * rho * rho;
    }
    const double p1 = p.pw_rho1 * p.pw_theta_v;
    const double p2 = p1 + (p.pw_rho2 - p.pw_rho1) * p.pw_theta_m;
    if (rho <= p.pw_rho1) return rho * p.pw_theta_v;
    if (rho <= p.pw_rho2) return p1 + (rho - p.pw_rho1) * p.pw_theta_m;
    return p2 + (rho - p.pw_rho2) * p.pw_theta_l;
}

static double eos_rho_max(const lbm_params& p) {
    return p.eos == LBM_EOS_CS ? 0.999 * 4.0 / p.cs_b : 50.0;
}

// integral of p(rho)/rho^2 over [a, b] with composite 8-point Gauss-Legendre in ln(rho);
// for the piecewise EOS the interval is split at its knees (p is only piecewise smooth).
// Nodes and weights of the 8-point rule on [-1, 1] (the roots of the Legendre polynomial
// P_8 and w_j = 2 / ((1 - x_j^2) P_8'(x_j)^2), as tabulated in Abramowitz and Stegun,
// Handbook of Mathematical Functions, Table 25.4); the positive half, used symmetrically.
static double int_smooth(const lbm_params& p, double a, double b) {
    static const double xg[4] = {0.1834346424956498, 0.5255324099163290, 0.7966664774136267,
                                 0.9602898564975363};
    static const double wg[4] = {0.3626837833783620, 0.3137066458778873, 0.2223810344533745,
                                 0.1012285362903763};
    const double la = std::log(a), lb = std::log(b);
    const int panels = 64;
    const double hw = (lb - la) / panels;
    double s = 0;
    for (int k = 0; k < panels; ++k) {
        const double mid = la + (k + 0.5) * hw;
        for (int j = 0; j < 4; ++j)
            for (int sg = -1; sg <= 1; sg += 2) {
                const double t = mid + sg * xg[j] * 0.5 * hw;
                const double r = std::exp(t);
                s += wg[j] * 0.5 * hw * eos_p(p, r) / r;
            }
    }
    return s;
}

static double int_p_over_rho2(const lbm_params& p, double a, double b) {
    if (p.eos != LBM_EOS_PIECEWISE) return int_smooth(p, a, b);
    double cuts[4] = {a, 0, 0, b};
    int n = 1;
    for (double k : {p.pw_rho1, p.pw_rho2})
        if (k > a && k < b) cuts[n++] = k;
    cuts[n++] = b;
    double s = 0;
    for (int i = 0; i + 1 < n; ++i) s += int_smooth(p, cuts[i], cuts[i + 1]);
    return s;
}

extern "C" lbm_status lbm_coexistence(const lbm_params* pp, double* rho_v, double* rho_l) {
    if (!pp || !rho_v || !rho_l) return fail(nullptr, LBM_EINVAL, "null argument");
    const lbm_params& p = *pp;
    const double hi = eos_rho_max(p), lo = 1e-9;
    // spinodals: sample dp/drho for the unstable branch, refine the sign changes by bisection
    const int M = 4000;
    auto dp = [&](double r) { const double h = 1e-7 * std::max(r, 1e-6);
                              return (eos_p(p, r + h) - eos_p(p, r - h)) / (2 * h); };
    auto refine = [&](double a, double b) {       // dp changes sign in [a, b]
        const bool sa = dp(a) < 0;
        for (int it = 0; it < 60; ++it) {
            const double m = 0.5 * (a + b);
            if ((dp(m) < 0) == sa) a = m; else b = m;
        }
        return 0.5 * (a + b);
    };
    double s_lo = -1, s_hi = -1, prev = dp(lo);
    double rprev = lo;
    for (int k = 1; k <= M; ++k) {
        const double r = lo + (hi - lo) * k / M;
        const double v = dp(r);
        if (prev >= 0 && v < 0 && s_lo < 0) s_lo = refine(rprev, r);
        if (prev < 0 && v >= 0) s_hi = refine(rprev, r);
        prev = v; rprev = r;
    }
    if (s_lo < 0 || s_hi < 0)
        return fail(nullptr, LBM_EINVAL, "equation of state has no two-phase region");
    const double pmax = eos_p(p, s_lo), pmin = std::max(eos_p(p, s_hi), eos_p(p, lo));
    auto root = [&](double p0, double a, double b) {   // p(r) = p0 on a monotone branch
        double fa = eos_p(p, a) - p0;
        for (int it = 0; it < 100; ++it) {
            const double m = 0.5 * (a + b), fm = eos_p(p, m) - p0;
            if ((fm < 0) == (fa < 0)) { a = m; fa = fm; } else b = m;
        }
        return 0.5 * (a + b);
    };
    auto area = [&](double p0, double* rv, double* rl) {
        *rv = root(p0, lo, s_lo);
        *rl = root(p0, hi, s_hi);
        return p0 * (1.0 / *rl - 1.0 / *rv) + int_p_over_rho2(p, *rv, *rl);
    };
    double a = pmin + 1e-12 * std::fabs(pmax), b = pmax - 1e-12 * std::fabs(pmax), rv, rl;
    double fa = area(a, &rv, &rl);
    for (int it = 0; it < 80; ++it) {
        const double m = 0.5 * (a + b), fm = area(m, &rv, &rl);
        if ((fm < 0) == (fa < 0)) { a = m; fa = fm; } else b = m;
        if (b - a <= 1e-16 * std::fabs(pmax)) break;
    }
    area(0.5 * (a + b), &rv, &rl);
    *rho_v = rv; *rho_l = rl;
    return LBM_OK;
}

// ---------------------------------------------------------------------------------------
extern "C" lbm_status lbm_params_default(lbm_params* p) {
    if (!p) return LBM_EINVAL;
    std::memset(p, 0, sizeof *p);
    p->lattice = 19; p->storage = LBM_FP32;
    p->nx = p->ny = p->nz = 64;
    p->eos = LBM_EOS_CS;
    p->cs_a = 0.5; p->cs_b = 4.0; p->cs_R = 1.0; p->T_over_Tc = 0.7;
    p->pw_theta_v = 1.0 / 6.0; p->pw_theta_m = -1.0 / 120.0; p->pw_theta_l = 1.0 / 3.0;
    p->pw_rho1 = 0.0013246030524; p->pw_rho2 = 0.9758004064415;
    p->G = -1.0; p->sigma = 0.1; p->kappa = 0.0; p->G_ads = 0.0;
    p->wall_psi = LBM_WALL_PSI_MIRROR;
    p->nu_l = p->nu_v = 0.1; p->rho_l = 1.0; p->rho_v = 0.001;
    p->s0 = 1.0; p->s1 = 1.0; p->s2b = 0.6; p->s3 = 1.2; p->s3b = 0.6;
    p->s4 = 1.2; p->s4b = 1.2; p->s5 = 1.2; p->s6 = 1.2;
    return LBM_OK;
}


extern "C" int64_t lbm_footprint_bytes(const lbm_params* p) {
    if (!p || p->nx < 1 || p->ny < 1 || p->nz < 1) return -1;
    const long long N = (long long)p->nx * p->ny * p->nz;
    const int Q = p->lattice == 27 ? 27 : 19;
    const size_t b = storage_bytes(p->storage);
    const size_t r = p->storage == LBM_FP64 ? 8 : 4;
    const size_t links = p->cylinder ? 4 : 0;     // link words of the fused step
    return (int64_t)(2 * Q * plane_stride(N) * b + N * r + N + N * links);
}

template <typename R>
static Phys<R> make_phys(const lbm_params& p) {
    Phys<R> P{};
    P.rho_ref = (R)p.rho_ref;
    P.G = (R)p.G; P.two_over_G = (R)(2.0 / p.G);
    P.sigma = (R)p.sigma; P.kappa = (R)p.kappa; P.G_ads = (R)p.G_ads;
    P.eos = p.eos == LBM_EOS_CS ? EOS_CS : EOS_PIECEWISE;
    P.cs_a = (R)p.cs_a; P.cs_b = (R)p.cs_b;
    P.cs_RT = (R)(p.cs_R * p.T_over_Tc * 0.3773 * p.cs_a / (p.cs_b * p.cs_R));
    P.pw_tv = (R)p.pw_theta_v; P.pw_tm = (R)p.pw_theta_m; P.pw_tl = (R)p.pw_theta_l;
    P.pw_r1 = (R)p.pw_rho1; P.pw_r2 = (R)p.pw_rho2;
    const double p1 = p.pw_rho1 * p.pw_theta_v;
    P.pw_p1 = (R)p1; P.pw_p2 = (R)(p1 + (p.pw_rho2 - p.pw_rho1) * p.pw_theta_m);
    P.s_nu = (R)(1.0 / (3.0 * p.nu_l + 0.5));
    P.s_e = (R)p.s2b; P.s3 = (R)p.s3; P.s3b = (R)p.s3b; P.s4 = (R)p.s4; P.s4b = (R)p.s4b;
    P.s5 = (R)p.s5; P.s6 = (R)p.s6;
    P.var_nu = p.nu_v != p.nu_l;
    P.nu_v = (R)p.nu_v; P.rho_v = (R)p.rho_v;
    P.dnu_drho = P.var_nu ? (R)((p.nu_l - p.nu_v) / (p.rho_l - p.rho_v)) : R(0);
    P.bfx = (R)p.body_force[0]; P.bfy = (R)p.body_force[1]; P.bfz = (R)p.body_force[2];
    P.wall_psi = p.wall_psi;
    return P;
}


static bool rate_ok(double s) { return s > 0.0 && s < 2.0 && std::isfinite(s); }

static lbm_status validate(const lbm_params& p) {
    if (p.lattice != 19 && p.lattice != 27) return fail(nullptr, LBM_EINVAL, "lattice must be 19 or 27");
    if (p.storage < LBM_FP64 || p.storage > LBM_FP16) return fail(nullptr, LBM_EINVAL, "unknown storage type");
    if (p.nx < 1 || p.ny < 1 || p.nz < 1) return fail(nullptr, LBM_EINVAL, "lattice sizes must be >= 1");
    const long long N = (long long)p.nx * p.ny * p.nz;
    if (N > 0x7fffffffLL) return fail(nullptr, LBM_EINVAL, "more than 2^31-1 nodes");
    if (p.nz > 65535 || p.ny > 65535 * 4)
        return fail(nullptr, LBM_EINVAL, "nz above 65535 or ny above 262140 (launch grid limits)");
    if (p.eos != LBM_EOS_CS && p.eos != LBM_EOS_PIECEWISE) return fail(nullptr, LBM_EINVAL, "unknown eos");
    if (!(p.G < 0.0)) return fail(nullptr, LBM_EINVAL, "G must be negative (attractive)");
    if (p.eos == LBM_EOS_CS && !(p.cs_a > 0 && p.cs_b > 0 && p.cs_R > 0 && p.T_over_Tc > 0))
        return fail(nullptr, LBM_EINVAL, "Carnahan-Starling a, b, R, T must be positive");
    if (p.eos == LBM_EOS_PIECEWISE &&
        !(p.pw_theta_v > 0 && p.pw_theta_l > 0 && p.pw_theta_m < 0 && p.pw_rho1 > 0 && p.pw_rho2 > p.pw_rho1))
        return fail(nullptr, LBM_EINVAL, "piecewise EOS needs theta_v, theta_l > 0 > theta_m and 0 < rho1 < rho2");
    const double finite[] = {p.rho_ref, p.sigma, p.kappa, p.G_ads, p.G, p.body_force[0],
                             p.body_force[1], p.body_force[2], p.cyl_y, p.cyl_z, p.cyl_r};
    for (double v : finite)
        if (!std::isfinite(v)) return fail(nullptr, LBM_EINVAL, "non-finite parameter value");
    if (p.cylinder && !(p.cyl_r > 0)) return fail(nullptr, LBM_EINVAL, "cylinder radius must be positive");
    if (!(p.nu_l > 0) || !(p.nu_v > 0)) return fail(nullptr, LBM_EINVAL, "viscosities must be positive");
    if (p.nu_v != p.nu_l && !(p.rho_l != p.rho_v)) return fail(nullptr, LBM_EINVAL, "rho_l == rho_v with nu_l != nu_v");
    const double rates[] = {p.s2b, p.s3, p.s3b, p.s4, p.s4b, p.s5, p.s6, 1.0 / (3 * p.nu_l + 0.5),
                            1.0 / (3 * p.nu_v + 0.5)};
    for (double s : rates)
        if (!rate_ok(s)) return fail(nullptr, LBM_EINVAL, "relaxation rate %g outside (0, 2)", s);
    for (int a = 0; a < 3; ++a)
        for (int s = 0; s < 2; ++s)
            if (p.bc[a][s] != LBM_BC_PERIODIC && p.bc[a][s] != LBM_BC_WALL)
                return fail(nullptr, LBM_EINVAL, "unknown boundary condition");
    if (p.reduce_every < 0) return fail(nullptr, LBM_EINVAL, "reduce_every must be >= 0");
    if (p.step_kernel != LBM_STEP_FUSED && p.step_kernel != LBM_STEP_TWO_PASS)
        return fail(nullptr, LBM_EINVAL, "unknown step_kernel");
    if (p.wall_psi < LBM_WALL_PSI_NODE || p.wall_psi > LBM_WALL_PSI_MIRROR)
        return fail(nullptr, LBM_EINVAL, "unknown wall_psi");
    return LBM_OK;
}


// Solid nodes: wall layers on the faces marked LBM_BC_WALL and the nodes whose centre lies
// in the x-aligned cylinder. The mask is written on the device (k_build_solid, the same
// predicate); the host only counts solid nodes, from one (y, z) plane since the geometry
// does not depend on x except through the x walls.
static bool solid_yz(const lbm_params& p, int y, int z) {
    if (p.bc[1][0] == LBM_BC_WALL && y == 0) return true;
    if (p.bc[1][1] == LBM_BC_WALL && y == p.ny - 1) return true;
    if (p.bc[2][0] == LBM_BC_WALL && z == 0) return true;
    if (p.bc[2][1] == LBM_BC_WALL && z == p.nz - 1) return true;
    if (p.cylinder) {
        const double dy = y - p.cyl_y, dz = z - p.cyl_z;
        if (dy * dy + dz * dz <= p.cyl_r * p.cyl_r) return true;
    }
    return false;
}

static long long count_fluid(const lbm_params& p, bool& any_solid) {
    long long yz_fluid = 0;
    for (int z = 0; z < p.nz; ++z)
        for (int y = 0; y < p.ny; ++y) yz_fluid += !solid_yz(p, y, z);
    int x_fluid = p.nx;
    if (p.bc[0][0] == LBM_BC_WALL) --x_fluid;
    if (p.bc[0][1] == LBM_BC_WALL && p.nx > 1) --x_fluid;
    x_fluid = std::max(x_fluid, 0);
    const long long fluid = yz_fluid * x_fluid;
    any_solid = fluid != (long long)p.nx * p.ny * p.nz;
    return fluid;
}

// Link words for the fused step on a solid mask (stream-ordered after the mask).
hipError_t build_links(lbm_ctx* c) {
    if (c->links) return hipSuccess;
    hipError_t e = dmalloc(c->stream, (void**)&c->links, (size_t)c->N * sizeof(uint32_t));
    if (e != hipSuccess) return e;
    const Launch L = node_launch(c);
    if (c->Q == 27)
        hipLaunchKernelGGL(k_build_links<27>, L.grid, L.block, 0, c->stream, c->links, c->solid, grid_of(c));
    else
        hipLaunchKernelGGL(k_build_links<19>, L.grid, L.block, 0, c->stream, c->links, c->solid, grid_of(c));
    return hipGetLastError();
}

static void free_all(lbm_ctx* c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) {
        for (void* b : c->f) dfree(c->stream, b);
        dfree(c->stream, c->psi);
        dfree(c->stream, c->solid);
        dfree(c->stream, c->links);
        dfree(c->stream, c->mom);
        dfree(c->stream, c->partial);
        dfree(c->stream, c->dtot);
        (void)hipStreamSynchronize(c->stream);      // this lattice's work only
    }
    if (c->hhealth) (void)hipHostFree(c->hhealth);
    if (c->health_ev) (void)hipEventDestroy(c->health_ev);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

extern "C" lbm_status lbm_create(const lbm_params* pp, lbm_ctx** out) {
    if (!pp || !out) return fail(nullptr, LBM_EINVAL, "null argument");
    *out = nullptr;
    lbm_status st = validate(*pp);
    if (st != LBM_OK) return st;
    double rv, rl;
    if (lbm_coexistence(pp, &rv, &rl) != LBM_OK)
        return fail(nullptr, LBM_EINVAL, "equation of state has no two-phase region");
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(nullptr, LBM_ENOMEM, "host allocation failed");
    c->p = *pp;
    c->Q = pp->lattice;
    c->N = (long long)pp->nx * pp->ny * pp->nz;
    c->stride = plane_stride(c->N);
    c->elem = storage_bytes(pp->storage);
    c->pd = make_phys<double>(*pp);
    c->pf = make_phys<float>(*pp);
    c->addr64 = pp->step_kernel == LBM_STEP_FUSED && needs_addr64(*pp);
    c->fused_cfg = default_fused_cfg(c);
    auto bail = [&](lbm_status s) { g_create_error = c->err; free_all(c); delete c; return s; };
#define CHK(call) do { hipError_t e_ = (call); if (e_ != hipSuccess) {                     \
        fail(c, e_ == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE, "%s failed: %s", #call, \
             hipGetErrorString(e_));                                                      \
        return bail(e_ == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE); } } while (0)
    if (count_fluid(*pp, c->any_solid) == 0) {       // host-only: before any device call
        fail(c, LBM_EINVAL, "geometry leaves no fluid node");
        return bail(LBM_EINVAL);
    }
    CHK(hipGetDevice(&c->device));
    CHK(hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, c->device));
    if (c->device >= kMaxDevices) {
        fail(c, LBM_EINVAL, "device index %d above %d", c->device, kMaxDevices - 1);
        return bail(LBM_EINVAL);
    }
    CHK(ensure_scratch(c->device));
    if (pp->stream) c->stream = (hipStream_t)pp->stream;
    else { CHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)); c->own_stream = true; }
    const size_t fbytes = (size_t)c->Q * c->stride * c->elem;
    CHK(dmalloc(c->stream, &c->f[0], fbytes));
    CHK(dmalloc(c->stream, &c->f[1], fbytes));
    CHK(hipMemsetAsync(c->f[0], 0, fbytes, c->stream));
    CHK(hipMemsetAsync(c->f[1], 0, fbytes, c->stream));
    CHK(dmalloc(c->stream, &c->psi, (size_t)c->N * (pp->storage == LBM_FP64 ? 8 : 4)));
    CHK(dmalloc(c->stream, (void**)&c->solid, (size_t)c->N));
    {
        const Launch L = node_launch(c);
        hipLaunchKernelGGL(k_build_solid, L.grid, L.block, 0, c->stream, c->solid, grid_of(c),
                           pp->cylinder, pp->cyl_y, pp->cyl_z, pp->cyl_r);
        CHK(hipGetLastError());
    }
    if (geom_of(c) == GEOM_MASK) CHK(build_links(c));
    if (c->elem != 8 && c->any_solid) solid_free_range(c->p, c->sf0, c->sf1);
    CHK(dmalloc(c->stream, (void**)&c->dtot, 8 * sizeof(double)));
    CHK(hipHostMalloc((void**)&c->hhealth, 2 * sizeof(double), hipHostMallocDefault));
    CHK(hipEventCreateWithFlags(&c->health_ev, hipEventDisableTiming));
#undef CHK
    *out = c;
    return LBM_OK;
}

extern "C" lbm_status lbm_destroy(lbm_ctx* c) {
    if (!c) return LBM_OK;
    free_all(c);
    delete c;
    return LBM_OK;
}

extern "C" const char* lbm_last_error(const lbm_ctx* c) {
    return c ? c->err.c_str() : g_create_error.c_str();
}

extern "C" int64_t lbm_steps_done(const lbm_ctx* c) { return c ? c->steps : -1; }

static lbm_status ensure_partial(lbm_ctx* c, long long n) {
    if (c->partial_cap >= n) return LBM_OK;
    dfree(c->stream, c->partial);
    c->partial = nullptr;
    HIPCHK(c, dmalloc(c->stream, (void**)&c->partial, (size_t)n * sizeof(double)));
    c->partial_cap = n;
    return LBM_OK;
}

template <template <int, typename> class Fn, typename... A>
static lbm_status dispatch(lbm_ctx* c, A... args) {
    if (c->Q == 19) {
        if (c->p.storage == LBM_FP64) return Fn<19, double>::run(c, args...);
        if (c->p.storage == LBM_FP32) return Fn<19, float>::run(c, args...);
        return Fn<19, _Float16>::run(c, args...);
    }
    if (c->p.storage == LBM_FP64) return Fn<27, double>::run(c, args...);
    if (c->p.storage == LBM_FP32) return Fn<27, float>::run(c, args...);
    return Fn<27, _Float16>::run(c, args...);
}

// Optional per-kernel timing of a step: an event pair around each launch.
struct KernelTimer {
    static constexpr int kMax = 4;
    hipEvent_t ev[2 * kMax];
    double total_ms[kMax];
    int nk = 0;
};
static const char* const kTwoPassNames[] = {"k_density_psi", "k_collide"};
static const char* const kFusedNames[] = {"k_step_fused"};

extern "C" lbm_status lbm_fused_plan(const lbm_params* p, int32_t cus, lbm_fused_plan_t* out) {
    if (!p || !out) return fail(nullptr, LBM_EINVAL, "null argument");
    if (cus < 1) return fail(nullptr, LBM_EINVAL, "cus must be >= 1");
    const lbm_status st = validate(*p);
    if (st != LBM_OK) return st;
    const int elem = (int)storage_bytes(p->storage), Q = p->lattice;
    const bool addr64 = needs_addr64(*p);
    const int cfg = fused_cfg_for(p->nx, elem, Q, addr64, p->cylinder != 0);
    const FusedCfg& f = kFusedCfgs[cfg];
    const FusedPlan pl = fused_plan(*p, elem, cfg, cus);
    out->config = cfg;
    out->tile_x = f.tx;
    out->tile_y = f.ty;
    out->full_rows = f.fullx ? 1 : 0;
    out->prefetch = fused_prefetch_fits(f, Q, elem) ? 1 : 0;
    out->z_chunk = pl.zc;
    out->xcd_order = pl.remap;
    out->hints = addr64 ? (pl.hints & ~kHintNtStore) : pl.hints;
    out->addr64 = addr64 ? 1 : 0;
    int sf0 = 0, sf1 = 0;
    bool any_solid = p->cylinder != 0;
    for (int a = 0; a < 3; ++a)
        any_solid = any_solid || p->bc[a][0] == LBM_BC_WALL || p->bc[a][1] == LBM_BC_WALL;
    if (elem != 8 && any_solid) solid_free_range(*p, sf0, sf1);
    out->solid_free_lo = sf0;
    out->solid_free_hi = sf1;
    out->workgroups = pl.workgroups;
    return LBM_OK;
}

// Calls f(geometry, store hint) with both as compile-time constants (std::integral_constant):

// One time step of the context's schedule (fused, or the two passes) from the current
// buffer into the other, with an event pair around each kernel when timed.
template <int Q, typename T>
struct StepFn {
    static lbm_status run(lbm_ctx* c, int64_t nsteps, KernelTimer* tm) {
        const bool fused = c->p.step_kernel == LBM_STEP_FUSED;
        for (int64_t s = 0; s < nsteps; ++s) {
            if (tm) HIPCHK(c, hipEventRecord(tm->ev[0], c->stream));
            if (fused) {
                StepOps<Q, T>::fused(c, c->f[c->cur], c->f[1 - c->cur]);
                if (tm) HIPCHK(c, hipEventRecord(tm->ev[1], c->stream));
                if (tm) tm->nk = 1;
            } else {
                StepOps<Q, T>::psi(c, c->f[c->cur]);
                if (tm) HIPCHK(c, hipEventRecord(tm->ev[1], c->stream));
                if (tm) HIPCHK(c, hipEventRecord(tm->ev[2], c->stream));
                StepOps<Q, T>::collide(c, c->f[c->cur], c->f[1 - c->cur]);
                if (tm) HIPCHK(c, hipEventRecord(tm->ev[3], c->stream));
                if (tm) tm->nk = 2;
            }
            if (tm) {
                HIPCHK(c, hipEventSynchronize(tm->ev[2 * tm->nk - 1]));
                for (int k = 0; k < tm->nk; ++k) {
                    float ms = 0.f;
                    HIPCHK(c, hipEventElapsedTime(&ms, tm->ev[2 * k], tm->ev[2 * k + 1]));
                    tm->total_ms[k] += ms;
                }
            }
            c->cur = 1 - c->cur;
            c->steps++;
        }
        HIPCHK(c, hipGetLastError());
        return LBM_OK;
    }
};

// Health check of the current state (k_health over the fluid nodes of the solid mask, then
// one block), its result copied to pinned host memory and marked by health_ev; read by
// poll_health.
template <int Q, typename T>
struct HealthFn {
    static lbm_status run(lbm_ctx* c) {
        const Launch L = node_launch(c);
        lbm_status st = ensure_partial(c, 2 * nblocks(L));
        if (st != LBM_OK) return st;
        hipLaunchKernelGGL((k_health<Q, T>), L.grid, L.block, 0, c->stream,
                           (const T*)c->f[c->cur], c->solid, c->partial, grid_of(c), c->p.rho_ref);
        hipLaunchKernelGGL(k_health_final, dim3(1), dim3(256), 0, c->stream, c->partial,
                           nblocks(L), c->dtot + 5);
        HIPCHK(c, hipGetLastError());
        HIPCHK(c, hipMemcpyAsync(c->hhealth, c->dtot + 5, 2 * sizeof(double),
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipEventRecord(c->health_ev, c->stream));
        c->health_pending = true;
        return LBM_OK;
    }
};

lbm_status enqueue_health(lbm_ctx* c) { return dispatch<HealthFn>(c); }

// Read the last health check if it has completed (wait = block until it has).
static lbm_status poll_health(lbm_ctx* c, bool wait) {
    if (!c->health_pending) return LBM_OK;
    if (wait) HIPCHK(c, hipEventSynchronize(c->health_ev));
    else if (hipEventQuery(c->health_ev) != hipSuccess) return LBM_OK;
    c->health_pending = false;
    if (c->hhealth[1] != 0.0 || !(c->hhealth[0] > 0.0)) {
        c->failed = true;
        return fail(c, LBM_ENONFINITE, "non-finite or non-positive density detected (min rho %g)",
                    c->hhealth[0]);
    }
    return LBM_OK;
}

// nsteps steps, with a health check after every step whose count is a multiple of
// reduce_every (if > 0).
static lbm_status run_steps(lbm_ctx* c, int64_t nsteps, KernelTimer* tm) {
    const int64_t every = c->p.reduce_every;
    while (nsteps > 0) {
        int64_t n = nsteps;
        if (every > 0) n = std::min<int64_t>(n, every - c->steps % every);
        lbm_status st = dispatch<StepFn>(c, n, tm);
        if (st != LBM_OK) return st;
        nsteps -= n;
        if (every > 0 && c->steps % every == 0) {
            st = enqueue_health(c);
            if (st != LBM_OK) return st;
        }
    }
    return LBM_OK;
}

extern "C" lbm_status lbm_step(lbm_ctx* c, int64_t nsteps) {
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (nsteps < 0) return fail(c, LBM_EINVAL, "nsteps must be >= 0");
    if (!c->initialised) return fail(c, LBM_ESTATE, "populations not initialised");
    if (c->failed) return fail(c, LBM_ESTATE, "a previous health check failed");
    HIPCHK(c, hipSetDevice(c->device));
    lbm_status st = poll_health(c, false);
    if (st != LBM_OK) return st;
    return run_steps(c, nsteps, nullptr);
}

extern "C" lbm_status lbm_health_status(lbm_ctx* c, int32_t wait) {
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (c->failed) return fail(c, LBM_ENONFINITE, "a previous health check failed");
    HIPCHK(c, hipSetDevice(c->device));
    return poll_health(c, wait != 0);
}

extern "C" lbm_status lbm_kernel_times(lbm_ctx* c, int64_t nsteps, double* avg_ms,
                                       const char** names, int32_t cap, int32_t* count) {
    if (!c || !avg_ms || !count || cap < 1) return fail(c, LBM_EINVAL, "null argument");
    if (nsteps < 1) return fail(c, LBM_EINVAL, "nsteps must be >= 1");
    if (!c->initialised) return fail(c, LBM_ESTATE, "populations not initialised");
    if (c->failed) return fail(c, LBM_ESTATE, "a previous health check failed");
    HIPCHK(c, hipSetDevice(c->device));
    KernelTimer tm{};
    for (int k = 0; k < 2 * KernelTimer::kMax; ++k) HIPCHK(c, hipEventCreate(&tm.ev[k]));
    lbm_status st = run_steps(c, nsteps, &tm);
    for (int k = 0; k < 2 * KernelTimer::kMax; ++k) (void)hipEventDestroy(tm.ev[k]);
    if (st != LBM_OK) return st;
    const int n = std::min<int>(tm.nk, cap);
    for (int k = 0; k < n; ++k) {
        avg_ms[k] = tm.total_ms[k] / (double)nsteps;
        if (names) names[k] = c->p.step_kernel == LBM_STEP_FUSED ? kFusedNames[k] : kTwoPassNames[k];
    }
    *count = n;
    return LBM_OK;
}

extern "C" lbm_status lbm_synchronize(lbm_ctx* c) {
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    HIPCHK(c, hipSetDevice(c->device));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return poll_health(c, true);
}

// ---------------------------------------------------------------------------------------
template <int Q, typename T>
struct InitFieldsFn {
    static lbm_status run(lbm_ctx* c, const double* drho, const double* du) {
        using R = typename Arith<T>::type;
        const Launch L = node_launch(c);
        const Phys<R>& P = phys_of<R>(c);
        c->cur = 0;
        hipLaunchKernelGGL((k_init_fields<Q, T>), L.grid, L.block, 0, c->stream, drho, du,
                           (T*)c->f[0], c->solid, grid_of(c), P);
        HIPCHK(c, hipGetLastError());
        return LBM_OK;
    }
};

static lbm_status ensure_mom(lbm_ctx* c) {
    if (c->mom) return LBM_OK;
    HIPCHK(c, dmalloc(c->stream, (void**)&c->mom, (size_t)5 * c->N * sizeof(double)));
    return LBM_OK;
}

static void reset_state(lbm_ctx* c) {
    c->initialised = true;
    c->failed = false;
    c->health_pending = false;
    c->steps = 0;
}

extern "C" lbm_status lbm_init_droplet(lbm_ctx* c, double cx, double cy, double cz, double R,
                                       double W, double rho_in, double rho_out, double ux,
                                       double uy, double uz, double noise_amp, uint64_t seed) {
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (!(W > 0) || !(R >= 0) || !(rho_in > 0) || !(rho_out > 0) || rho_in == rho_out)
        return fail(c, LBM_EINVAL, "need W > 0, R >= 0, rho_in, rho_out > 0 and distinct");
    HIPCHK(c, hipSetDevice(c->device));
    lbm_status st = ensure_mom(c);
    if (st != LBM_OK) return st;
    const Launch L = node_launch(c);
    double* rho0 = c->mom;
    double* u0 = c->mom + c->N;
    hipLaunchKernelGGL(k_droplet_fields, L.grid, L.block, 0, c->stream, rho0, u0, grid_of(c), cx,
                       cy, cz, R, W, rho_in, rho_out, ux, uy, uz, noise_amp, seed);
    st = dispatch<InitFieldsFn>(c, (const double*)rho0, (const double*)u0);
    if (st != LBM_OK) return st;
    reset_state(c);
    return LBM_OK;
}

extern "C" lbm_status lbm_init_fields(lbm_ctx* c, const double* rho, const double* u) {
    if (!c || !rho) return fail(c, LBM_EINVAL, "null argument");
    HIPCHK(c, hipSetDevice(c->device));
    lbm_status st = ensure_mom(c);
    if (st != LBM_OK) return st;
    HIPCHK(c, hipMemcpyAsync(c->mom, rho, c->N * sizeof(double), hipMemcpyHostToDevice, c->stream));
    if (u) HIPCHK(c, hipMemcpyAsync(c->mom + c->N, u, 3 * c->N * sizeof(double), hipMemcpyHostToDevice, c->stream));
    st = dispatch<InitFieldsFn>(c, (const double*)c->mom, (const double*)(u ? c->mom + c->N : nullptr));
    if (st != LBM_OK) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    reset_state(c);
    return LBM_OK;
}

template <int Q, typename T>
struct PopFn {
    static lbm_status run(lbm_ctx* c, double* host, bool set) {
        double* dbuf = nullptr;
        const size_t bytes = (size_t)Q * c->N * sizeof(double);
        HIPCHK(c, dmalloc(c->stream, (void**)&dbuf, bytes));
        const Launch L = node_launch(c);
        hipError_t e = hipSuccess;
        if (set) {
            e = hipMemcpyAsync(dbuf, host, bytes, hipMemcpyHostToDevice, c->stream);
            if (e == hipSuccess) {
                c->cur = 0;
                hipLaunchKernelGGL((k_scatter<Q, T>), L.grid, L.block, 0, c->stream, dbuf,
                                   (T*)c->f[0], c->solid, grid_of(c), c->p.rho_ref);
                e = hipGetLastError();
            }
        } else {
            hipLaunchKernelGGL((k_gather_out<Q, T>), L.grid, L.block, 0, c->stream,
                               (const T*)c->f[c->cur], dbuf, c->solid, grid_of(c), c->p.rho_ref);
            e = hipGetLastError();
            if (e == hipSuccess) e = hipMemcpyAsync(host, dbuf, bytes, hipMemcpyDeviceToHost, c->stream);
        }
        dfree(c->stream, dbuf);
        hipError_t e2 = hipStreamSynchronize(c->stream);
        if (e != hipSuccess || e2 != hipSuccess)
            return fail(c, LBM_EDEVICE, "population transfer failed: %s",
                        hipGetErrorString(e != hipSuccess ? e : e2));
        return LBM_OK;
    }
};

extern "C" lbm_status lbm_set_populations(lbm_ctx* c, const double* f) {
    if (!c || !f) return fail(c, LBM_EINVAL, "null argument");
    HIPCHK(c, hipSetDevice(c->device));
    lbm_status st = dispatch<PopFn>(c, const_cast<double*>(f), true);
    if (st == LBM_OK) reset_state(c);
    return st;
}

extern "C" lbm_status lbm_get_populations(lbm_ctx* c, double* f) {
    if (!c || !f) return fail(c, LBM_EINVAL, "null argument");
    if (!c->initialised) return fail(c, LBM_ESTATE, "populations not initialised");
    HIPCHK(c, hipSetDevice(c->device));
    return dispatch<PopFn>(c, f, false);
}

template <int Q, typename T>
struct MomentsFn {
    static lbm_status run(lbm_ctx* c, double* rho, double* u, double* p, double* totals) {
        using R = typename Arith<T>::type;
        lbm_status st = ensure_mom(c);
        if (st != LBM_OK) return st;
        const Launch L = node_launch(c);
        st = ensure_partial(c, 5 * nblocks(L));
        if (st != LBM_OK) return st;
        const Phys<R>& P = phys_of<R>(c);
        StepOps<Q, T>::psi(c, c->f[c->cur]);
        double* drho = c->mom;
        double* du = c->mom + c->N;
        double* dp = c->mom + 4 * c->N;
        hipLaunchKernelGGL((k_moments<Q, T>), L.grid, L.block, 0, c->stream,
                           (const T*)c->f[c->cur], (const R*)c->psi, drho, du, dp, c->partial,
                           grid_of(c), P);
        hipLaunchKernelGGL(k_sum_rows<5>, dim3(1), dim3(256), 0, c->stream, c->partial,
                           nblocks(L), c->dtot);
        HIPCHK(c, hipGetLastError());
        const size_t nb = c->N * sizeof(double);
        if (rho) HIPCHK(c, hipMemcpyAsync(rho, drho, nb, hipMemcpyDeviceToHost, c->stream));
        if (u) HIPCHK(c, hipMemcpyAsync(u, du, 3 * nb, hipMemcpyDeviceToHost, c->stream));
        if (p) HIPCHK(c, hipMemcpyAsync(p, dp, nb, hipMemcpyDeviceToHost, c->stream));
        if (totals) HIPCHK(c, hipMemcpyAsync(totals, c->dtot, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return LBM_OK;
    }
};

extern "C" lbm_status lbm_moments(lbm_ctx* c, double* rho, double* u, double* p, double* totals) {
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (!c->initialised) return fail(c, LBM_ESTATE, "populations not initialised");
    HIPCHK(c, hipSetDevice(c->device));
    lbm_status st = dispatch<MomentsFn>(c, rho, u, p, totals);
    if (st != LBM_OK) return st;
    return poll_health(c, true);
}

// The five totals of lbm_moments into a caller-owned device array, with the per-block
// partial sums in the device scratch (no allocation, no synchronisation).
template <int Q, typename T>
struct TotalsNoAllocFn {
    static lbm_status run(lbm_ctx* c, double* scratch_ptr, double* totals_dev) {
        using R = typename Arith<T>::type;
        const long long blocks = std::min<long long>(kTotalsBlocks, (c->N + 255) / 256);
        StepOps<Q, T>::psi(c, c->f[c->cur]);
        hipLaunchKernelGGL((k_totals<Q, T>), dim3((unsigned)blocks), dim3(256), 0, c->stream,
                           (const T*)c->f[c->cur], (const R*)c->psi, scratch_ptr, grid_of(c),
                           phys_of<R>(c));
        hipLaunchKernelGGL(k_sum_rows<5>, dim3(1), dim3(256), 0, c->stream, scratch_ptr, blocks,
                           totals_dev);
        HIPCHK(c, hipGetLastError());
        return LBM_OK;
    }
};

extern "C" lbm_status lbm_totals_noalloc(lbm_ctx* c, double* totals_dev) {
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (!totals_dev) return fail(c, LBM_EINVAL, "null totals_dev");
    if (!c->initialised) return fail(c, LBM_ESTATE, "populations not initialised");
    HIPCHK(c, hipSetDevice(c->device));
    double* ptr = scratch_of(c->device);
    if (!ptr) return fail(c, LBM_EDEVICE, "device scratch of device %d not set up", c->device);
    return dispatch<TotalsNoAllocFn>(c, ptr, totals_dev);
}

template <int Q, typename T>
struct LiquidFn {
    static lbm_status run(lbm_ctx* c, double threshold, double rho_v, double rho_l, int reach,
                          int64_t* count_z, int64_t* wetted_z, double* volume) {
        using R = typename Arith<T>::type;
        const Launch L = node_launch(c);
        const long long nb = nblocks(L), nz = c->p.nz;
        const long long per_plane = (long long)L.grid.x * L.grid.y;   // blocks of one z plane
        lbm_status st = ensure_partial(c, 3 * nb + 3 * nz + 3);
        if (st != LBM_OK) return st;
        double* plane = c->partial + 3 * nb;       // nz rows: liquid, in contact, volume
        double* tot = plane + 3 * nz;
        const Phys<R>& P = phys_of<R>(c);
        StepOps<Q, T>::psi(c, c->f[c->cur]);
        hipLaunchKernelGGL((k_liquid_stats<Q, T>), L.grid, L.block, 0, c->stream,
                           (const T*)c->f[c->cur], (const R*)c->psi, c->partial, grid_of(c),
                           P.rho_ref, threshold, rho_v, rho_l, reach);
        hipLaunchKernelGGL(k_sum_rows<3>, dim3((unsigned)nz), dim3(256), 0, c->stream,
                           c->partial, per_plane, plane);
        hipLaunchKernelGGL(k_sum_rows<3>, dim3(1), dim3(256), 0, c->stream, plane, nz, tot);
        HIPCHK(c, hipGetLastError());
        std::vector<double> h((size_t)(3 * nz + 3));
        HIPCHK(c, hipMemcpyAsync(h.data(), plane, h.size() * sizeof(double),
                                 hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (count_z)
            for (long long k = 0; k < nz; ++k) count_z[k] = (int64_t)h[(size_t)(3 * k)];
        if (wetted_z)
            for (long long k = 0; k < nz; ++k) wetted_z[k] = (int64_t)h[(size_t)(3 * k + 1)];
        if (volume) *volume = h[(size_t)(3 * nz + 2)];
        return LBM_OK;
    }
};

extern "C" lbm_status lbm_liquid_stats(lbm_ctx* c, double threshold, double rho_v, double rho_l,
                                       int32_t reach, int64_t* count_z, int64_t* wetted_z,
                                       double* volume) {
    if (!c) return fail(nullptr, LBM_EINVAL, "null context");
    if (!c->initialised) return fail(c, LBM_ESTATE, "populations not initialised");
    if (!(rho_l > rho_v) || !std::isfinite(rho_l) || !std::isfinite(rho_v) || !std::isfinite(threshold))
        return fail(c, LBM_EINVAL, "need finite threshold and rho_l > rho_v");
    if (reach < 1 || reach > 8) return fail(c, LBM_EINVAL, "reach must be in [1, 8]");
    HIPCHK(c, hipSetDevice(c->device));
    lbm_status st = dispatch<LiquidFn>(c, threshold, rho_v, rho_l, (int)reach, count_z,
                                       wetted_z, volume);
    if (st != LBM_OK) return st;
    return poll_health(c, true);
}

extern "C" lbm_status lbm_copy_bandwidth(int64_t bytes, int32_t reps, double* gbs) {
    if (!gbs || bytes < 16 * 1024 || reps < 1) return LBM_EINVAL;
    const long long n = bytes / 16;
    void *a = nullptr, *b = nullptr;
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    lbm_status st = LBM_OK;
    auto ok = [&](hipError_t e) {
        if (e != hipSuccess && st == LBM_OK) st = e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EDEVICE;
        return st == LBM_OK;
    };
    if (ok(hipStreamCreateWithFlags(&s, hipStreamNonBlocking)) && ok(hipMalloc(&a, n * 16)) &&
        ok(hipMalloc(&b, n * 16)) && ok(hipMemsetAsync(a, 0, n * 16, s)) &&
        ok(hipEventCreate(&e0)) && ok(hipEventCreate(&e1))) {
        const dim3 grid(1024), block(256);      // 4 waves per CU slot: the best of a sweep
        hipLaunchKernelGGL(k_copy_stream, grid, block, 0, s, (const lbm_f4*)a, (lbm_f4*)b, n);
        if (ok(hipGetLastError()) && ok(hipEventRecord(e0, s))) {
            for (int r = 0; r < reps; ++r)
                hipLaunchKernelGGL(k_copy_stream, grid, block, 0, s, (const lbm_f4*)a, (lbm_f4*)b, n);
            float ms = 0;
            if (ok(hipGetLastError()) && ok(hipEventRecord(e1, s)) && ok(hipEventSynchronize(e1)) &&
                ok(hipEventElapsedTime(&ms, e0, e1)))
                *gbs = 2.0 * 16.0 * (double)n * reps / (ms * 1e-3) / 1e9;
        }
    }
    if (s) (void)hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (a) (void)hipFree(a);
    if (b) (void)hipFree(b);
    if (s) (void)hipStreamDestroy(s);
    return st;
}
