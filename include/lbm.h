/*
 * lbm.h - C ABI of the MI355X (gfx950) library for the fused time step of the
 * non-orthogonal multiple-relaxation-time lattice Boltzmann method with the
 * pseudopotential multiphase model of Fei, Du, Luo, Succi, Lauricella, Montessori and
 * Wang, "Modeling realistic multiphase flows using a non-orthogonal
 * multiple-relaxation-time lattice Boltzmann method" (arXiv 2306.16274).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Lattice units: dx = dt = c = 1, c_s^2 = 1/3 (Sec. II A).
 *  - A lattice of nx*ny*nz nodes is indexed n = x + nx*(y + ny*z) (x fastest).
 *  - Host arrays passed in or out are float64 and owned by the caller. Field arrays hold
 *    one value per node in that order; vector fields (u) are 3 planes of N values
 *    (u_x, u_y, u_z); population arrays are Q planes of N values in the velocity order
 *    of Eq. (1) (D3Q27) or Eq. (C1) (D3Q19: the first 19 of the D3Q27 list).
 *  - The context owns every device buffer it allocates. A stream given in lbm_params is
 *    borrowed (never destroyed); with stream == NULL the context creates its own.
 *  - Populations exchanged through lbm_set_populations / lbm_get_populations are the
 *    f_bar(x, t) of Sec. II A (after streaming, before collision): rho = sum_i f_bar_i and
 *    rho u = sum_i f_bar_i e_i + F/2 (Eq. (10)). Solid nodes carry no populations and
 *    read back as 0.
 *  - Every call returns an lbm_status; LBM_OK is 0. On error, lbm_last_error() returns
 *    a context-owned message (valid until the next call on that context).
 *  - Calls on one context are not thread-safe; distinct contexts are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx lbm_ctx;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,      /* bad argument or parameter (message says which)            */
    LBM_ENOMEM = -2,      /* device or pinned host allocation failed                   */
    LBM_EDEVICE = -3,     /* a HIP runtime call failed                                 */
    LBM_ENONFINITE = -4,  /* the periodic health check found a non-finite or negative
                             density; the state stays readable, further steps refused  */
    LBM_ESTATE = -5       /* call not allowed in the current state (e.g. step before
                             initialisation, or after LBM_ENONFINITE)                   */
} lbm_status;

enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16 = 2 };       /* population storage type   */
enum { LBM_EOS_CS = 0, LBM_EOS_PIECEWISE = 1 };          /* equation of state         */
enum { LBM_BC_PERIODIC = 0, LBM_BC_WALL = 1 };           /* per domain face           */
enum { LBM_STEP_FUSED = 0, LBM_STEP_TWO_PASS = 1 };      /* kernel schedule of a step */
enum { LBM_WALL_PSI_NODE = 0, LBM_WALL_PSI_FLUID_MEAN = 1,  /* psi at solid neighbours   */
       LBM_WALL_PSI_ZERO = 2, LBM_WALL_PSI_MIRROR = 3 };

/*
 * Problem statement. Defaults (lbm_params_default) follow Sec. II B: s0 = s1 = 1,
 * s2b = s3b = 0.6, all other non-viscous rates 1.2; G = -1 (Sec. III A); sigma = 0.1
 * (Sec. III A); kappa = 0; G_ads = 0 (neutral wall, Sec. III E).
 */
typedef struct {
    int32_t lattice;          /* 19 (D3Q19, Appendix C) or 27 (D3Q27, Sec. II A-B)        */
    int32_t storage;          /* LBM_FP64: stored and computed in float64.
                                 LBM_FP32 / LBM_FP16: stored as deviations
                                 f_i - w_i*rho_ref, computed in float32                 */
    int32_t nx, ny, nz;       /* lattice size, each >= 1                                 */
    int32_t eos;              /* LBM_EOS_CS or LBM_EOS_PIECEWISE                         */
    double rho_ref;           /* shift of the stored populations (0 = plain storage)     */
    /* Carnahan-Starling: p = rho R T (1+eta+eta^2-eta^3)/(1-eta)^3 - a rho^2,
       eta = b rho / 4, T = T_over_Tc * 0.3773 a / (b R)                                 */
    double cs_a, cs_b, cs_R, T_over_Tc;
    /* Piecewise-linear EOS, Eq. (18): slopes and the two spinodal densities             */
    double pw_theta_v, pw_theta_m, pw_theta_l, pw_rho1, pw_rho2;
    double G;                 /* interaction strength of Eq. (16)                        */
    double sigma;             /* mechanical-stability parameter of Eq. (B1); the paper's
                                 0.1 is for its piecewise EOS: with Carnahan-Starling
                                 (a = 0.5, b = 4) a flat interface settles on the Maxwell
                                 densities at 0.115-0.119 for 0.5-0.7 T_c               */
    double kappa;             /* surface-tension tuning of Eq. (B2)                      */
    double G_ads;             /* fluid-solid interaction strength of Eq. (22)            */
    double nu_l, nu_v;        /* kinematic viscosity; nu_v != nu_l enables Eq. (24)      */
    double rho_l, rho_v;      /* densities anchoring the linear nu(rho) of Eq. (24)      */
    double s0, s1, s2b, s3, s3b, s4, s4b, s5, s6;   /* rates of Eq. (12) / Eq. (C3);
                                 s_nu (s2) follows from nu: nu = (1/s_nu - 1/2)/3          */
    int32_t bc[3][2];         /* [axis x,y,z][lo,hi]: LBM_BC_WALL makes the node layer
                                 at index 0 (lo) or n-1 (hi) solid; neighbours always
                                 wrap periodically, so a wall-free axis is periodic     */
    int32_t cylinder;         /* nonzero: solid x-aligned cylinder                       */
    double cyl_y, cyl_z, cyl_r;   /* solid where (y-cyl_y)^2 + (z-cyl_z)^2 <= cyl_r^2    */
    double body_force[3];     /* uniform body force added to F (default 0)               */
    void* stream;             /* hipStream_t to enqueue on, or NULL                      */
    int32_t reduce_every;     /* health check cadence in steps (0 = never)               */
    int32_t step_kernel;      /* LBM_STEP_FUSED: one pass per step, rho/psi of a tile halo
                                 recomputed on chip (default). LBM_STEP_TWO_PASS: a
                                 density/psi pass, then the collision pass. Same results
                                 up to rounding order.                                    */
    int32_t wall_psi;         /* psi taken at a solid neighbour in F_int (Eq. (16)) and
                                 Q_ab (Eq. (B2)), which the paper leaves open:
                                 LBM_WALL_PSI_NODE (psi of the fluid node itself),
                                 LBM_WALL_PSI_FLUID_MEAN (sum w_i psi(x+e_i) / sum w_i over
                                 the fluid neighbours of x), LBM_WALL_PSI_ZERO or
                                 LBM_WALL_PSI_MIRROR (psi(x + e') with e' = e_i less every
                                 component along which the axis neighbour of x is solid:
                                 for a flat wall the mirror image of x + e_i across the
                                 wall; psi(x) where e' = 0 or x + e' is solid; the
                                 default: it makes G_ads = 0 neutral, 90 degrees, and
                                 G_ads = 0.23 give 157 degrees, as Sec. III E states). The
                                 wetting force of Eq. (22) is added in every case.         */
} lbm_params;

/* Fill *p with the defaults above (D3Q19, FP32, 64^3, CS EOS at T = 0.7 T_c, a = 0.5,
   b = 4, R = 1, nu = 0.1, fully periodic, rho_ref = 0, wall_psi = LBM_WALL_PSI_MIRROR).
   Returns LBM_EINVAL on NULL.                                                           */
lbm_status lbm_params_default(lbm_params* p);

/* Validate *p, allocate the lattice on the current HIP device and return a context in
   *out. Rejects (LBM_EINVAL, before any device call): lattice not 19/27, unknown storage,
   EOS, boundary condition or step kernel, sizes < 1 or beyond the launch grid, G >= 0,
   non-positive EOS constants, rates outside (0,2), nu <= 0, non-finite parameters, a
   cylinder radius <= 0, an EOS without a two-phase region, a geometry without fluid
   nodes, more than 2^31 - 1 nodes. The populations are
   undefined until one of the lbm_init_* / lbm_set_populations calls.                  */
lbm_status lbm_create(const lbm_params* p, lbm_ctx** out);

/* Free everything the context owns. NULL is accepted.                                 */
lbm_status lbm_destroy(lbm_ctx* c);

/* Message of the last failed call on c (or, if c == NULL, of the last failed lbm_create
   of the calling thread).                                                              */
const char* lbm_last_error(const lbm_ctx* c);

/* Initial state f_bar = M^-1 m^eq(rho0, u0) (Sec. II B) of a droplet centred at
   (cx, cy, cz) with radius R: rho0 = (rho_in+rho_out)/2 - (rho_in-rho_out)/2
   tanh(2 (r - R)/W), the radial form of the interface profile of Eq. (21). The velocity
   (ux, uy, uz) is carried by the liquid fraction clamp((rho0-rho_out)/(rho_in-rho_out),
   0, 1) of the noise-free profile. Inside |r - R| < W the density is multiplied by
   1 + noise_amp (2 U_n - 1), U_n the SplitMix64 uniform of node n under seed. Resets the
   step counter and the health flag. Asynchronous on the context stream.               */
lbm_status lbm_init_droplet(lbm_ctx* c, double cx, double cy, double cz, double R, double W,
                            double rho_in, double rho_out, double ux, double uy, double uz,
                            double noise_amp, uint64_t seed);

/* Initial state f_bar = M^-1 m^eq(rho, u) from host fields: rho (N values) and u
   (3 planes of N, or NULL for rest). Values at solid nodes are ignored. Synchronous.  */
lbm_status lbm_init_fields(lbm_ctx* c, const double* rho, const double* u);

/* Replace / read the state f_bar(x, t) (Q planes of N float64, host memory).
   Synchronous. Set rounds to the storage type.                                        */
lbm_status lbm_set_populations(lbm_ctx* c, const double* f);
lbm_status lbm_get_populations(lbm_ctx* c, double* f);

/* Advance nsteps time steps (Sec. II A: streaming with halfway bounce-back, rho and psi,
   F_int of Eq. (16), F_ads of Eq. (22), Q_ab of Eq. (B2), the moment-space collision of
   Eq. (8) with the forcing moments of Eq. (B1), f_bar* = M^-1 m*). Enqueues on the
   context stream and returns without waiting, except every reduce_every steps, where the
   result of the previous health check is read. nsteps >= 0.
   The launch configuration of the fused step (tile shape: full rows for nx = 256, 320 or
   384, else 64x8 or 64x4 tiles; z-chunk length; nontemporal hints) is chosen from the
   domain width, the storage type and the lattice; a population buffer of 4 GiB or more
   takes 64x8 (4-byte storage) or 64x4 tiles with 64-bit offsets and plain stores. On
   walled and cylinder lattices with 2- or 4-byte storage, the planes with no solid node
   within two planes run the arithmetic of a lattice without solid nodes (the same values
   for those nodes). For tuning, the environment variables LBM_FUSED_CONFIG, LBM_FUSED_ZC,
   LBM_FUSED_REMAP, LBM_FUSED_HINTS and LBM_SOLID_FREE (0: no solid-free planes) override
   this; every configuration gives the same populations (bitwise, up to the sign of exact
   zeros).                                                                              */
lbm_status lbm_step(lbm_ctx* c, int64_t nsteps);

/* Number of time steps taken since the last initialisation.                           */
int64_t lbm_steps_done(const lbm_ctx* c);

/* Macroscopic fields at the current time (after streaming, before collision):
   rho = sum f_bar, u = (sum f_bar e + F/2)/rho (Eq. (10)), p = rho/3 + G psi^2/2
   (Eq. (17)). Any output pointer may be NULL. totals (5 values) receives the float64
   sums over fluid nodes of rho, rho u_x, rho u_y, rho u_z and rho |u|^2 / 2. Solid nodes
   read 0. Synchronous.                                                                 */
lbm_status lbm_moments(lbm_ctx* c, double* rho, double* u, double* p, double* totals);

/* Totals without allocation, for callers that cannot allocate device memory (code under
   HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the five
   float64 totals of lbm_moments (sums over fluid nodes of rho, rho u_x, rho u_y, rho u_z
   and rho |u|^2 / 2, with u of Eq. (10)) written to totals_dev, a caller-owned DEVICE
   array of 5 doubles. Enqueued on the context stream; returns without waiting (order a
   read of totals_dev after the stream). Allocates nothing and copies nothing to the host:
   the partial sums of its reduction go to a fixed device scratch array of the library
   (1024 blocks x 5 doubles = 40 KiB per device, set up by the first lbm_create on that
   device and held until the process ends); the reduction runs at most 1024 blocks that
   stride over the lattice, so every lattice size fits. The summation tree differs from
   lbm_moments (rounding-level differences; fixed, so repeated calls agree bitwise).
   Every call on a device overwrites that device's scratch: calls that overlap on one
   device (different streams, not ordered by events) race and may return wrong totals.
   The psi buffer of the context is rewritten, as lbm_moments does.
   Errors: LBM_EINVAL for NULL arguments, LBM_ESTATE before initialisation, LBM_EDEVICE if
   the scratch of the device was not set up.                                            */
lbm_status lbm_totals_noalloc(lbm_ctx* c, double* totals_dev);

/* Liquid-phase diagnostics of the current state, reduced on the device: the spreading
   diameter of the film on a wall (Sec. IV A, from the liquid area of the first fluid
   layer), the contact time (Sec. IV B, the droplet has left the solid when no liquid node
   touches it) and the liquid volume (Sec. IV B). A fluid node is liquid when rho > threshold,
   with rho formed and compared in float64 exactly as lbm_moments returns it.
     count_z  NULL or nz int64: liquid nodes in each z plane (index k = plane z = k);
     wetted_z NULL or nz int64: liquid nodes of each z plane with a solid node at x + k e_i
              for some lattice velocity e_i and 1 <= k <= reach (reach 1: a solid neighbour;
              larger reach also counts liquid held off a hydrophobic wall by a thin vapour
              layer);
     volume   NULL or one double: sum over fluid nodes of clamp((rho - rho_v)/(rho_l - rho_v),
              0, 1), a fixed-order float64 sum.
   Errors: LBM_EINVAL unless rho_l > rho_v, all three are finite and 1 <= reach <= 8;
   LBM_ESTATE before initialisation. Synchronous.                                        */
lbm_status lbm_liquid_stats(lbm_ctx* c, double threshold, double rho_v, double rho_l,
                            int32_t reach, int64_t* count_z, int64_t* wetted_z, double* volume);

/* Measurement aid: run nsteps time steps (as lbm_step) with a HIP event pair around every
   kernel launch on the context stream, waiting after each step. avg_ms[k] receives the
   mean duration in ms of the k-th kernel of a step and names[k] (if names != NULL) its
   name (static strings); *count the number of kernels per step (at most cap).          */
lbm_status lbm_kernel_times(lbm_ctx* c, int64_t nsteps, double* avg_ms, const char** names,
                            int32_t cap, int32_t* count);

/* Measurement aid: attainable HBM bandwidth of a plain streaming copy on the current
   device (bytes read + bytes written per second, in GB/s), the practical ceiling for the
   step kernels. Allocates two buffers of `bytes` (>= 16 KiB) for the duration of the call,
   times `reps` copies with HIP events on a private stream. Synchronous.                 */
lbm_status lbm_copy_bandwidth(int64_t bytes, int32_t reps, double* gbs);

/* Result of the periodic health checks (reduce_every, and the checks after lbm_batch_run)
   without enqueueing anything: LBM_ENONFINITE if a completed check found a non-finite or
   non-positive density (now or earlier; the context then refuses further steps), else
   LBM_OK. wait = 0 does not block (a check still in flight counts as passed for now);
   wait != 0 waits for the last check enqueued. For a serving loop that evicts failed
   lattices without draining the device.                                                */
lbm_status lbm_health_status(lbm_ctx* c, int32_t wait);

/* Wait for all work enqueued on the context stream.                                   */
lbm_status lbm_synchronize(lbm_ctx* c);

/* Coexistence densities (Maxwell equal-area construction, the conditions of Eq. (19))
   of the equation of state described by *p. Host-only.                                 */
lbm_status lbm_coexistence(const lbm_params* p, double* rho_v, double* rho_l);

/* Device bytes a context created from *p allocates (for admission control), or -1.
   Includes the fused step's link words (4 bytes per node) when p has a cylinder; a batch
   that contains a cylinder lattice adds them to its other members as well.            */
int64_t lbm_footprint_bytes(const lbm_params* p);

/* Launch plan of the fused step (step_kernel = LBM_STEP_FUSED) for a lattice created from
   *p on a device with `cus` compute units (256 on MI355X): what lbm_step launches, chosen
   from the width, the storage type and the lattice, with the LBM_FUSED_* environment
   overrides applied as lbm_step applies them. Host-only. Errors: LBM_EINVAL for a NULL
   argument, cus < 1 or parameters lbm_create would reject.                              */
typedef struct {
    int32_t config;       /* launch configuration index (LBM_FUSED_CONFIG)                 */
    int32_t tile_x;       /* (x, y) columns of one workgroup: tile_x * tile_y threads       */
    int32_t tile_y;
    int32_t full_rows;    /* 1: a tile spans whole x rows (tile_x == nx)                    */
    int32_t prefetch;     /* 1: the planes ahead are loaded into LDS asynchronously        */
    int32_t z_chunk;      /* planes marched by one workgroup (LBM_FUSED_ZC)                 */
    int32_t xcd_order;    /* 1: tiles mapped to XCDs in contiguous ranges (LBM_FUSED_REMAP) */
    int32_t hints;        /* bit 0: nontemporal stores; bit 1: nontemporal interior loads  */
    int32_t addr64;       /* 1: 64-bit byte offsets (population buffer of 4 GiB or more)    */
    int32_t solid_free_lo; /* planes solid_free_lo .. solid_free_hi - 1 of a walled or      */
    int32_t solid_free_hi; /* cylinder lattice run the arithmetic of a lattice without solid
                              nodes (2- and 4-byte storage; LBM_SOLID_FREE); both 0 for FP64,
                              for lattices without solid nodes and where no plane qualifies */
    int64_t workgroups;   /* workgroups of one time step                                    */
} lbm_fused_plan_t;
lbm_status lbm_fused_plan(const lbm_params* p, int32_t cus, lbm_fused_plan_t* out);

/*
 * Batched stepping (serving many independent lattices). A batch holds a fixed set of
 * contexts (D3Q19, all FP32 or all FP64 storage, each initialised) and advances all of
 * them together: one kernel launch per time step covers the tiles of every member, and
 * steps_per_launch consecutive launches are captured once into a HIP graph. Each member
 * takes exactly the time step of lbm_step (the same populations: the per-node arithmetic
 * is shared). FP32 batches whose members are at most 384 nodes wide run row tiles (768
 * threads covering as many whole rows of a member as fit, each row wrapping in x, the next
 * plane prefetched into LDS) through 12-plane z-chunks, others 64x4 tiles through 16-plane
 * z-chunks; nontemporal stores when every member's rows are whole
 * 128-byte lines; workgroups mapped to XCDs in contiguous ranges. LBM_BATCH_ROWS,
 * LBM_BATCH_TILE, LBM_BATCH_ZC, LBM_BATCH_PF, LBM_BATCH_NT and LBM_BATCH_REMAP override
 * this for tuning.
 * The batch borrows the contexts (they must outlive it and must not be stepped on their
 * own while the batch runs); it orders its work after, and each member's later work
 * after, the batch's graph launches through events.
 */
typedef struct lbm_batch lbm_batch;

/* Build a batch of n distinct contexts. steps_per_launch: even, >= 2 (time steps per
   graph replay). stream: hipStream_t for the replays, or NULL for a batch-owned stream.
   Does not wait for the members' pending work (lbm_batch_run orders after it).
   Errors: LBM_EINVAL if a context is NULL or repeated, members differ in device or storage,
   a member is D3Q27, FP16 or has a population buffer of 4 GiB or more; LBM_ESTATE if a
   member is not initialised or failed its health check; LBM_EDEVICE / LBM_ENOMEM from the
   runtime (nothing is left allocated).                                                 */
lbm_status lbm_batch_create(lbm_ctx* const* ctxs, int32_t n, int32_t steps_per_launch,
                            void* stream, lbm_batch** out);

/* Advance every member by nlaunch * steps_per_launch time steps (asynchronous).        */
lbm_status lbm_batch_run(lbm_batch* b, int64_t nlaunch);

/* Release the batch (not the member contexts): waits for the batch's own replays only.
   NULL is accepted.                                                                     */
lbm_status lbm_batch_destroy(lbm_batch* b);

/* Message of the last failed lbm_batch_* call of the calling thread.                    */
const char* lbm_batch_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
