/*
 * phonon_lbm.h -- C ABI of the MI355X (gfx950) phonon lattice Boltzmann library.
 *
 * The library advances the D2Q8 lattice Boltzmann equation for phonon
 * transport under Callaway's dual relaxation model (Guo & Wang, "Lattice
 * Boltzmann scheme for hydrodynamic equation of phonon transport", Sec. 2):
 *
 *   e_i(x + c_i, t + 1) - e_i(x, t) = (e_i^eq - e_i) / tau + S_i      (Eq. 13)
 *
 * with the eight velocities of Eq. 14 (no rest population), the drifting
 * equilibrium of Eq. 15, the resistive source of Eq. 16 with the weights of
 * Eqs. 17-18, tau = tau_C + 1/2 (Eq. 49), the moments of Eqs. 53-54, and the
 * boundary treatments of Sec. 2.5 (Eqs. 55, 58, 59-60).  Units are lattice
 * units: dx = dt = c = 1 (so the group speed is sqrt(5/3), Eq. 48).
 *
 * Directions are numbered as in the paper: 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1)
 * 5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1); the +x movers {1,5,8} and -x movers
 * {3,6,7} are the sets of Eqs. 59-60.
 *
 * Conventions for every entry point:
 *   - returns an lbm_status (0 on success); no C++ exception crosses the ABI;
 *   - a failing call leaves a message readable with lbm_last_error(handle);
 *   - fields passed in or out are row-major (ny rows of nx values, x fastest);
 *   - host pointers are caller-owned and only read or written during the call;
 *   - device pointers (on_device != 0) must be device memory of the handle's
 *     device; the call enqueues work on the handle's stream and synchronises it
 *     before returning;
 *   - a handle is not thread-safe; distinct handles are independent.
 */
#ifndef PHONON_LBM_H
#define PHONON_LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_ctx* lbm_handle;

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,          /* bad argument: NULL, size, relaxation time, index */
    LBM_ENOMEM = -2,          /* device or host allocation failed */
    LBM_EHIP = -3,            /* a HIP runtime call failed (message says which) */
    LBM_ESTATE = -4,          /* call not valid in the handle's current state */
    LBM_EUNSUPPORTED = -5,    /* boundary combination the paper does not define */
    LBM_ENONFINITE = -6       /* a reduction found Inf/NaN (e.g. FP16 overflow) */
} lbm_status;

/* Storage type of the populations.  Arithmetic is FP32 in every case; what is
 * stored is the scaled deviation g_i = (e_i - R_i(x)) / s from a reference
 * state R: the equilibrium omega_i C_V T_ref(x) plus a uniform x-flux (and,
 * with the GRADIENT seam, the non-equilibrium share the ramp sustains).  With
 * check steps on, the reference flux follows the lattice's mean heat flux.
 *   F32, F16, BF16 : the eight g_i in that type (64 / 32 / 32 bytes per node
 *                    and step, read plus write).
 *   F16_SPLIT, BF16_SPLIT : the energy E = sum_i g_i in FP32 and the eight
 *                    non-equilibrium shares h_i = g_i - omega_i E (Eq. 17
 *                    weights) in 16 bits (40 bytes per node and step).  The
 *                    heat flux lives in the h_i alone, so it keeps 16-bit
 *                    precision relative to itself rather than to the energy;
 *                    one node per lane only (vec 1), CHUNKED layout only. */
typedef enum {
    LBM_F32 = 0,
    LBM_F16 = 1,
    LBM_BF16 = 2,
    LBM_F16_SPLIT = 3,
    LBM_BF16_SPLIT = 4
} lbm_storage;

/* Boundary kinds (Sec. 2.5), per axis.  Walls are the nodes 0 and n-1.
 *   PERIODIC   : wrap-around advection.
 *   ISOTHERMAL : wall nodes hold omega_i C_V T_s in all eight directions (Eq. 55).
 *   DIFFUSE    : adiabatic diffuse reflection; after advection the populations
 *                leaving the wall share the incident energy in proportion to
 *                omega_i (Eq. 58); the wall node then relaxes like any node.
 *   GRADIENT   : periodic temperature-gradient seam along x (Eqs. 59-60) with
 *                period nx and T_h - T_c = grad_x * nx; handled exactly as a
 *                periodic deviation from a reference state built on the ramp
 *                T_ref(x) = t0 - grad_x * x (with the non-equilibrium share
 *                the ramp sustains and a uniform flux), so the seam needs no
 *                branch and the stored values are the departures from it.
 *   HEATFLUX   : prescribed heat flux q_0 into the domain (Eq. 56): the
 *                populations leaving the wall share the incident energy plus
 *                q_0 (2 tau_r + 1)/(2 tau_r) in proportion to omega_i (Eq. 57),
 *                so the heat flux of the wall node is exactly q_0.  q_0 is set
 *                per wall with lbm_set_wall_flux (0 until then: DIFFUSE).
 * Each wall may take its own kind (lbm_instance.wall_bc).  Supported: walls on
 * one axis with the other PERIODIC (GRADIENT x only with non-isothermal y
 * walls); walls on both axes only when both x walls are ISOTHERMAL: the paper
 * leaves corner nodes undefined, and here the isothermal x walls own them
 * (enough for the square of Sec. 3.1.2).  Anything else: LBM_EUNSUPPORTED. */
typedef enum {
    LBM_BC_PERIODIC = 0,
    LBM_BC_ISOTHERMAL = 1,
    LBM_BC_DIFFUSE = 2,
    LBM_BC_GRADIENT = 3,
    LBM_BC_HEATFLUX = 4
} lbm_bc;

/* How lbm_step issues the per-step work of a multi-instance handle. */
typedef enum {
    LBM_SCHED_BATCHED = 0,       /* one launch per step covering every instance (default) */
    LBM_SCHED_PER_INSTANCE = 1,  /* one launch per instance per step (comparison baseline) */
    LBM_SCHED_GRAPH = 2          /* batched launches replayed from a captured hipGraph */
} lbm_schedule;

/* One independent lattice. */
typedef struct {
    int32_t nx, ny;        /* nodes, >= 2 each; wall nodes are 0 and n-1 */
    int32_t bc_x, bc_y;    /* lbm_bc */
    double tau_n;          /* tau_N / dt > 0 (normal scattering) */
    double tau_r;          /* tau_R / dt > 0, +inf allowed (resistive scattering) */
    double cv;             /* C_V > 0; 0 selects 1 */
    double t0;             /* reference temperature (at x = 0 for GRADIENT) */
    double grad_x;         /* GRADIENT only: temperature drop per node along +x */
    double t_wall[4];      /* ISOTHERMAL wall temperatures: x=0, x=nx-1, y=0, y=ny-1 */
    double scale;          /* storage scale s (a power of two), 0 = chosen at init */
    int32_t wall_bc[4];    /* per-wall kind (x=0, x=nx-1, y=0, y=ny-1) overriding the axis
                              kind: 0 = the axis kind, else ISOTHERMAL, DIFFUSE or HEATFLUX,
                              on a walled axis only */
} lbm_instance;

/* Device layout of the populations (both hold the same values; the choice
 * only changes where they sit in memory).
 *   PLANES : eight direction planes of ny rows, x contiguous, each row padded
 *            to 256 bytes and each plane followed by a 4 KB pad.
 *   CHUNKED: rows cut into 64-node segments; a segment stores its eight
 *            direction runs back to back (2 KB in FP32), so the eight loads of
 *            a wavefront read one contiguous region.
 *   AUTO   : CHUNKED. */
typedef enum { LBM_LAYOUT_AUTO = 0, LBM_LAYOUT_PLANES = 1, LBM_LAYOUT_CHUNKED = 2 } lbm_layout;

typedef struct {
    int32_t n_instances;         /* >= 1 */
    int32_t storage;             /* lbm_storage */
    int32_t check_interval;      /* K: FP64 residual/total reductions at steps K, 2K, ...;
                                    0 = 100; -1 = never; otherwise >= 2 */
    int32_t flags;               /* LBM_FLAG_* */
    const lbm_instance* inst;    /* n_instances entries, copied at create */
    void* stream;                /* hipStream_t to enqueue on; NULL = null stream */
    int32_t layout;              /* lbm_layout */
    uint32_t seed;               /* stream of the stochastic-rounding bits (any value) */
} lbm_config;

/* Do not allocate device memory at create: the caller provides it with lbm_bind
 * (for example a torch tensor), sized by lbm_required_bytes. */
#define LBM_FLAG_EXTERNAL_MEMORY 0x1

/* Round the stored populations stochastically instead of to nearest.  With
 * round-to-nearest a very smooth field can freeze: once the per-step change
 * of a population is below half a unit in the last place of its stored value,
 * every node rounds the same way (the rounded map reaches a spurious fixed
 * point).  Stochastic rounding picks the upper or lower neighbour with
 * probability proportional to distance, so the stored state is unbiased.  The
 * random bits are a counter-based hash of (column, row, step, direction, seed)
 * (a column hash combined with a row-and-step hash): runs are deterministic
 * and do not depend on launch shape or schedule.
 * FP32: the update is added exactly (two-sum) and the result rounded to one of
 * its two FP32 neighbours; FP16/BF16: random bits below the kept mantissa are
 * added before truncation.  Requires one node per lane (launch shape vec 1). */
#define LBM_FLAG_STOCHASTIC_ROUNDING 0x2

/* 16-bit storage: round every time step of a fused launch to the storage
 * type, as a stored step is, so that the populations do not depend on how
 * the steps are grouped into launches (the same bits as single steps).
 * Without it a fused launch keeps the results of all but its last step in
 * FP32 registers and rounds only the state it stores: one rounding to 16 bits
 * per launch instead of k, which makes the 16-bit kinds faster (six steps per
 * launch instead of four) and more accurate, and the results depend on the
 * launch plan (the steps per launch, the check interval and where lbm_step
 * calls end).  Readouts after such a launch replay it in full up to the FP64
 * moments of its last step, so they match what the launch computed.  No
 * effect on FP32 storage, whose rounding is its arithmetic. */
#define LBM_FLAG_ROUND_EVERY_STEP 0x4

/* Version string of the library. */
const char* lbm_version(void);

/* Message of the last failing call on this handle ("" if none).  With a NULL
 * handle: the last failure of lbm_create / lbm_required_bytes in this thread.
 * Valid until the next call on the handle. */
const char* lbm_last_error(lbm_handle h);

/* Device bytes a handle of this configuration needs (the two population
 * buffers and a third region that readouts rebuild the last time step in: a
 * population buffer, or for 16-bit storage without LBM_FLAG_ROUND_EVERY_STEP
 * at least 24 bytes per node of FP64 moments; the residual snapshot,
 * reduction partials, tables). */
int lbm_required_bytes(const lbm_config* cfg, size_t* bytes);

/* Validate cfg, compute per-instance coefficients (Eqs. 49, 54, 16) and the
 * tile schedule, and (unless LBM_FLAG_EXTERNAL_MEMORY) allocate device memory.
 * *out is set only on success.  Errors: EINVAL (sizes, tau <= 0, bad enum,
 * check_interval), EUNSUPPORTED (boundary pair), ENOMEM, EHIP. */
int lbm_create(const lbm_config* cfg, lbm_handle* out);

/* Attach caller-owned device memory of at least lbm_required_bytes bytes,
 * 256-byte aligned.  Borrowed for the handle's lifetime, never freed by the
 * library.  Only for handles created with LBM_FLAG_EXTERNAL_MEMORY, before
 * lbm_init.  Errors: EINVAL, ESTATE. */
int lbm_bind(lbm_handle h, void* device_buf, size_t bytes);

/* Initialise instance `inst` at time n = 0 to the equilibrium of Eq. 15 for
 * temperature T and heat flux (qx, qy): e_i = omega_i C_V T + (5 a_i / 3)
 * c_i . (q / beta), beta = 2 tau_r / (2 tau_r + 1), so that Eq. 54 read back
 * at n = 0 returns q.  Isothermal wall nodes take their wall equilibrium
 * (Eq. 55).  T, qx, qy: host FP64 arrays of ny*nx; T NULL = T_ref (t0, or the
 * GRADIENT ramp); qx/qy NULL = 0.  With scale = 0 the storage scale becomes
 * s = 2^(ceil(log2 A) - 13) for FP16 (A = largest |T - T_ref|, |wall - T_ref|,
 * |q|; s = 1 if A = 0) and s = 1 for FP32/BF16.  All instances must be
 * initialised before lbm_step; re-initialising any instance resets the step
 * count of the handle to 0.  Errors: EINVAL, ESTATE (no memory bound), EHIP. */
int lbm_init(lbm_handle h, int32_t inst, const double* T, const double* qx, const double* qy);

/* As lbm_init with device FP64 arrays (same layout).  FP16 storage needs an
 * explicit scale (lbm_instance.scale != 0) here: EINVAL otherwise. */
int lbm_init_device(lbm_handle h, int32_t inst, const double* T, const double* qx,
                    const double* qy);

/* Enqueue nsteps time steps of every instance on the handle's stream (no host
 * synchronisation).  Each step, per node: pull the eight populations along
 * c_i (periodic wrap, the GRADIENT ramp term omega_i C_V grad_x c_ix / s),
 * apply the boundary treatment to the unknown ones, form E = sum g_i and
 * j = sum c_i g_i, and relax (Eq. 13 with Eqs. 15-16).  At every K-th step
 * the FP64 residual and totals of lbm_residual are formed (from the moments
 * of that step and the one before it).  Several steps may run in one launch
 * (lbm_set_step_fusion), the last ones of the call included; with FP32
 * storage, or with LBM_FLAG_ROUND_EVERY_STEP, the results do not depend on
 * how the steps are grouped (16-bit storage otherwise: see that flag).
 * Errors: EINVAL (nsteps < 0), ESTATE (not initialised), EHIP. */
int lbm_step(lbm_handle h, int64_t nsteps);

/* Steps taken since the last initialisation. */
int64_t lbm_steps_done(lbm_handle h);

/* Macroscopic fields of instance `inst` at the current time n (Eqs. 53-54):
 * T = T_ref + s E / C_V and q = s beta j of the post-advection, post-boundary
 * (pre-relaxation) populations, computed in FP64 and written as FP32.
 * on_device != 0: T, qx, qy are device pointers.  Any of them may be NULL. */
int lbm_moments(lbm_handle h, int32_t inst, float* T, float* qx, float* qy, int32_t on_device);

/* As lbm_moments in FP64, returning the deviation dT = T - T_ref(x) instead of
 * T (T_ref = t0, or the GRADIENT ramp), so that small deviations keep their
 * digits. */
int lbm_moments_f64(lbm_handle h, int32_t inst, double* dT, double* qx, double* qy,
                    int32_t on_device);

/* For callers that cannot allocate (code under HIP graph capture, serving
 * loops, harnesses that forbid hipMalloc): lbm_moments_f64 into HOST arrays
 * without any allocation.  lbm_moments_f64 with host outputs stages the fields
 * in a device buffer it allocates on first use; this variant stages them in a
 * fixed device array of the library (24 MiB per device, held until the
 * process ends; its address is resolved at lbm_create).  dT, qx, qy: host
 * arrays of ny*nx doubles (any may be NULL), as lbm_moments_f64.  The
 * instance may have at most 2^20 nodes: larger ones fail with LBM_EINVAL and
 * nothing is written.  Every call on one device shares the array: calls that
 * overlap on one device (other threads, other handles) race; a call is
 * complete when it returns (it synchronises the handle's stream).
 * Errors: EINVAL (index, size), ESTATE (not initialised), EUNSUPPORTED (the
 * array is not available on this device), EHIP. */
int lbm_moments_f64_noalloc(lbm_handle h, int32_t inst, double* dT, double* qx, double* qy);

/* FP64 totals of instance `inst` at the current time, computed now:
 * out[0] = sum (e - C_V T_ref) = C_V sum dT, out[1] = sum q_x, out[2] = sum q_y.
 * Errors: ENONFINITE if any total is not finite. */
int lbm_totals(lbm_handle h, int32_t inst, double out[3]);

/* Relative one-step residual of the last check step n (a multiple of K):
 * r = ||m^n - m^(n-1)||_2 / ||m^n||_2 over all nodes, m = (T - T_ref, q_x, q_y),
 * moments formed in FP64 from the stored populations.  r = 0 exactly means
 * the rounded map has reached a fixed point.  Synchronises the stream.
 * Errors: ESTATE (no check step yet), ENONFINITE (Inf/NaN in the reduction,
 * e.g. FP16 overflow). */
int lbm_residual(lbm_handle h, int32_t inst, double* r);

/* The whole last check record: step n, residual, and the FP64 totals of
 * lbm_totals taken at that step.  Same errors as lbm_residual. */
typedef struct {
    int64_t step;
    double residual;
    double totals[3];
} lbm_check_info;
int lbm_last_check(lbm_handle h, int32_t inst, lbm_check_info* out);

/* Coefficients the kernels use for instance `inst`, as doubles.  The
 * relaxation is applied in its eigen-decomposition: energy kept, heat-flux
 * share times rho, the rest times 1 - 1/tau (from Eqs. 13, 15, 16, 54).
 * out[0] = 1/tau (FP32-rounded), out[1] = beta (FP32-rounded),
 * out[2] = 1 - rho = 2/(2 tau_r + 1) (FP32-rounded), out[3] = s,
 * out[4] = tau (exact), out[5] = rho = (2 tau_r - 1)/(2 tau_r + 1) (exact). */
int lbm_coefficients(lbm_handle h, int32_t inst, double out[6]);

/* Heat flux q0 (energy per unit length and time step, lattice units) into the
 * domain through wall `wall` of instance `inst` (0: x = 0, 1: x = nx-1,
 * 2: y = 0, 3: y = ny-1), which must be a HEATFLUX wall (Eqs. 56-57).  It
 * applies to the steps enqueued after the call (the value is written by a
 * one-thread kernel on the handle's stream, so no synchronisation is needed
 * and captured graphs replay with the current value); it survives lbm_init.
 * Switching q0 to 0 after some steps gives the heat pulse of Sec. 3.4.
 * The automatic FP16 scale is taken from the initial field at lbm_init and
 * knows nothing of later wall fluxes: with a uniform start give the instance
 * an explicit scale (about the expected temperature rise / 2^11).
 * Errors: EINVAL (index, wall not HEATFLUX, non-finite q0), ESTATE (no memory). */
int lbm_set_wall_flux(lbm_handle h, int32_t inst, int32_t wall, double q0);

/* Most time steps per launch where allowed (temporal blocking, Eq. 13 applied
 * k times to a tile before its populations go back to HBM; the intermediate
 * states are rounded as stored steps are, with 16-bit storage only under
 * LBM_FLAG_ROUND_EVERY_STEP): a run of k >= 2 steps is advanced by one
 * launch; a run ends at the latest on a check step (whose residual and
 * totals the launch forms) or on the last step of an lbm_step call; 1 issues
 * every step on its own.  Moments read after a call that ended on such a run
 * are rebuilt by replaying it once (the same bits as the launch itself).
 * With FP32 storage or that flag the populations are identical for every
 * setting and the check-step residual and totals agree to the order of their
 * FP64 summation.  The most
 * steps per launch depends on the storage kind (7 FP32, 6 for the 16-bit
 * kinds, 4 for 16-bit handles with LBM_FLAG_ROUND_EVERY_STEP:
 * lbm_max_step_fusion gives the kind's most).  Default
 * for a new handle: that most when its instances hold at least 1024 strips of
 * the fused kernel in all (64 - 2 k columns by 32 rows each, k the most), so
 * that a fused launch fills the chip, else 1.  The per-instance schedule
 * always issues single steps.  Drops captured graphs.  Errors: EINVAL (steps
 * < 1 or more than the handle's most). */
int lbm_set_step_fusion(lbm_handle h, int32_t steps);

/* The current most time steps per launch; -1 for an invalid handle. */
int32_t lbm_get_step_fusion(lbm_handle h);

/* The most time steps one fused launch takes for storage kind `storage`
 * (lbm_storage; 16-bit handles with LBM_FLAG_ROUND_EVERY_STEP take at most
 * 4); -1 for an invalid kind.  Needs no device. */
int32_t lbm_max_step_fusion(int32_t storage);

/* Select how multi-instance steps are issued (lbm_schedule).  GRAPH captures
 * K batched steps (the check interval, or 64 when checks are off) once per
 * buffer parity and replays them; steps not filling a chunk run eagerly. */
int lbm_set_schedule(lbm_handle h, int32_t schedule);

/* Streams over which the BATCHED schedule spreads a handle's instances
 * (the batched launches of Sec. 3.2's parameter sweep): 1, or 2, which splits
 * the instances into two runs of consecutive instances holding about equal
 * numbers of fused-kernel strips and issues the second run's launches on a
 * stream the handle creates (default priority) at its first use; each
 * lbm_step call makes that stream wait for the work issued on the handle's
 * stream so far and makes the handle's stream wait for it before returning,
 * so later calls on the handle's stream see every step.  While one run's
 * launch drains its last wavefronts, the other run's launch fills the chip.
 * 0 restores the default: 2 for handles of two or more instances, else 1.
 * The GRAPH schedule captures the two parts as two branches of its graphs
 * (setting the streams drops captured graphs); PER_INSTANCE uses one stream.
 * Results are the same bits for every setting.  Errors: EINVAL (n outside
 * 0 .. 2). */
int lbm_set_streams(lbm_handle h, int32_t n);

/* Streams the batched schedule uses now (1 or 2); -1 for an invalid handle. */
int32_t lbm_get_streams(lbm_handle h);

/* Kernel launch shape: nodes per thread along x (1, 2 or 4), threads per
 * block along x (a multiple of 64, <= 512) and rows per block, with
 * block_x * block_y <= 512; xcd_remap != 0 maps consecutive tiles to the same
 * XCD.  Applies to later steps; invalidates captured graphs.  Errors: EINVAL. */
typedef struct {
    int32_t vec;
    int32_t block_x;
    int32_t block_y;
    int32_t xcd_remap;
    int32_t nontemporal;   /* != 0: streaming (non-temporal) population stores */
} lbm_launch_shape;
int lbm_set_launch_shape(lbm_handle h, const lbm_launch_shape* shape);
int lbm_get_launch_shape(lbm_handle h, lbm_launch_shape* shape);

/* Time every candidate launch shape on this handle's own instances and keep
 * the fastest, then time fused launches of every number of steps up to the
 * storage kind's most against it and set the steps per launch
 * (lbm_set_step_fusion) to the fastest.  Must be called after
 * lbm_create and before lbm_init (it runs steps on scratch contents); each
 * candidate is timed over `steps` steps (0 = 20) with HIP events.  If the environment variable LBM_AUTOTUNE_CACHE
 * names a file, a result for the same device, storage and instance shapes is
 * read from it instead of timing, and new results are appended to it.
 * report (may be NULL) receives a JSON summary of the timings.
 * Errors: ESTATE (already initialised), EHIP. */
int lbm_autotune(lbm_handle h, int32_t steps, char* report, size_t report_len);

/* Release device memory the library allocated and the handle itself.
 * Bound memory is not freed.  NULL is ignored. */
void lbm_destroy(lbm_handle h);

#ifdef __cplusplus
}
#endif

#endif /* PHONON_LBM_H */
