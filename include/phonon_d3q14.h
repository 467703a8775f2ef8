/*
 * phonon_d3q14.h -- C ABI of the three-dimensional (D3Q14) path of the MI355X
 * (gfx950) phonon lattice Boltzmann library (same shared library as
 * phonon_lbm.h).
 *
 * The paper (Guo & Wang, "Lattice Boltzmann scheme for hydrodynamic equation
 * of phonon transport") builds its scheme on the D2Q8 lattice and names the
 * three-dimensional D3Q14 lattice as a direct extension (Sec. 2.2) without
 * giving its weights.  This path keeps every equation of the scheme -- the
 * update of Eq. 13, the equilibrium of Eq. 15, the resistive source of Eq. 16,
 * the moments of Eqs. 53-54, c = sqrt(3/5) v_g (Eq. 48) and tau = tau_C/dt +
 * 1/2 (Eq. 49) -- on the 14 velocities
 *
 *     axis movers  (+-1, 0, 0), (0, +-1, 0), (0, 0, +-1)      (6)
 *     corner movers (+-1, +-1, +-1)                           (8)
 *
 * (no rest population), with the weights that make the moment identities of
 * the Chapman-Enskog analysis (Sec. 2.3, Eqs. 22-28) hold on this set, which
 * is what the recovery of the hydrodynamic equation (Eq. 47) uses:
 *
 *     omega_i = 1/9 (axis), 1/24 (corner)   (sum 1; second moment 5/9)
 *     a_i     = 1/5 (axis), 1/40 (corner)   (second moment 3/5; fourth
 *                                            moments 3/5 and 1/5)
 *
 * the unique solution of those conditions on this velocity set.  The box is
 * periodic on every axis (the paper's wall treatments are two-dimensional).
 * Units are lattice units: dx = dt = c = 1.
 *
 * Conventions are those of phonon_lbm.h: every entry point returns an
 * lbm_status (0 on success) and leaves a message for lbm3d_last_error on
 * failure; fields are (nz, ny, nx) arrays with x fastest; host pointers are
 * caller-owned and used only during the call; device pointers (on_device != 0)
 * must be memory of the handle's device; calls that read results synchronise
 * the handle's stream; a handle is not thread-safe.
 */
#ifndef PHONON_D3Q14_H
#define PHONON_D3Q14_H

#include <stddef.h>
#include <stdint.h>

#include "phonon_lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm3d_ctx* lbm3d_handle;

typedef struct {
    int32_t nx, ny, nz;     /* nodes per axis, >= 1 each, fewer than 2^32 nodes in all */
    int32_t storage;        /* LBM_F32, LBM_F16 or LBM_BF16 (the split kinds are D2Q8 only) */
    int32_t flags;          /* LBM_FLAG_EXTERNAL_MEMORY, LBM_FLAG_STOCHASTIC_ROUNDING,
                               LBM_FLAG_ROUND_EVERY_STEP */
    int32_t layout;         /* lbm_layout: PLANES = 14 direction planes (rows padded to 64
                               nodes); CHUNKED = 64-node row segments holding their 14
                               direction runs back to back; AUTO = CHUNKED */
    uint32_t seed;          /* stream of the stochastic-rounding bits */
    double tau_n;           /* tau_N / dt > 0 */
    double tau_r;           /* tau_R / dt > 0, +inf allowed */
    double cv;              /* C_V > 0; 0 selects 1 */
    double t0;              /* reference temperature of the stored deviations */
    double scale;           /* storage scale s (a power of two), 0 = chosen at init */
    void* stream;           /* hipStream_t to enqueue on; NULL = null stream */
} lbm3d_config;

/* Launch shape of the step kernel: a thread block covers a tile of
 * 64 * tile_waves consecutive nodes in each of rows_per_tile rows, one node per
 * thread (64 * tile_waves * rows_per_tile <= 512 threads). */
typedef struct {
    int32_t rows_per_tile;  /* 1, 2 or 4 */
    int32_t xcd_remap;      /* 1: each of the 8 XCDs takes one contiguous range of tiles */
    int32_t nontemporal;    /* 1: streaming stores */
    int32_t tile_waves;     /* 1, 2, 4 or 8 wavefronts (64-node segments) along x */
    int32_t zchunk;         /* two steps per launch: planes each block marches through (>= 1;
                               default 32) */
} lbm3d_launch_shape;

/* Message of the last failing call on this handle ("" if none); with NULL, the
 * last failure of lbm3d_create / lbm3d_required_bytes in this thread. */
const char* lbm3d_last_error(lbm3d_handle h);

/* Device bytes a handle of this configuration needs: two population buffers
 * (14 direction planes each) and the reduction scratch. */
int lbm3d_required_bytes(const lbm3d_config* cfg, size_t* bytes);

/* Validate cfg, compute the relaxation coefficients (Eqs. 49, 54, 16) and,
 * unless LBM_FLAG_EXTERNAL_MEMORY, allocate the device memory.  *out is set
 * only on success.  Errors: EINVAL (sizes, tau <= 0, storage, flags), ENOMEM,
 * EHIP. */
int lbm3d_create(const lbm3d_config* cfg, lbm3d_handle* out);

/* Attach caller-owned device memory of at least lbm3d_required_bytes bytes,
 * 256-byte aligned, borrowed for the handle's lifetime (never freed by the
 * library).  Only with LBM_FLAG_EXTERNAL_MEMORY, before lbm3d_init.
 * Errors: EINVAL, ESTATE. */
int lbm3d_bind(lbm3d_handle h, void* device_buf, size_t bytes);

/* Initialise at time n = 0 to the equilibrium of Eq. 15 for temperature T and
 * heat flux q: e_i = omega_i C_V T + (5 a_i / 3) c_i . (q / beta), beta =
 * 2 tau_r / (2 tau_r + 1), so that Eq. 54 read back at n = 0 returns q.  T,
 * qx, qy, qz: FP64 arrays of nz*ny*nx (device arrays if on_device != 0); T
 * NULL = t0, a NULL flux component = 0.  With scale = 0, s becomes
 * 2^(ceil(log2 A) - 13) for FP16 (A = largest |T - t0| and |q|; s = 1 if
 * A = 0; needs host arrays) and 1 for FP32/BF16.  Resets the step count.
 * Errors: EINVAL (FP16 with scale 0 and device arrays), ESTATE (no memory), EHIP. */
int lbm3d_init(lbm3d_handle h, const double* T, const double* qx, const double* qy, const double* qz,
               int32_t on_device);

/* Enqueue nsteps time steps on the handle's stream (no host synchronisation).
 * Each step, per node: pull the 14 populations along c_i (periodic wrap),
 * form E = sum g_i and J = sum c_i g_i, relax (Eq. 13 with Eqs. 15-16), store.
 * Errors: EINVAL (nsteps < 0), ESTATE (not initialised), EHIP. */
int lbm3d_step(lbm3d_handle h, int64_t nsteps);

/* Steps taken since the last initialisation. */
int64_t lbm3d_steps_done(lbm3d_handle h);

/* FP64 fields at the current time n (Eqs. 53-54): dT = T - t0 = s E / C_V and
 * q = s beta J of the populations the next step pulls.  Any output may be
 * NULL.  Host outputs go through a temporary device buffer. */
int lbm3d_moments(lbm3d_handle h, double* dT, double* qx, double* qy, double* qz, int32_t on_device);

/* The same fields at `count` nodes given by linear index (z * ny + y) * nx + x:
 * out[4k + 0..3] = dT, qx, qy, qz of node k.  nodes and out are both host or
 * both device arrays.  Errors: EINVAL (index out of range, for host arrays;
 * an out-of-range index in a device array yields NaN in its four outputs). */
int lbm3d_sample(lbm3d_handle h, const int64_t* nodes, int64_t count, double* out, int32_t on_device);

/* FP64 totals at the current time: out[0] = C_V sum dT, out[1..3] = sum q.
 * Errors: ENONFINITE if any total is not finite. */
int lbm3d_totals(lbm3d_handle h, double out[4]);

/* Time steps per launch: 2 advances two steps in one pass over HBM where an
 * lbm3d_step call has at least two steps left (temporal blocking: each block
 * owns 60 x 12 nodes of every plane of a z-range, marches along z, and keeps
 * the intermediate state in LDS and registers: rounded exactly as a stored
 * step for FP32 storage and under LBM_FLAG_ROUND_EVERY_STEP, else in FP32);
 * 1 issues every step on its own.  FP32 and that flag: results identical
 * either way; 16-bit storage otherwise rounds one state per launch, so its
 * results depend on the steps per launch (see LBM_FLAG_ROUND_EVERY_STEP).
 * Default: 2 when the box holds at least 256 such blocks (60 x 12 nodes of 32
 * planes each: one per CU), else 1.  Errors: EINVAL (steps not 1 or 2). */
int lbm3d_set_step_fusion(lbm3d_handle h, int32_t steps);

/* The current time steps per launch (1 or 2); -1 for an invalid handle. */
int32_t lbm3d_get_step_fusion(lbm3d_handle h);

/* Launch shape of the step kernel (default: 4 rows of one segment per tile,
 * ordinary stores, XCD remap off for the chunked layout and on for planes).
 * Errors: EINVAL. */
int lbm3d_set_launch_shape(lbm3d_handle h, const lbm3d_launch_shape* shape);
int lbm3d_get_launch_shape(lbm3d_handle h, lbm3d_launch_shape* shape);

/* Time every single-step tile shape (rows_per_tile x tile_waves) with and
 * without the XCD remap, then streaming stores on the fastest, then two steps
 * per launch over z ranges of 16, 32 and 64 planes, each with and without
 * streaming stores, for `steps` steps each (0 selects 20) on buffers filled
 * with a fixed pattern of moderate finite values; keep the fastest shape, z
 * range, store kind and steps per launch.  Must run before lbm3d_init (it
 * overwrites the buffers).  report, if not NULL, receives a JSON summary
 * ({"timings_us": [[rows, xcd, nt, tile_waves, us], ...], "best": [rows, xcd,
 * nt, tile_waves, single-step us], "pair_us_per_step": [[zchunk, nt, us],
 * ...], "zchunk": z, "steps_per_launch": 1 or 2}) truncated to report_len.
 * Errors: ESTATE (memory not bound, or already initialised), EHIP. */
int lbm3d_autotune(lbm3d_handle h, int32_t steps, char* report, size_t report_len);

/* Free the handle and the memory it allocated. */
void lbm3d_destroy(lbm3d_handle h);

#ifdef __cplusplus
}
#endif

#endif /* PHONON_D3Q14_H */
