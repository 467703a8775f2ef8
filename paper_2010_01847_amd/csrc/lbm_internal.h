// Shared between the device code (lbm_device.hip) and the host runtime
// (lbm_runtime.cpp): the per-instance descriptor the kernels read, the launch
// parameters, and the host-side launch entry points of the device file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace plbm {

constexpr int kMaxBlock = 512;     // threads per block upper bound (launch bounds)
constexpr int kPartials = 5;       // per-tile FP64 partials: sum dE, sum qx, sum qy, |dm|^2, |m|^2
constexpr int kGroup = 1024;       // tile records per first-stage reduction block

// A compensated FP64 sum: the value is hi + lo with |lo| <= ulp(hi) / 2, and hi
// alone is the sum rounded to double.  The reductions carry their partial sums
// in this form (partial records are kPartials of them).  The total x-flux is
// summed compensated from the first node on, so it is the correctly rounded
// sum of its node values except with a probability of order N 2^-53 times the
// sum's condition number, whatever the grouping of the nodes into tiles: the
// reference-flux update at check steps, which rounds a small difference of
// that total to FP32, then does not depend on the kernel, launch shape or
// schedule that formed it.  The other sums are only reported.
struct DD {
    double hi, lo;
};

// Per-instance descriptor, resident in device memory (one 256-byte record).
//
// Element address of direction i at node (x, y):
//     off + y * row + (x >> cshift) * chunk + (x & cmask) + i * plane
//   planes layout : row = pitch, plane = ny * pitch + pad, chunk = 0,
//                   cshift = 31, cmask = 0x7fffffff   (x contiguous per plane)
//   chunked layout: 64-node row segments, each holding its 8 direction runs
//                   back to back: row = nchunks * 512, chunk = 512, plane = 64,
//                   cshift = 6, cmask = 63
struct alignas(64) InstDesc {
    int32_t nx, ny;
    int32_t bc_x, bc_y;
    int32_t tiles_x;        // tiles along x for the current launch shape
    int32_t tile_begin;     // first global tile index of this instance
    int32_t ntiles;         // tiles of this instance
    int32_t cshift;         // log2 of the chunk width (31: no chunking)
    int32_t cmask;          // chunk width - 1
    int32_t layout;         // 1 = planes, 2 = chunked
    int32_t group_begin;    // first reduction group of this instance (kGroup tiles each)
    int32_t ngroups;        // reduction groups of this instance
    int32_t wk[4];          // boundary kind of each wall (x=0, x=nx-1, y=0, y=ny-1); 0 on periodic axes
    int32_t p_tiles_x;      // fused kernel: strips along x (fused_width columns each)
    int32_t p_tile_begin;   // fused kernel: first global tile of this instance
    int32_t p_ntiles;       // fused kernel: tiles of this instance
    int32_t p_group_begin;  // fused kernel: first reduction group (kGroup of its tiles each)
    int32_t p_ngroups;      // fused kernel: reduction groups of this instance
    int64_t row;            // elements between rows
    int64_t plane;          // elements between direction runs
    int64_t chunk;          // elements between 64-node chunks (0: planes layout)
    int64_t off;            // element offset of this instance in a buffer
    int64_t node_off;       // offset of this instance in node-indexed arrays (snapshot)
    float inv_tau;          // 1 / tau: decay of the non-equilibrium share per step
    float sigma;            // 1 - rho = 2 / (2 tau_r + 1): decay of the flux share per step
    float wall_g[4];        // C_V (T_wall - T_ref) / s for isothermal walls (times omega_i)
    float wall_q[4];        // q_0 / (beta s) for heat-flux walls (added to the incident sum)
    float flux_a, flux_d;   // (1 / tau - sigma) x 1/3 and x 1/12: the folded flux coefficients (relax_folded)
    double s_cv;            // s / C_V   (dT = s E / C_V)
    double s_beta;          // s * beta  (q = q_ref + s beta j)
    double s;               // storage scale
    double cv;
};
static_assert(sizeof(InstDesc) == 256, "descriptor layout");

// Reference state of the stored deviations, one per instance, in device
// memory (kept apart from InstDesc: the device updates it, the host does not
// rewrite it when the launch shape changes).  Stored quantity:
// g_i = (e_i - R_i(x)) / s before relaxation, with
//     R_i(x) = omega_i C_V T_ref(x) + c_ix p_i,   T_ref = t0 - G x,
//     p_axis = J/3 + pa0,   pa0 = (2/9) C_V G + (tau - 1) C_V G / 27,
//     p_diag = J/12 + pd0,  pd0 = C_V G / 36 - (tau - 1) C_V G / 54,
// (G = 0 without the gradient seam).  sum_i c_ix R_i = J + j_b with
// j_b = (5/9) C_V G, and J is the x-flux of R after relaxation.  One step
// (advection across the seam of Eqs. 59-60, relaxation of Eqs. 13, 15, 16)
// maps R onto itself plus the uniform forcing c_ix w_i (rho (J + j_b) - J)
// (w = 1/3 axis, 1/12 diagonal), which vanishes at the bulk steady state
// J = j_b (tau_r - 1/2).  For an adaptive instance the finalisation kernel
// moves J to the lattice's mean x-flux at every check step, which keeps the
// stored values small in transients and at steady state alike; the stored
// populations then change by the uniform c_ix w_i (J_old - J_new) / s
// ("shift"), which the next step adds to its pulled values once.
struct alignas(64) RefState {
    double J;               // post-relaxation reference x-flux (energy units)
    double q_ref;           // heat flux of R: beta (J + j_b)
    double p_axis, p_diag;  // c_ix shares of R (energy units)
    double jb, pa0, pd0;    // j_b and the J-independent parts of p
    double rho, sigma;      // flux factor per step and 1 - rho (computed directly)
    double beta, s;         // Eq. 54 factor; storage scale
    double inv_nodes;       // 1 / (nx ny)
    float force_a, force_d; // forcing per step / s, axis and diagonal (times c_ix)
    float shift_a, shift_d; // pending shift / s (times c_ix); shift_d = shift_a / 4 exactly
    float wall_kd;          // p_diag / s: offset of the diagonals leaving a diffuse y wall
    int32_t adapt;          // 1: J follows the mean flux at check steps
};
static_assert(sizeof(RefState) == 128, "reference state layout");

// Set the J-dependent fields of r for reference flux J (host at
// initialisation, device at check steps).
__host__ __device__ inline void ref_set_flux(RefState& r, double J) {
    r.J = J;
    r.q_ref = r.beta * (J + r.jb);
    r.p_axis = J / 3.0 + r.pa0;
    r.p_diag = J / 12.0 + r.pd0;
    // rho (J + j_b) - J, with 1 - rho kept as its own (accurate) coefficient
    const double f = r.rho * r.jb - r.sigma * J;
    r.force_a = (float)(f / (3.0 * r.s));
    r.force_d = (float)(f / (12.0 * r.s));
    r.wall_kd = (float)(r.p_diag / r.s);
}

// Launch shape chosen by the runtime (or the autotuner).
struct Shape {
    int vec = 1;         // nodes per thread along x
    int bx = 256;        // threads per block along x (multiple of 64)
    int by = 1;          // rows per block
    int xcd = 1;         // XCD-aware tile remap
    int nt = 0;          // non-temporal stores
    int tile_w() const { return vec * bx; }
};

enum StepMode { kPlain = 0, kSnap = 1, kCheck = 2 };
// How a fused launch ends (see march_kernel): plain steps only, on the
// snapshot step (FP64 moments written to the snapshot), on the check step
// (the snapshot kept in registers, per-tile check sums written), or, for the
// readout of 16-bit storage, with the FP64 moments of its last step's pulled
// nodes written to a.snap and no populations stored.
enum FusedEnd { kEndPlain = 0, kEndSnap = 1, kEndCheck = 2, kEndMoments = 3 };

// Fused kernel (several time steps per pass over HBM, temporal blocking): a
// wavefront takes a strip of fused_width output columns (a window of 64
// columns with a halo of fuse_max nodes on each side) of a chunk of
// kMarchRows rows, and marches along y advancing up to fuse_max steps; see the
// device file.  The kernel is bound by vector ALU issue, not by HBM (with six
// steps per launch an FP32 update moves about a fifth of the single-step
// bytes), so the most steps per launch is a per-kind balance between the HBM
// bytes saved, the halo nodes recomputed and the registers the delay lines
// take (FP32: 88 / 102 / 116 / 130 VGPRs at 4 / 5 / 6 / 7 steps).  For the
// 16-bit kinds it also depends on how many of a launch's steps are rounded to
// the storage type (FusedRounding): rounding every step, four steps per
// launch were the fastest (FP16-SR 743, F16_SPLIT 819 us per launch on
// 8192^2); rounding the last one, six.  Chunks of 64 or 128 rows instead of
// 32: FP32 302 / 289 GLUPS at six steps against 315.
constexpr int kMarchRows = 32;
// Elements between direction runs in the chunked layout (64-node segments).
constexpr int kChunkPlane = 64;
__host__ __device__ constexpr int fuse_max(int storage) {
    return storage == 0 ? 7 : 6;
}
__host__ __device__ constexpr int fused_width(int storage) { return 64 - 2 * fuse_max(storage); }
// Most steps per launch of a 16-bit handle that rounds every step
// (LBM_FLAG_ROUND_EVERY_STEP).
constexpr int kFuseEveryStep = 4;
// Which of a fused launch's steps round their results to the storage type
// (FP32 storage rounds every step, that being its arithmetic):
//   kRoundEvery: every step (the same bits as single steps);
//   kRoundLast : the last one (16-bit default); the others keep the FP32
//                result of the relaxation in registers, and readouts rebuild
//                time n by replaying the whole launch with kEndMoments.
enum FusedRounding { kRoundEvery = 0, kRoundLast = 1 };
// Fewest fused-kernel strips (wavefronts) over all instances for which fused
// launches are the default: one per SIMD of the chip.
constexpr int64_t kFuseMinStrips = 1024;

struct StepArgs {
    const InstDesc* desc;
    const int32_t* tile_inst;   // global tile -> instance
    const void* src;            // post-relaxation populations of step n-1
    void* dst;                  // post-relaxation populations of step n
    double* snap;               // FP64 (dT, qx, qy) per node (node_off indexed), SNAP/CHECK
    DD* partials;               // kPartials compensated sums per global tile, CHECK
    int32_t tile_base;          // first global tile of this launch
    int32_t ntiles;             // tiles in this launch
    const RefState* ref;        // per-instance reference states
    int32_t apply_shift;        // 1: add the pending reference shift to the pulled values
    const uint32_t* ctr_in;     // steps completed before this step (device counter)
    uint32_t* ctr_out;          // written with ctr_in + steps by the launch's first tile
    uint32_t seed;              // stream of the stochastic-rounding bits
    int32_t sr;                 // 1: round stores stochastically (nodes per lane must be 1)
};

// Host-side launchers defined in lbm_device.hip; they return hipError_t.
// snap_stride: nodes of the whole handle (the snapshot holds dT, qx, qy planes).
hipError_t launch_step(int storage, const Shape& sh, int mode, const StepArgs& a,
                       int64_t snap_stride, hipStream_t st);

// k time steps (m .. m + k - 1, 2 <= k <= fuse_max(storage)) in one pass over
// HBM, ending as `end` (FusedEnd) says: kEndSnap, the last one is the snapshot
// step (its FP64 moments go to a.snap, snap_stride doubles per field);
// kEndCheck, the last one is the check step (kPartials check sums per fused
// tile go to a.partials, for launch_finalize with fused != 0); chunked != 0
// for the chunked layout; a.apply_shift refers to the first of them;
// a.tile_inst / tile_base / ntiles index the fused tile table; `rounding`
// (FusedRounding) says which steps round to the storage type: kRoundEvery
// (FP32 always; 16-bit k <= kFuseEveryStep) gives the same bits as k single
// steps (the check sums equal theirs up to the order of summation);
// kRoundLast is 16-bit only, and the only one with kEndMoments (whose FP64
// moments go to a.snap as kEndSnap's do).
hipError_t launch_fused(int storage, const Shape& sh, const StepArgs& a, int k, int end, int chunked,
                        int rounding, int64_t snap_stride, hipStream_t st);

// Moments of the state at time n of one instance.  With pull != 0 the state is
// rebuilt from the post-relaxation populations of step n-1 (advection plus
// boundary treatment), else read in place (time 0, pre-relaxation state).
// out_kind: 0 = FP32 absolute T (+ q) ; 1 = FP64 deviation dT (+ q).
// partials (may be null): kPartials compensated sums per tile of this
// instance (block) for totals.
hipError_t launch_moments(int storage, const InstDesc* d_desc, const RefState* d_ref, int inst,
                          const InstDesc& h_desc, const void* buf, int pull, int pending_shift,
                          int out_kind, void* T, void* qx, void* qy, double t0, double grad,
                          DD* partials, hipStream_t st);

// Equilibrium initialisation: writes the pre-relaxation state to `pre` and its
// relaxation to `post`.  T, qx, qy: device FP64 (qx, qy may be null).
hipError_t launch_init(int storage, const InstDesc* d_desc, const RefState* d_ref, int inst,
                       const InstDesc& h_desc, void* pre, void* post, const double* T,
                       const double* qx, const double* qy, double t0, double grad, double beta,
                       hipStream_t st);

// Deterministic per-instance reduction of tile partials into results
// (kPartials doubles per instance), in two fixed-order stages: groups of
// kGroup tile records (group_inst: group -> instance; groups g0 .. g0 +
// ngroups - 1) into gpart, then one block per instance (i0 .. i0 + ninst - 1)
// over its groups.  fused != 0: the
// records are per fused-kernel tile (InstDesc p_* fields), else per
// single-step tile.  The second stage copies each instance's reference state
// to d_ref_prev and then moves an adaptive instance's reference flux to its
// mean heat flux.
hipError_t launch_finalize(const InstDesc* d_desc, const int32_t* group_inst, int g0, int ngroups, RefState* d_ref,
                           RefState* d_ref_prev, int i0, int ninst, const DD* partials, DD* gpart,
                           double* results, int fused, hipStream_t st);

// Fill `bytes` (a multiple of 4) with the timing scratch pattern of the
// device file (moderate finite values in every storage type, changing bits).
hipError_t launch_fill(void* buf, size_t bytes, uint32_t seed, hipStream_t st);

// One-thread kernel writing *dst = v on the stream (stream-ordered updates of
// descriptor fields between steps).
hipError_t launch_set_float(float* dst, float v, hipStream_t st);

// Moments of instance `inst` from FP64 (dT, qx, qy) planes laid out as the
// snapshot (a kEndMoments launch's output), in launch_moments' output forms
// and partials.
hipError_t launch_plane_moments(const InstDesc* d_desc, int inst, const InstDesc& h, const double* planes,
                                int64_t stride, int out_kind, void* T, void* qx, void* qy, double t0, double grad,
                                DD* partials, hipStream_t st);

// Launch every fused-kernel variant of a storage kind, rounding (sr), layout
// and step rounding (every_step != 0 or FP32: kRoundEvery; else kRoundLast,
// with the readout's kEndMoments) once with no tiles (no memory is touched),
// so that the runtime's first-launch work is done before the first real
// launch.
hipError_t preload_fused(int storage, int sr, int chunked, int every_step, hipStream_t st);

// Copy n <= 64 32-bit words on the device (a kernel, so that it can sit in a
// captured graph).
hipError_t launch_copy_u32(uint32_t* dst, const uint32_t* src, int n, hipStream_t st);

// Reduction of nparts moments-kernel partials (tiles of 256 nodes) of one
// instance, through gpart (ceil(nparts / kGroup) records), into one record.
hipError_t launch_finalize_range(const DD* partials, int nparts, DD* gpart, DD* result, hipStream_t st);

}  // namespace plbm
