// Shared between the device code (lbm_device.hip) and the host runtime
// (lbm_runtime.cpp): the per-instance descriptor the kernels read, the launch
// parameters, and the host-side launch entry points of the device file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace plbm {

constexpr int kMaxBlock = 512;     // threads per block upper bound (launch bounds)
constexpr int kPartials = 5;       // per-tile FP64 partials: sum dE, sum qx, sum qy, |dm|^2, |m|^2

// Per-instance descriptor, resident in device memory (one 192-byte record).
// Stored quantity: g_i = (e_i - R_i(x)) / s, the deviation from a reference
// state R that one step maps exactly onto itself (advection then relaxation):
//   R_i(x) = omega_i C_V T_ref(x) + c_ix p_i,   T_ref = t0 - grad * x,
// where p_i (one value for axis, one for diagonal directions) is the flux and
// non-equilibrium share of the bulk steady state under the imposed gradient
// (zero without a gradient).  The interior update is then the bare relaxation
// of g; diffuse walls get the constant offset wall_kd; with tau_R infinite no
// bulk steady state exists and the per-step forcing force_a/force_d is used.
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
    int64_t row;            // elements between rows
    int64_t plane;          // elements between direction runs
    int64_t chunk;          // elements between 64-node chunks (0: planes layout)
    int64_t off;            // element offset of this instance in a buffer
    int64_t node_off;       // offset of this instance in node-indexed arrays (snapshot)
    float inv_tau;          // 1 / tau: decay of the non-equilibrium share per step
    float sigma;            // 1 - rho = 2 / (2 tau_r + 1): decay of the flux share per step
    float force_a;          // per-step forcing c_ix * force_{a,d} (gradient with tau_R = inf)
    float force_d;
    float wall_g[4];        // C_V (T_wall - T_ref) / s for isothermal walls (times omega_i)
    float wall_kd;          // diffuse-wall offset p_diag / s of the leaving diagonal populations
    int32_t has_force;      // force_a/force_d nonzero
    double s_cv;            // s / C_V   (dT = s E / C_V)
    double s_beta;          // s * beta  (q = q_ref + s beta j)
    double s;               // storage scale
    double cv;
    double q_ref;           // heat flux (x) of the reference state
    double p_axis, p_diag;  // reference shares p_i (energy density units)
};
static_assert(sizeof(InstDesc) == 192, "descriptor layout");

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

struct StepArgs {
    const InstDesc* desc;
    const int32_t* tile_inst;   // global tile -> instance
    const void* src;            // post-relaxation populations of step n-1
    void* dst;                  // post-relaxation populations of step n
    double* snap;               // FP64 (dT, qx, qy) per node (node_off indexed), SNAP/CHECK
    double* partials;           // kPartials per global tile, CHECK
    int32_t tile_base;          // first global tile of this launch
    int32_t ntiles;             // tiles in this launch
    const uint32_t* ctr_in;     // steps completed before this step (device counter)
    uint32_t* ctr_out;          // written with ctr_in + 1 by the block of global tile 0
    uint32_t seed;              // stream of the stochastic-rounding bits
    int32_t sr;                 // 1: round stores stochastically (nodes per lane must be 1)
};

// Host-side launchers defined in lbm_device.hip; they return hipError_t.
// snap_stride: nodes of the whole handle (the snapshot holds dT, qx, qy planes).
hipError_t launch_step(int storage, const Shape& sh, int mode, const StepArgs& a,
                       int64_t snap_stride, hipStream_t st);

// Moments of the state at time n of one instance.  With pull != 0 the state is
// rebuilt from the post-relaxation populations of step n-1 (advection plus
// boundary treatment), else read in place (time 0, pre-relaxation state).
// out_kind: 0 = FP32 absolute T (+ q) ; 1 = FP64 deviation dT (+ q).
// partials (may be null): kPartials per tile of this instance (block) for totals.
hipError_t launch_moments(int storage, const InstDesc* d_desc, int inst, const InstDesc& h_desc,
                          const void* buf, int pull, int out_kind, void* T, void* qx, void* qy,
                          double t0, double grad, double* partials, hipStream_t st);

// Equilibrium initialisation: writes the pre-relaxation state to `pre` and its
// relaxation to `post`.  T, qx, qy: device FP64 (qx, qy may be null).
hipError_t launch_init(int storage, const InstDesc* d_desc, int inst, const InstDesc& h_desc,
                       void* pre, void* post, const double* T, const double* qx,
                       const double* qy, double t0, double grad, double beta, hipStream_t st);

// Deterministic per-instance reduction of tile partials into results
// (kPartials doubles per instance).  One block per instance.
hipError_t launch_finalize(const InstDesc* d_desc, int ninst, const double* partials,
                           double* results, hipStream_t st);

// Reduction of moments-kernel partials (tiles of 256 nodes) of one instance.
hipError_t launch_finalize_range(const double* partials, int nparts, double* result,
                                 hipStream_t st);

}  // namespace plbm
