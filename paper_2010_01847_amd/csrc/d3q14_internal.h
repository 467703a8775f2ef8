// Shared between the D3Q14 device code (d3q14_device.hip) and its host
// runtime (d3q14_runtime.cpp): box geometry, relaxation coefficients, launch
// parameters and the host-side launch entry points of the device file.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace plbm3 {

constexpr int kQ = 14;          // 6 axis movers + 8 corner movers
constexpr int kTileX = 64;      // nodes of a row per tile (one wavefront)
constexpr int kRowAlign = 64;   // row pitch in elements is a multiple of this

// Geometry of one periodic box in device memory, with row = z * ny + y:
//   layout 0 (planes):  element i * plane + row * pitch + x;
//   layout 1 (chunked): element ((row * nseg + x / 64) * 14 + i) * 64 + x % 64.
// Elements at x >= nx are padding, never read.
//
// Work split: a thread block covers a tile of 64 * tile_waves consecutive
// nodes of each of rows_per_tile rows (one wavefront per 64-node segment).
struct Geometry {
    int32_t nx, ny, nz;
    int32_t layout;             // 0 planes, 1 chunked
    int32_t pitch;              // planes: elements per row (nx rounded up to kRowAlign)
    int32_t nseg;               // 64-node segments per row
    int64_t plane;              // planes: elements from one direction plane to the next
    uint32_t tile_waves;        // 1, 2, 4 or 8 wavefronts along x per tile
    uint32_t rows_per_tile;     // 1, 2 or 4 rows per tile (tile_waves * rows_per_tile <= 8)
    uint32_t ntx, nty;          // tiles along x and y
    uint32_t ntiles;            // ntx * nty * nz
};

// Per-direction factors of one relaxation in FP32 (see the device file):
// g_i + inv_tau (omega_i E - g_i) + k_i (c_i . J).
struct Coeffs {
    float inv_tau;
    float omega_axis, omega_corner;
    float k_axis, k_corner;
};

struct StepArgs {
    Geometry g;
    Coeffs c;
    const void* src;            // post-relaxation populations of the previous step
    void* dst;                  // this step's post-relaxation populations
    uint32_t step;              // step index (stochastic rounding counter)
    uint32_t seed;
    int32_t xcd_remap;          // hand each XCD a contiguous range of tiles
    int32_t nontemporal;        // streaming (non-temporal) stores
};

// storage: 0 FP32, 1 FP16, 2 BF16; sr: stochastic rounding of the stores.
hipError_t launch_step(int storage, int sr, const StepArgs& a, hipStream_t st);

// Two steps per launch (steps `step` and `step + 1`): a block of 64 * kPairNW
// threads owns 60 x kPairYO output nodes of each plane of a range of zchunk
// planes and marches along z (see the device file).  Measured at 512^3 FP32
// (GLUPS, best z range, XCD remap on; single steps 50):
//   rows x waves  4 x 4: 58.8 (50 KB LDS, 142 VGPRs)   4 x 8: 57.0
//                 6 x 10: 65.7   8 x 12: 69.8   12 x 16: 71.1 (107 KB LDS,
//                 88 VGPRs, one block of 16 wavefronts per CU)
// 12 x 16 is the largest tile that keeps one window row per wavefront
// (88 VGPRs) within the 1024-thread block and 160 KB LDS limits.
constexpr int kPairW3 = 60;
#ifndef PLBM3_PAIR_ROWS
#define PLBM3_PAIR_ROWS 12
#endif
#ifndef PLBM3_PAIR_WAVES
#define PLBM3_PAIR_WAVES 16
#endif
constexpr int kPairYO = PLBM3_PAIR_ROWS;
constexpr int kPairNW = PLBM3_PAIR_WAVES;
// Fewest two-step tiles (blocks) for which two steps per launch are the
// default: one per CU.
constexpr int64_t kPairMinTiles = 256;
struct PairArgs {
    Geometry g;
    Coeffs c;
    const void* src;
    void* dst;
    uint32_t step;
    uint32_t seed;
    int32_t xcd_remap;
    int32_t nontemporal;
    uint32_t ptx, pty, ptz;     // tiles along x (60 nodes), y (kPairYO rows), z (zchunk planes)
    uint32_t ntiles;            // ptx * pty * ptz
    int32_t zchunk;
};
// every_step: 16-bit storage rounds the first step's results to the storage
// type as well (the same bits as two single steps); FP32 always does.
hipError_t launch_pair(int storage, int sr, int every_step, const PairArgs& a, hipStream_t st);

// Fill `bytes` (a multiple of 4) with the timing scratch pattern of the
// device file (moderate finite values in every storage type, changing bits).
hipError_t launch_fill(void* buf, size_t bytes, uint32_t seed, hipStream_t st);

// Equilibrium initial state: element (i, x) holds the scaled deviation of the
// Eq. 15 equilibrium at node x + c_i, so that the first pull reads e_i(x, 0).
hipError_t launch_init(int storage, const Geometry& g, void* dst, const double* T, const double* qx,
                       const double* qy, const double* qz, double t0, double cv, double inv_beta,
                       double inv_s, hipStream_t st);

// FP64 moments of the pulled populations at every node: dT = E * e_scale,
// q = J * q_scale.  Null outputs are skipped.
hipError_t launch_moments(int storage, const Geometry& g, const void* src, double e_scale, double q_scale,
                          double* dT, double* qx, double* qy, double* qz, hipStream_t st);

// The same at `count` listed nodes (linear index (z * ny + y) * nx + x);
// out[4k + 0..3] = dT, qx, qy, qz of node k.
hipError_t launch_sample(int storage, const Geometry& g, const void* src, double e_scale, double q_scale,
                         const int64_t* nodes, int64_t count, double* out, hipStream_t st);

// Number of first-stage blocks of launch_totals and the FP64 partials they need
// (4 doubles each).
int totals_blocks(const Geometry& g);

// FP64 sums over all stored populations: out[0] = sum g, out[1..3] = sum c g
// (unscaled), two fixed-order stages.
hipError_t launch_totals(int storage, const Geometry& g, const void* src, double* partials, double* out,
                         hipStream_t st);

}  // namespace plbm3
