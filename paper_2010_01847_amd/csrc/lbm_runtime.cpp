// Host runtime of the phonon lattice Boltzmann library: the C ABI of
// phonon_lbm.h.  It validates configurations, derives the per-instance
// coefficients (Eqs. 49, 54 and the relaxation-plus-source factor from
// Eqs. 13, 15, 16), lays the populations out in device memory, builds the tile
// schedule, and issues the kernels of lbm_device.hip on the caller's stream,
// eagerly or from captured HIP graphs.
#include "../../include/phonon_lbm.h"
#include "lbm_internal.h"

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace plbm;

namespace {

constexpr uint32_t kMagic = 0x4c424d31u;   // "LBM1"
constexpr size_t kAlign = 256;
thread_local std::string g_create_error;

struct Status {
    int code;
    std::string msg;
};

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int esize_of(int storage) { return storage == LBM_F32 ? 4 : 2; }
bool is_split(int storage) { return storage == LBM_F16_SPLIT || storage == LBM_BF16_SPLIT; }
bool is_f16(int storage) { return storage == LBM_F16 || storage == LBM_F16_SPLIT; }

// Row pitch in elements for the planes layout: row bytes a multiple of 256.
int32_t pitch_of(int32_t nx, int es) {
    const int per = (int)(kAlign / es);
    return (int32_t)(((int64_t)nx + per - 1) / per * per);
}

// Pad after each direction plane of the planes layout.  Eight planes whose
// starts are a power of two apart load the same HBM channels together; a
// 4 KB offset between consecutive planes spreads them (measured on MI355X:
// an 8-in/8-out plane copy of 8192^2 FP32 goes from 5.44 to 5.84 TB/s).
size_t plane_pad_bytes() {
    static const size_t v = [] {
        const char* e = getenv("LBM_PLANE_PAD_BYTES");
        return e ? (size_t)strtoull(e, nullptr, 10) / kAlign * kAlign : (size_t)4096;
    }();
    return v;
}

struct Geometry {
    int64_t row, plane, chunk, elems;
    int32_t cshift, cmask;
};

// Element geometry of one instance (see InstDesc for the address formula).
// Every instance's size is a multiple of 64 elements, so every instance and
// plane start stays 256-byte (FP32) / 128-byte (16-bit) aligned.  Split
// storage (chunked only): a chunk holds the eight 16-bit h runs and then the
// FP32 energy run, 640 16-bit elements (1280 bytes).
Geometry geometry_of(const lbm_instance& in, int es, int layout, bool split = false) {
    Geometry g;
    if (split) {
        const int64_t nch = ((int64_t)in.nx + 63) / 64;
        g.row = nch * 640;
        g.plane = kChunkPlane;
        g.chunk = 640;
        g.cshift = 6;
        g.cmask = 63;
        g.elems = (int64_t)in.ny * g.row;
        return g;
    }
    if (layout == LBM_LAYOUT_PLANES) {
        g.row = pitch_of(in.nx, es);
        g.plane = (int64_t)in.ny * g.row + (int64_t)(plane_pad_bytes() / es);
        g.chunk = 0;
        g.cshift = 31;
        g.cmask = 0x7fffffff;
        g.elems = 8 * g.plane;
    } else {
        const int64_t nch = ((int64_t)in.nx + 63) / 64;
        g.row = nch * 512;
        g.plane = kChunkPlane;
        g.chunk = 512;
        g.cshift = 6;
        g.cmask = 63;
        g.elems = (int64_t)in.ny * g.row;
    }
    return g;
}

// Launch costs of a k-step launch on the second-sound lattice 8192^2
// (MI355X, microseconds; k = 1 is the single-step kernel), plain and ending on
// the check step.  A fused launch costs about the same for every k from 2 up
// to a kind-dependent point (it streams the same rows and the strips' halo
// whatever the number of stages; below five FP32 steps it is bound by memory
// requests, above by VALU issue), so the way a short run is cut into launches
// matters: 20 FP32 steps cost 3522 us as 7 + 7 + 6 and 4372 us as 5 + 5 + 5 +
// 5.  The check variants of five, six and seven FP32 steps need 131, 145 and
// 159 VGPRs (three waves per SIMD instead of four).  16-bit kinds: rounding
// every step (every_step) or only the last of a launch (FusedRounding).
// lbm_autotune replaces the plain figures by its own timings on the handle's
// lattices and scales the check figures.
static void default_costs(int storage, int every_step, double plain[8], double check[8]) {
    static const double p_tab[5][8] = {{0, 737, 1214, 1208, 1237, 1093, 1098, 1212},   // F32
                                       {0, 498, 572, 588, 650, 823, 947, 0},           // F16
                                       {0, 482, 573, 588, 722, 828, 948, 0},           // BF16
                                       {0, 483, 730, 742, 744, 869, 985, 0},           // F16_SPLIT
                                       {0, 482, 733, 745, 744, 873, 994, 0}};          // BF16_SPLIT
    static const double c_tab[5][8] = {{0, 0, 1216, 1095, 1095, 1217, 1360, 1558},
                                       {0, 0, 631, 757, 857, 1114, 1260, 0},
                                       {0, 0, 703, 788, 995, 1122, 1269, 0},
                                       {0, 0, 747, 797, 897, 1155, 1300, 0},
                                       {0, 0, 753, 814, 909, 1162, 1309, 0}};
    // 16-bit kinds rounding every step (kFuseEveryStep = 4 at most)
    static const double pe_tab[5][5] = {{0, 0, 0, 0, 0},
                                        {0, 496, 604, 600, 743},
                                        {0, 484, 607, 598, 738},
                                        {0, 486, 716, 717, 819},
                                        {0, 486, 721, 728, 861}};
    static const double ce_tab[5][5] = {{0, 0, 0, 0, 0},
                                        {0, 0, 638, 834, 1014},
                                        {0, 0, 679, 852, 1009},
                                        {0, 0, 731, 866, 1032},
                                        {0, 0, 728, 889, 1084}};
    for (int k = 0; k < 8; ++k) plain[k] = check[k] = 0.0;
    if (storage < 0 || storage > 4) return;
    const bool every = storage != LBM_F32 && every_step;
    const int kmax = every ? kFuseEveryStep : fuse_max(storage);
    for (int k = 1; k <= kmax; ++k) {
        plain[k] = every ? pe_tab[storage][k] : p_tab[storage][k];
        check[k] = every ? ce_tab[storage][k] : c_tab[storage][k];
    }
}

int resolve_layout(int layout) { return layout == LBM_LAYOUT_PLANES ? LBM_LAYOUT_PLANES : LBM_LAYOUT_CHUNKED; }

struct Coeffs {
    double tau, tau_c, beta, rho, one_minus_rho;
};

// tau = tau_C + 1/2 (Eq. 49), 1/tau_C = 1/tau_N + 1/tau_R; beta of Eq. 54;
// rho = (2 tau_r - 1)/(2 tau_r + 1), the per-step factor on the heat flux that
// Eqs. 13, 15, 16 and 54 give; 1 - rho = 2/(2 tau_r + 1) is kept separately
// (computed directly, not as 1 - rho) because the kernels apply it as the
// flux decay coefficient.
Coeffs coeffs_of(const lbm_instance& in) {
    Coeffs c;
    const bool inf_r = std::isinf(in.tau_r);
    const double inv_tc = 1.0 / in.tau_n + (inf_r ? 0.0 : 1.0 / in.tau_r);
    c.tau_c = 1.0 / inv_tc;
    c.tau = c.tau_c + 0.5;
    c.beta = inf_r ? 1.0 : 2.0 * in.tau_r / (2.0 * in.tau_r + 1.0);
    c.rho = inf_r ? 1.0 : (2.0 * in.tau_r - 1.0) / (2.0 * in.tau_r + 1.0);
    c.one_minus_rho = inf_r ? 0.0 : 2.0 / (2.0 * in.tau_r + 1.0);
    return c;
}

bool walled(int bc) { return bc == LBM_BC_ISOTHERMAL || bc == LBM_BC_DIFFUSE || bc == LBM_BC_HEATFLUX; }

// Kind of wall w (0: x = 0, 1: x = nx-1, 2: y = 0, 3: y = ny-1), 0 on a periodic axis.
int wall_kind(const lbm_instance& in, int w) {
    const int axis = w < 2 ? in.bc_x : in.bc_y;
    if (!walled(axis)) return 0;
    return in.wall_bc[w] ? in.wall_bc[w] : axis;
}

Status validate_instance(const lbm_instance& in, int k) {
    char b[256];
    if (in.nx < 2 || in.ny < 2) {
        snprintf(b, sizeof b, "instance %d: nx, ny must be >= 2 (got %d x %d)", k, in.nx, in.ny);
        return {LBM_EINVAL, b};
    }
    if ((int64_t)in.nx * in.ny > ((int64_t)1 << 31)) {
        snprintf(b, sizeof b, "instance %d: more than 2^31 nodes", k);
        return {LBM_EINVAL, b};
    }
    if (!(in.tau_n > 0.0) || std::isinf(in.tau_n) || !(in.tau_r > 0.0)) {
        snprintf(b, sizeof b, "instance %d: need 0 < tau_n < inf and tau_r > 0 (got %g, %g)", k,
                 in.tau_n, in.tau_r);
        return {LBM_EINVAL, b};
    }
    if (in.cv < 0.0 || !std::isfinite(in.cv)) {
        snprintf(b, sizeof b, "instance %d: cv must be finite and >= 0", k);
        return {LBM_EINVAL, b};
    }
    if (in.bc_x < 0 || in.bc_x > 4 || in.bc_y < 0 || in.bc_y > 4 || in.bc_y == LBM_BC_GRADIENT) {
        snprintf(b, sizeof b, "instance %d: bad boundary kind (bc_x %d, bc_y %d; GRADIENT is x only)",
                 k, in.bc_x, in.bc_y);
        return {LBM_EINVAL, b};
    }
    const bool wx = walled(in.bc_x);
    const bool wy = walled(in.bc_y);
    for (int w = 0; w < 4; ++w) {
        if (in.wall_bc[w] != 0 && (!walled(in.wall_bc[w]) || !(w < 2 ? wx : wy))) {
            snprintf(b, sizeof b, "instance %d: wall_bc[%d] = %d must be 0, or a wall kind on a walled axis",
                     k, w, in.wall_bc[w]);
            return {LBM_EINVAL, b};
        }
    }
    if (wx && wy && !(wall_kind(in, 0) == LBM_BC_ISOTHERMAL && wall_kind(in, 1) == LBM_BC_ISOTHERMAL)) {
        snprintf(b, sizeof b, "instance %d: walls on both axes need corner nodes, defined here only when "
                              "both x walls are isothermal", k);
        return {LBM_EUNSUPPORTED, b};
    }
    if (in.bc_x == LBM_BC_GRADIENT &&
        (wall_kind(in, 2) == LBM_BC_ISOTHERMAL || wall_kind(in, 3) == LBM_BC_ISOTHERMAL)) {
        snprintf(b, sizeof b, "instance %d: isothermal walls across a gradient seam are undefined", k);
        return {LBM_EUNSUPPORTED, b};
    }
    int ex = 0;
    if (in.scale < 0.0 || !std::isfinite(in.scale) ||
        (in.scale > 0.0 && std::frexp(in.scale, &ex) != 0.5)) {
        snprintf(b, sizeof b, "instance: scale must be 0 or a power of two (got %g)", in.scale);
        return {LBM_EINVAL, b};
    }
    if (!std::isfinite(in.t0) || !std::isfinite(in.grad_x)) return {LBM_EINVAL, "t0 and grad_x must be finite"};
    return {LBM_OK, ""};
}

// Worst-case tile count over launch shapes (smallest tile: 64 x 1 nodes).
int64_t max_tiles(const std::vector<lbm_instance>& v) {
    int64_t n = 0;
    for (auto& in : v) n += (int64_t)((in.nx + 63) / 64) * in.ny;
    return n;
}

// Two-step kernel tiles along x of one instance.
int64_t fused_tiles_x(const lbm_instance& in, int storage) {
    return (in.nx + fused_width(storage) - 1) / fused_width(storage);
}

// Worst-case count of first-stage reduction groups (per instance, kGroup
// tiles each).
int64_t max_groups(const std::vector<lbm_instance>& v) {
    int64_t n = 0;
    for (auto& in : v) n += ((int64_t)((in.nx + 63) / 64) * in.ny + kGroup - 1) / kGroup;
    return n;
}

struct Layout {
    size_t buf_bytes = 0;      // one population buffer
    size_t off_buf[3] = {0, 0, 0};   // ping-pong pair, and the readout buffer (see replay_tail)
    size_t off_snap = 0, off_part = 0, off_res = 0, off_mpart = 0, off_mres = 0, off_desc = 0,
           off_desc_prev = 0, off_ref = 0, off_ref_prev = 0, off_tiles = 0, off_ptiles = 0, off_groups = 0,
           off_pgroups = 0, off_gpart = 0, off_ctr = 0, total = 0;
    int64_t nodes = 0, tiles_max = 0, mparts_max = 0, groups_max = 0, ptiles = 0, pgroups = 0;
};

// Fused launches round every step: FP32 storage, or LBM_FLAG_ROUND_EVERY_STEP.
static int every_step_of(const lbm_config* cfg) {
    return (cfg->storage == LBM_F32 || (cfg->flags & LBM_FLAG_ROUND_EVERY_STEP)) ? 1 : 0;
}

// every_step: fused launches round every step (FP32, or 16-bit with
// LBM_FLAG_ROUND_EVERY_STEP); otherwise the readout buffer holds FP64 moment
// planes (see replay_tail) and is sized for them as well.
Layout layout_of(const std::vector<lbm_instance>& v, int storage, int check, int layout, int every_step) {
    Layout L;
    const int es = esize_of(storage);
    size_t elems = 0;
    for (auto& in : v) {
        elems += (size_t)geometry_of(in, es, layout, is_split(storage)).elems;
        L.nodes += (int64_t)in.nx * in.ny;
        L.mparts_max = std::max<int64_t>(L.mparts_max, (int64_t)((in.nx + 255) / 256) * in.ny);
    }
    L.buf_bytes = align_up(elems * es, kAlign);
    L.tiles_max = max_tiles(v);
    L.groups_max = max_groups(v);
    const int ph = kMarchRows;
    for (auto& in : v) {
        const int64_t pt = fused_tiles_x(in, storage) * (int64_t)((in.ny + ph - 1) / ph);
        L.ptiles += pt;
        L.pgroups += (pt + kGroup - 1) / kGroup;
    }
    // check-step records: per single-step tile or per fused-kernel tile
    const int64_t records = std::max(L.tiles_max, L.ptiles);
    // the same scratch serves the first stage of every check reduction and of
    // lbm_totals' reduction
    const int64_t gscratch = std::max({L.groups_max, L.pgroups, (L.mparts_max + kGroup - 1) / kGroup});
    size_t o = 0;
    L.off_buf[0] = o; o += L.buf_bytes;
    L.off_buf[1] = o; o += L.buf_bytes;
    L.off_buf[2] = o; o += every_step ? L.buf_bytes : std::max(L.buf_bytes, align_up(3 * (size_t)L.nodes * sizeof(double), kAlign));
    L.off_snap = o; o += check ? align_up(3 * (size_t)L.nodes * sizeof(double), kAlign) : 0;
    L.off_part = o; o += align_up((size_t)records * kPartials * sizeof(DD), kAlign);
    L.off_res = o; o += align_up(v.size() * kPartials * sizeof(double), kAlign);
    L.off_mpart = o; o += align_up((size_t)L.mparts_max * kPartials * sizeof(DD), kAlign);
    L.off_mres = o; o += align_up(kPartials * sizeof(DD), kAlign);
    L.off_desc = o; o += align_up(v.size() * sizeof(InstDesc), kAlign);
    L.off_desc_prev = o; o += align_up(v.size() * sizeof(InstDesc), kAlign);
    L.off_ref = o; o += align_up(v.size() * sizeof(RefState), kAlign);
    L.off_ref_prev = o; o += align_up(v.size() * sizeof(RefState), kAlign);
    L.off_tiles = o; o += align_up((size_t)L.tiles_max * sizeof(int32_t), kAlign);
    L.off_ptiles = o; o += align_up((size_t)L.ptiles * sizeof(int32_t), kAlign);
    L.off_groups = o; o += align_up((size_t)L.groups_max * sizeof(int32_t), kAlign);
    L.off_pgroups = o; o += align_up((size_t)L.pgroups * sizeof(int32_t), kAlign);
    L.off_gpart = o; o += align_up((size_t)gscratch * kPartials * sizeof(DD), kAlign);
    L.off_ctr = o; o += kAlign;                 // 32-bit step counters: ping-pong pair and the readout's
    L.total = o;
    return L;
}

}  // namespace

struct lbm_ctx {
    uint32_t magic = kMagic;
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t capture_stream = nullptr;
    int storage = 0;
    int layout = LBM_LAYOUT_CHUNKED;
    int sr = 0;                      // stochastic rounding of stores
    uint32_t seed = 0;
    int K = 100;                     // check interval, 0 = off
    std::vector<lbm_instance> inst;
    std::vector<InstDesc> desc;
    std::vector<RefState> ref;       // initial reference states (the device copy evolves)
    std::vector<std::array<double, 4>> qwall;   // heat flux into the domain per wall (HEATFLUX walls)
    std::vector<Coeffs> co;
    std::vector<char> inited;
    Shape shape;
    Layout L;
    int64_t ntiles = 0;
    std::vector<int32_t> tile_inst;
    std::vector<int32_t> group_inst;
    int64_t ngroups = 0;
    std::vector<int32_t> ptile_inst;   // fused kernel: tile -> instance
    std::vector<int32_t> pgroup_inst;  // fused kernel: reduction group -> instance
    int64_t npgroups = 0;
    // The instances one launch covers: all of them, or one of the parts that
    // the batched schedule issues on streams of their own (lbm_set_streams).
    struct Span {
        int i0 = 0, ni = 0;                            // instances
        int32_t t0 = 0, nt = 0, g0 = 0, ng = 0;        // single-step tiles and reduction groups
        int32_t pt0 = 0, pnt = 0, pg0 = 0, png = 0;    // fused-kernel tiles and reduction groups
        int ctr = 0;                                   // its step-counter pair: d_ctr()[ctr], [ctr + 1]
    };
    static constexpr int kMaxParts = 2;
    Span all;
    Span part[kMaxParts];
    int nparts = 1;
    int streams_req = 0;               // lbm_set_streams (0: the default)
    bool preloaded = false;            // the fused kernels were launched empty once (first lbm_step)
    hipStream_t part_stream = nullptr; // the second part's stream (created at first use)
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    hipStream_t cap_part_stream = nullptr;   // the same for graph capture
    hipEvent_t cap_fork = nullptr, cap_join = nullptr;
    int fuse = 1;                      // most time steps per launch where allowed (1 .. fuse_cap())
    int every_step = 1;                // fused launches round every step (FP32; LBM_FLAG_ROUND_EVERY_STEP)
    // most steps per launch of this handle's kind and step rounding
    int fuse_cap() const { return (storage != LBM_F32 && every_step) ? kFuseEveryStep : fuse_max(storage); }
    // relative cost of one launch of k steps (index k = 1 .. fuse_max): plain,
    // and fused ending on the check step (see plan_launch)
    double cost_plain[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    double cost_check[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int graph_flips = 0;               // buffer swaps of one captured chunk
    // The last launch of the steps issued so far, when it advanced k >= 2
    // steps: the post-relaxation state of step n - 1, from which the moments
    // at time n are rebuilt, was never written, so a readout first replays
    // steps n - k + 1 .. n - 1 from the launch's source buffer (still intact
    // until the next step) into the readout buffer.
    struct Tail {
        int k = 0;             // steps of the last launch (0: the last launch was a single step)
        int src = 0;           // buffer that launch read
        int apply_shift = 0;   // its first step applied the pending reference shift
        int checked = 0;       // it ended on a check step (the reference moved after it)
    } tail, graph_tail;
    int graph_tail_flip = 0;           // launches of a captured chunk before its last one, mod 2
    bool replayed = false;             // the readout buffer holds the replayed state
    bool desc_saved = false;           // d_desc_prev holds the descriptors of the last step
    std::vector<std::array<float, 4>> wall_q_last;   // their heat-flux terms (the only field that differs)
    std::vector<InstDesc> desc_prev_host;            // host source of d_desc_prev uploads
    bool external = false;
    char* base = nullptr;            // device memory (owned unless external)
    bool owned = false;
    int cur = 0;                     // buffer holding the post-relaxation state of the last step
    int64_t steps = 0;
    int64_t last_check = -1;
    int sched = LBM_SCHED_BATCHED;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int graph_chunk = 0;
    double* staging = nullptr;       // device FP64 staging for host I/O (lazy)
    size_t staging_bytes = 0;
    std::string err;

    char* ptr(size_t off) const { return base + off; }
    void* buf(int k) const { return base + L.off_buf[k]; }
    static constexpr int kReadout = 2;   // index of the readout buffer and of its step counter
    InstDesc* d_desc() const { return reinterpret_cast<InstDesc*>(base + L.off_desc); }
    RefState* d_ref() const { return reinterpret_cast<RefState*>(base + L.off_ref); }
    RefState* d_ref_prev() const { return reinterpret_cast<RefState*>(base + L.off_ref_prev); }
    InstDesc* d_desc_prev() const { return reinterpret_cast<InstDesc*>(base + L.off_desc_prev); }
    int32_t* d_pgroups() const { return reinterpret_cast<int32_t*>(base + L.off_pgroups); }
    // descriptors the last issued step ran with (a heat-flux change since then
    // applies to later steps only)
    const InstDesc* d_desc_last() const { return desc_saved ? d_desc_prev() : d_desc(); }
    int32_t* d_tiles() const { return reinterpret_cast<int32_t*>(base + L.off_tiles); }
    int32_t* d_ptiles() const { return reinterpret_cast<int32_t*>(base + L.off_ptiles); }
    int32_t* d_groups() const { return reinterpret_cast<int32_t*>(base + L.off_groups); }
    DD* d_gpart() const { return reinterpret_cast<DD*>(base + L.off_gpart); }
    double* d_snap() const { return K ? reinterpret_cast<double*>(base + L.off_snap) : nullptr; }
    DD* d_part() const { return reinterpret_cast<DD*>(base + L.off_part); }
    double* d_res() const { return reinterpret_cast<double*>(base + L.off_res); }
    DD* d_mpart() const { return reinterpret_cast<DD*>(base + L.off_mpart); }
    DD* d_mres() const { return reinterpret_cast<DD*>(base + L.off_mres); }
    uint32_t* d_ctr() const { return reinterpret_cast<uint32_t*>(base + L.off_ctr); }

    int fail(int code, const std::string& m) {
        err = m;
        return code;
    }
    int hip_fail(hipError_t e, const char* what) {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return LBM_EHIP;
    }
    void drop_graphs() {
        for (int k = 0; k < 2; ++k) {
            if (gexec[k]) (void)hipGraphExecDestroy(gexec[k]);
            if (graph[k]) (void)hipGraphDestroy(graph[k]);
            gexec[k] = nullptr;
            graph[k] = nullptr;
        }
        graph_chunk = 0;
    }
};

#define HIPCALL(h, expr)                                         \
    do {                                                         \
        hipError_t e_ = (expr);                                  \
        if (e_ != hipSuccess) return (h)->hip_fail(e_, #expr);   \
    } while (0)

static bool valid(lbm_handle h) { return h && h->magic == kMagic; }

// ------------------------------------------------------------------ schedule

static void make_parts(lbm_ctx* h);

static void build_tiles(lbm_ctx* h) {
    const Shape& s = h->shape;
    h->ntiles = 0;
    h->ngroups = 0;
    h->tile_inst.clear();
    h->group_inst.clear();
    h->ptile_inst.clear();
    h->pgroup_inst.clear();
    h->npgroups = 0;
    for (size_t k = 0; k < h->inst.size(); ++k) {
        InstDesc& d = h->desc[k];
        const int tw = s.tile_w();
        d.tiles_x = (d.nx + tw - 1) / tw;
        const int tys = (d.ny + s.by - 1) / s.by;
        d.tile_begin = (int32_t)h->ntiles;
        d.ntiles = d.tiles_x * tys;
        h->ntiles += d.ntiles;
        h->tile_inst.insert(h->tile_inst.end(), (size_t)d.ntiles, (int32_t)k);
        d.group_begin = (int32_t)h->ngroups;
        d.ngroups = (d.ntiles + kGroup - 1) / kGroup;
        h->ngroups += d.ngroups;
        h->group_inst.insert(h->group_inst.end(), (size_t)d.ngroups, (int32_t)k);
        d.p_tiles_x = (int32_t)fused_tiles_x(h->inst[k], h->storage);
        d.p_tile_begin = (int32_t)h->ptile_inst.size();
        d.p_ntiles = d.p_tiles_x * ((d.ny + kMarchRows - 1) / kMarchRows);
        h->ptile_inst.insert(h->ptile_inst.end(), (size_t)d.p_ntiles, (int32_t)k);
        d.p_group_begin = (int32_t)h->npgroups;
        d.p_ngroups = (d.p_ntiles + kGroup - 1) / kGroup;
        h->npgroups += d.p_ngroups;
        h->pgroup_inst.insert(h->pgroup_inst.end(), (size_t)d.p_ngroups, (int32_t)k);
    }
    make_parts(h);
}

static lbm_ctx::Span span_of(const lbm_ctx* h, int i0, int i1, int ctr) {
    lbm_ctx::Span sp;
    sp.i0 = i0;
    sp.ni = i1 - i0;
    sp.ctr = ctr;
    if (i1 <= i0) return sp;
    const InstDesc& a = h->desc[i0];
    const InstDesc& b = h->desc[i1 - 1];
    sp.t0 = a.tile_begin;
    sp.nt = b.tile_begin + b.ntiles - a.tile_begin;
    sp.g0 = a.group_begin;
    sp.ng = b.group_begin + b.ngroups - a.group_begin;
    sp.pt0 = a.p_tile_begin;
    sp.pnt = b.p_tile_begin + b.p_ntiles - a.p_tile_begin;
    sp.pg0 = a.p_group_begin;
    sp.png = b.p_group_begin + b.p_ngroups - a.p_group_begin;
    return sp;
}

// The parts of the batched schedule: with two streams, two runs of
// consecutive instances holding about equal numbers of fused-kernel strips
// (their tiles and reduction groups are contiguous in the tables); the second
// part keeps its own step-counter pair (entries 4 and 5), copied from the
// handle's at every fork, so that its launches never read a counter that the
// first part's launches are advancing.
static void make_parts(lbm_ctx* h) {
    const int n = (int)h->inst.size();
    h->all = span_of(h, 0, n, 0);
    h->part[0] = h->all;
    h->nparts = 1;
    const int want = h->streams_req ? h->streams_req : (n >= 2 ? 2 : 1);
    if (want < 2 || n < 2) return;
    const int64_t total = (int64_t)h->ptile_inst.size();
    int64_t acc = 0, best = INT64_MAX;
    int cut = 1;
    for (int k = 1; k < n; ++k) {
        acc += h->desc[k - 1].p_ntiles;
        const int64_t dev = std::llabs(2 * acc - total);
        if (dev < best) {
            best = dev;
            cut = k;
        }
    }
    h->part[0] = span_of(h, 0, cut, 0);
    h->part[1] = span_of(h, cut, n, 4);
    h->nparts = 2;
}

// Descriptors and the tile table.  The reference states are not part of it:
// the device moves them at check steps, and a launch-shape change must not
// reset them (see upload_ref).
static int upload_tables(lbm_ctx* h) {
    HIPCALL(h, hipMemcpyAsync(h->d_desc(), h->desc.data(), h->desc.size() * sizeof(InstDesc),
                              hipMemcpyHostToDevice, h->stream));
    if (h->desc_saved) {
        // the saved descriptors follow the new tile tables too; only their
        // heat-flux terms are those of the last step
        h->desc_prev_host = h->desc;
        for (size_t k = 0; k < h->desc.size(); ++k)
            for (int w = 0; w < 4; ++w) h->desc_prev_host[k].wall_q[w] = h->wall_q_last[k][w];
        HIPCALL(h, hipMemcpyAsync(h->d_desc_prev(), h->desc_prev_host.data(), h->desc.size() * sizeof(InstDesc),
                                  hipMemcpyHostToDevice, h->stream));
    }
    HIPCALL(h, hipMemcpyAsync(h->d_tiles(), h->tile_inst.data(), h->tile_inst.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, h->stream));
    HIPCALL(h, hipMemcpyAsync(h->d_groups(), h->group_inst.data(), h->group_inst.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, h->stream));
    HIPCALL(h, hipMemcpyAsync(h->d_ptiles(), h->ptile_inst.data(), h->ptile_inst.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, h->stream));
    HIPCALL(h, hipMemcpyAsync(h->d_pgroups(), h->pgroup_inst.data(), h->pgroup_inst.size() * sizeof(int32_t),
                              hipMemcpyHostToDevice, h->stream));
    HIPCALL(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

// Reference state of instance k (see RefState).  Per step the ramp
// T_ref = t0 - G x feeds the flux share j_b = (5/9) C_V G (the first moment of
// omega_i C_V G c_ix), the relaxation multiplies the flux by rho and the rest
// of the non-equilibrium part by 1 - 1/tau; the ramp then sustains the
// non-equilibrium share (tau - 1) (1/27, -1/54) C_V G c_ix (axis / diagonal)
// and the bulk steady flux J = rho j_b / (1 - rho) = j_b (tau_r - 1/2), whose
// heat flux beta (J + j_b) is Fourier's (5/9) C_V G tau_r.
//   adaptive (check steps on, x periodic or gradient seam, no isothermal
//   y walls): J starts at -j_b (the reference carries no first moment, like
//   a state initialised without heat flux) and follows the mean flux;
//   otherwise J is the bulk steady flux (-j_b when tau_R is infinite: there
//   is no steady state, and the forcing j_b is the ramp's whole feed).
static void ref_init(lbm_ctx* h, size_t k, double s) {
    const lbm_instance& in = h->inst[k];
    const Coeffs& c = h->co[k];
    RefState& r = h->ref[k];
    std::memset(&r, 0, sizeof r);
    const double Gp = in.bc_x == LBM_BC_GRADIENT ? in.cv * in.grad_x : 0.0;
    r.jb = 5.0 / 9.0 * Gp;
    r.pa0 = 2.0 / 9.0 * Gp + (c.tau - 1.0) * Gp / 27.0;
    r.pd0 = Gp / 36.0 - (c.tau - 1.0) * Gp / 54.0;
    r.rho = c.rho;
    r.sigma = c.one_minus_rho;
    r.beta = c.beta;
    r.s = s;
    r.inv_nodes = 1.0 / ((double)in.nx * (double)in.ny);
    r.adapt = (h->K > 0 && (in.bc_x == LBM_BC_PERIODIC || in.bc_x == LBM_BC_GRADIENT) &&
               wall_kind(in, 2) != LBM_BC_ISOTHERMAL && wall_kind(in, 3) != LBM_BC_ISOTHERMAL) ? 1 : 0;
    const double J = (r.adapt || std::isinf(in.tau_r)) ? -r.jb : r.jb * (in.tau_r - 0.5);
    ref_set_flux(r, J);
}

// Kernel coefficients of instance k for the effective storage scale s.
static void fill_desc(lbm_ctx* h, size_t k, double s) {
    const lbm_instance& in = h->inst[k];
    const Coeffs& c = h->co[k];
    InstDesc& d = h->desc[k];
    d.inv_tau = (float)(1.0 / c.tau);
    d.sigma = (float)c.one_minus_rho;
    d.flux_a = (float)((1.0 / c.tau - c.one_minus_rho) / 3.0);
    d.flux_d = (float)((1.0 / c.tau - c.one_minus_rho) / 12.0);
    for (int w = 0; w < 4; ++w) d.wall_g[w] = (float)(in.cv * (in.t_wall[w] - in.t0) / s);
    for (int w = 0; w < 4; ++w) d.wall_q[w] = (float)(h->qwall[k][w] / (c.beta * s));
    d.s = s;
    d.cv = in.cv;
    d.s_cv = s / in.cv;
    d.s_beta = s * c.beta;
    ref_init(h, k, s);
}

// Reference state of instance k (k < 0: all) to the device.
static int upload_ref(lbm_ctx* h, int k) {
    const size_t first = k < 0 ? 0 : (size_t)k;
    const size_t n = k < 0 ? h->ref.size() : 1;
    HIPCALL(h, hipMemcpyAsync(h->d_ref() + first, h->ref.data() + first, n * sizeof(RefState),
                              hipMemcpyHostToDevice, h->stream));
    HIPCALL(h, hipMemcpyAsync(h->d_ref_prev() + first, h->ref.data() + first, n * sizeof(RefState),
                              hipMemcpyHostToDevice, h->stream));
    HIPCALL(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

// ------------------------------------------------------------------ static readout scratch
//
// Staging of lbm_moments_f64_noalloc: the FP64 fields of one instance, in a
// file-scope device array, so that the call allocates nothing.  Every device
// the library runs on holds one copy (24 MiB) until the process ends.  In
// host code `scratch` only names the symbol; its device address, per device,
// comes from hipGetSymbolAddress at lbm_create (once per device, with that
// device current) and only that address is passed to kernels and copies.

constexpr int64_t kNoAllocNodes = int64_t(1) << 20;   // largest instance the call reads out
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[3 * kNoAllocNodes];

namespace {
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}

// Resolve (once) the device address of `scratch` on the current device `dev`.
static hipError_t scratch_setup(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipSuccess;   // the no-allocation call reports it
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev]) return hipSuccess;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
    return hipSuccess;
}

static double* scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[dev];
}

// ------------------------------------------------------------------ C ABI

extern "C" {

const char* lbm_version(void) { return "phonon-lbm 0.1 (gfx950, D2Q8 Callaway dual relaxation)"; }

const char* lbm_last_error(lbm_handle h) {
    if (!h) return g_create_error.c_str();
    if (!valid(h)) return "invalid handle";
    return h->err.c_str();
}

static Status check_config(const lbm_config* cfg, std::vector<lbm_instance>* out) {
    if (!cfg) return {LBM_EINVAL, "config is NULL"};
    if (cfg->n_instances < 1 || !cfg->inst) return {LBM_EINVAL, "need n_instances >= 1 and inst != NULL"};
    if (cfg->storage < 0 || cfg->storage > 4)
        return {LBM_EINVAL, "storage must be LBM_F32, LBM_F16, LBM_BF16, LBM_F16_SPLIT or LBM_BF16_SPLIT"};
    if (is_split(cfg->storage) && cfg->layout == LBM_LAYOUT_PLANES)
        return {LBM_EUNSUPPORTED, "split storage uses the chunked layout only"};
    if (cfg->check_interval != 0 && cfg->check_interval != -1 && cfg->check_interval < 2)
        return {LBM_EINVAL, "check_interval must be 0 (default 100), -1 (off) or >= 2"};
    if (cfg->flags & ~(LBM_FLAG_EXTERNAL_MEMORY | LBM_FLAG_STOCHASTIC_ROUNDING | LBM_FLAG_ROUND_EVERY_STEP))
        return {LBM_EINVAL, "unknown flags"};
    if (cfg->layout < 0 || cfg->layout > 2)
        return {LBM_EINVAL, "layout must be LBM_LAYOUT_AUTO, _PLANES or _CHUNKED"};
    out->assign(cfg->inst, cfg->inst + cfg->n_instances);
    for (int k = 0; k < cfg->n_instances; ++k) {
        lbm_instance& in = (*out)[k];
        if (in.cv == 0.0) in.cv = 1.0;
        Status s = validate_instance(in, k);
        if (s.code) return s;
    }
    return {LBM_OK, ""};
}

static int check_of(const lbm_config* cfg) {
    return cfg->check_interval == 0 ? 100 : (cfg->check_interval < 0 ? 0 : cfg->check_interval);
}

int lbm_required_bytes(const lbm_config* cfg, size_t* bytes) {
    std::vector<lbm_instance> v;
    Status s = check_config(cfg, &v);
    if (s.code) {
        g_create_error = s.msg;
        return s.code;
    }
    if (!bytes) {
        g_create_error = "bytes is NULL";
        return LBM_EINVAL;
    }
    *bytes = layout_of(v, cfg->storage, check_of(cfg), resolve_layout(cfg->layout), every_step_of(cfg)).total;
    return LBM_OK;
}

int lbm_create(const lbm_config* cfg, lbm_handle* out) {
    g_create_error.clear();
    if (!out) {
        g_create_error = "out is NULL";
        return LBM_EINVAL;
    }
    std::vector<lbm_instance> v;
    Status s = check_config(cfg, &v);
    if (s.code) {
        g_create_error = s.msg;
        return s.code;
    }
    lbm_ctx* h = new (std::nothrow) lbm_ctx();
    if (!h) {
        g_create_error = "host allocation failed";
        return LBM_ENOMEM;
    }
    h->inst = v;
    h->storage = cfg->storage;
    h->K = check_of(cfg);
    h->stream = reinterpret_cast<hipStream_t>(cfg->stream);
    h->external = (cfg->flags & LBM_FLAG_EXTERNAL_MEMORY) != 0;
    h->sr = (cfg->flags & LBM_FLAG_STOCHASTIC_ROUNDING) ? 1 : 0;
    h->every_step = every_step_of(cfg);
    h->seed = cfg->seed;
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        g_create_error = std::string("hipGetDevice: ") + hipGetErrorString(e);
        delete h;
        return LBM_EHIP;
    }
    e = scratch_setup(h->device);
    if (e != hipSuccess) {
        g_create_error = std::string("hipGetSymbolAddress of the readout scratch: ") + hipGetErrorString(e);
        delete h;
        return LBM_EHIP;
    }
    const int es = esize_of(h->storage);
    h->layout = resolve_layout(cfg->layout);
    h->L = layout_of(v, h->storage, h->K, h->layout, h->every_step);
    h->desc.resize(v.size());
    h->ref.resize(v.size());
    h->qwall.assign(v.size(), std::array<double, 4>{0.0, 0.0, 0.0, 0.0});
    h->co.resize(v.size());
    h->inited.assign(v.size(), 0);
    size_t eoff = 0;
    int64_t noff = 0;
    for (size_t k = 0; k < v.size(); ++k) {
        InstDesc& d = h->desc[k];
        std::memset(&d, 0, sizeof d);
        const Geometry geo = geometry_of(v[k], es, h->layout, is_split(h->storage));
        d.nx = v[k].nx;
        d.ny = v[k].ny;
        d.bc_x = v[k].bc_x;
        d.bc_y = v[k].bc_y;
        for (int w = 0; w < 4; ++w) d.wk[w] = wall_kind(v[k], w);
        d.layout = h->layout;
        d.row = geo.row;
        d.plane = geo.plane;
        d.chunk = geo.chunk;
        d.cshift = geo.cshift;
        d.cmask = geo.cmask;
        d.off = (int64_t)eoff;
        d.node_off = noff;
        eoff += (size_t)geo.elems;
        noff += (int64_t)d.nx * d.ny;
        h->co[k] = coeffs_of(v[k]);
        fill_desc(h, k, v[k].scale > 0.0 ? v[k].scale : 1.0);
    }
    // default launch shape (fastest or within 0.1% of it on MI355X for an
    // 8192^2 lattice, FP32 and FP16, chunked layout): one node per lane with
    // the wavefront-per-row-segment kernel, 4 waves along x per block,
    // XCD-aware tile order
    h->shape.vec = 1;
    h->shape.bx = 256;
    h->shape.by = 1;
    h->shape.xcd = 1;
    h->shape.nt = 0;
    build_tiles(h);
    // steps per launch: the kind's most when the instances hold enough strips
    // of the fused kernel to fill the chip, else single steps.  Measured on
    // MI355X (FP32, us per step, single / six fused): 1024 x 256 4.5 / 12.2,
    // 1024^2 10.3 / 12.6 (640 strips), 2048 x 1024 17.7 / 14.4 (1280 strips),
    // 8192^2 741 / 213: a fused launch takes about one strip's marching time
    // however few strips there are.
    h->fuse = (int64_t)h->ptile_inst.size() >= kFuseMinStrips ? h->fuse_cap() : 1;
    default_costs(h->storage, h->every_step, h->cost_plain, h->cost_check);
    e = hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        g_create_error = std::string("hipStreamCreate: ") + hipGetErrorString(e);
        delete h;
        return LBM_EHIP;
    }
    if (!h->external) {
        e = hipMalloc(&h->base, h->L.total);
        if (e != hipSuccess) {
            g_create_error = std::string("hipMalloc of ") + std::to_string(h->L.total) +
                             " bytes: " + hipGetErrorString(e);
            (void)hipStreamDestroy(h->capture_stream);
            delete h;
            return e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EHIP;
        }
        h->owned = true;
        int rc = upload_tables(h);
        if (!rc) rc = upload_ref(h, -1);
        if (rc) {
            g_create_error = h->err;
            (void)hipFree(h->base);
            (void)hipStreamDestroy(h->capture_stream);
            delete h;
            return rc;
        }
    }
    *out = h;
    return LBM_OK;
}

int lbm_bind(lbm_handle h, void* device_buf, size_t bytes) {
    if (!valid(h)) return LBM_EINVAL;
    if (!h->external) return h->fail(LBM_ESTATE, "handle owns its memory (created without LBM_FLAG_EXTERNAL_MEMORY)");
    if (h->base) return h->fail(LBM_ESTATE, "memory already bound");
    if (!device_buf || bytes < h->L.total)
        return h->fail(LBM_EINVAL, "buffer NULL or smaller than lbm_required_bytes (" +
                                       std::to_string(h->L.total) + ")");
    if (reinterpret_cast<uintptr_t>(device_buf) % kAlign)
        return h->fail(LBM_EINVAL, "buffer must be 256-byte aligned");
    h->base = static_cast<char*>(device_buf);
    const int rc = upload_tables(h);
    return rc ? rc : upload_ref(h, -1);
}

void lbm_destroy(lbm_handle h) {
    if (!valid(h)) return;
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    else (void)hipDeviceSynchronize();
    // the second part's launches before the memory goes (every lbm_step call
    // joins them into the handle's stream; this also covers a call that failed)
    if (h->part_stream) (void)hipStreamSynchronize(h->part_stream);
    h->drop_graphs();
    if (h->owned && h->base) (void)hipFree(h->base);
    if (h->staging) (void)hipFree(h->staging);
    if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
    if (h->part_stream) (void)hipStreamDestroy(h->part_stream);
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
    if (h->ev_join) (void)hipEventDestroy(h->ev_join);
    if (h->cap_part_stream) (void)hipStreamDestroy(h->cap_part_stream);
    if (h->cap_fork) (void)hipEventDestroy(h->cap_fork);
    if (h->cap_join) (void)hipEventDestroy(h->cap_join);
    h->magic = 0;
    delete h;
}

static int ensure_staging(lbm_ctx* h, size_t bytes) {
    if (h->staging_bytes >= bytes) return LBM_OK;
    if (h->staging) {
        HIPCALL(h, hipStreamSynchronize(h->stream));
        (void)hipFree(h->staging);
        h->staging = nullptr;
        h->staging_bytes = 0;
    }
    hipError_t e = hipMalloc(&h->staging, bytes);
    if (e != hipSuccess) return h->fail(e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EHIP,
                                        std::string("staging hipMalloc: ") + hipGetErrorString(e));
    h->staging_bytes = bytes;
    return LBM_OK;
}

static int check_inst(lbm_ctx* h, int32_t k) {
    if (k < 0 || k >= (int32_t)h->inst.size())
        return h->fail(LBM_EINVAL, "instance index out of range");
    if (!h->base) return h->fail(LBM_ESTATE, "no device memory bound");
    return LBM_OK;
}

// Automatic storage scale: FP16 keeps the largest expected |g| near 2^12 or
// below, far under its 65504 limit and well above its normal range floor.
static double auto_scale(const lbm_ctx* h, const lbm_instance& in, double amp) {
    if (!is_f16(h->storage)) return 1.0;
    for (int w = 0; w < 4; ++w)
        if (wall_kind(in, w) == LBM_BC_ISOTHERMAL) amp = std::max(amp, std::fabs(in.t_wall[w] - in.t0));
    if (in.bc_x == LBM_BC_GRADIENT) {
        const double tr = std::isinf(in.tau_r) ? 1e6 : in.tau_r;
        amp = std::max(amp, 5.0 / 9.0 * in.cv * std::fabs(in.grad_x) * std::max(tr, 1.0));
    }
    if (!(amp > 0.0) || !std::isfinite(amp)) return 1.0;
    return std::ldexp(1.0, (int)std::ceil(std::log2(amp)) - 13);
}

static int do_init(lbm_ctx* h, int32_t k, const double* dT, const double* dqx, const double* dqy) {
    const lbm_instance& in = h->inst[k];
    const InstDesc& d = h->desc[k];
    HIPCALL(h, hipMemcpyAsync(h->d_desc(), h->desc.data(), h->desc.size() * sizeof(InstDesc),
                              hipMemcpyHostToDevice, h->stream));
    HIPCALL(h, hipMemcpyAsync(h->d_ref() + k, &h->ref[k], sizeof(RefState), hipMemcpyHostToDevice,
                              h->stream));
    HIPCALL(h, hipMemcpyAsync(h->d_ref_prev() + k, &h->ref[k], sizeof(RefState), hipMemcpyHostToDevice,
                              h->stream));
    const double grad = in.bc_x == LBM_BC_GRADIENT ? in.grad_x : 0.0;
    HIPCALL(h, launch_init(h->storage, h->d_desc(), h->d_ref(), k, d, h->buf(1 - h->cur), h->buf(h->cur),
                           dT, dqx, dqy, in.t0, grad, h->co[k].beta, h->stream));
    HIPCALL(h, hipMemsetAsync(h->d_ctr(), 0, 2 * sizeof(uint32_t), h->stream));
    HIPCALL(h, hipStreamSynchronize(h->stream));
    if (h->steps != 0) {
        // the handle restarts at n = 0: every other instance must be re-initialised
        std::fill(h->inited.begin(), h->inited.end(), 0);
        h->steps = 0;
    }
    h->last_check = -1;
    h->inited[k] = 1;
    h->tail = lbm_ctx::Tail();
    h->replayed = false;
    h->desc_saved = false;
    h->drop_graphs();
    return LBM_OK;
}

int lbm_init(lbm_handle h, int32_t k, const double* T, const double* qx, const double* qy) {
    if (!valid(h)) return LBM_EINVAL;
    int rc = check_inst(h, k);
    if (rc) return rc;
    const lbm_instance& in = h->inst[k];
    const size_t n = (size_t)in.nx * in.ny;
    const double grad = in.bc_x == LBM_BC_GRADIENT ? in.grad_x : 0.0;
    std::vector<double> tmp;
    if (!T) {
        tmp.resize(n);
        for (int y = 0; y < in.ny; ++y)
            for (int x = 0; x < in.nx; ++x) tmp[(size_t)y * in.nx + x] = in.t0 - grad * x;
        T = tmp.data();
    }
    double amp = 0.0;
    for (int y = 0; y < in.ny; ++y)
        for (int x = 0; x < in.nx; ++x) {
            const size_t i = (size_t)y * in.nx + x;
            const double v = T[i] - (in.t0 - grad * x);
            const double a = std::max({std::fabs(v), qx ? std::fabs(qx[i]) : 0.0, qy ? std::fabs(qy[i]) : 0.0});
            if (!std::isfinite(a)) return h->fail(LBM_EINVAL, "non-finite initial field");
            amp = std::max(amp, a);
        }
    fill_desc(h, k, in.scale > 0.0 ? in.scale : auto_scale(h, in, amp));
    rc = ensure_staging(h, 3 * n * sizeof(double));
    if (rc) return rc;
    HIPCALL(h, hipMemcpyAsync(h->staging, T, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
    const double* dqx = nullptr;
    const double* dqy = nullptr;
    if (qx) {
        HIPCALL(h, hipMemcpyAsync(h->staging + n, qx, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
        dqx = h->staging + n;
    }
    if (qy) {
        HIPCALL(h, hipMemcpyAsync(h->staging + 2 * n, qy, n * sizeof(double), hipMemcpyHostToDevice, h->stream));
        dqy = h->staging + 2 * n;
    }
    return do_init(h, k, h->staging, dqx, dqy);
}

int lbm_init_device(lbm_handle h, int32_t k, const double* T, const double* qx, const double* qy) {
    if (!valid(h)) return LBM_EINVAL;
    int rc = check_inst(h, k);
    if (rc) return rc;
    if (!T) return h->fail(LBM_EINVAL, "T is NULL (device init needs a temperature field)");
    const lbm_instance& in = h->inst[k];
    if (is_f16(h->storage) && in.scale == 0.0)
        return h->fail(LBM_EINVAL, "FP16 storage with device init needs an explicit scale");
    fill_desc(h, k, in.scale > 0.0 ? in.scale : 1.0);
    return do_init(h, k, T, qx, qy);
}

int64_t lbm_steps_done(lbm_handle h) { return valid(h) ? h->steps : -1; }

static int mode_of(const lbm_ctx* h, int64_t m) {
    if (!h->K) return kPlain;
    if (m % h->K == 0) return kCheck;
    if ((m + 1) % h->K == 0) return kSnap;
    return kPlain;
}

// Issue step number m (1-based) of the instances of `sp` on stream st reading
// buffer `src_k`.
static int issue_step(lbm_ctx* h, int64_t m, int src_k, hipStream_t st, int sched, const lbm_ctx::Span& sp) {
    const int mode = mode_of(h, m);
    StepArgs a;
    a.desc = h->d_desc();
    a.tile_inst = h->d_tiles();
    a.src = h->buf(src_k);
    a.dst = h->buf(1 - src_k);
    a.snap = h->d_snap();
    a.partials = h->d_part();
    a.ctr_in = h->d_ctr() + sp.ctr + src_k;
    a.ctr_out = h->d_ctr() + sp.ctr + (1 - src_k);
    a.seed = h->seed;
    a.sr = h->sr;
    a.ref = h->d_ref();
    // the step after a check step applies the reference shift that the check
    // step's finalisation set (zero for non-adaptive instances and at n = 0)
    a.apply_shift = (h->K > 0 && (m - 1) % h->K == 0) ? 1 : 0;
    if (sched == LBM_SCHED_PER_INSTANCE) {
        for (int k = sp.i0; k < sp.i0 + sp.ni; ++k) {
            a.tile_base = h->desc[k].tile_begin;
            a.ntiles = h->desc[k].ntiles;
            HIPCALL(h, launch_step(h->storage, h->shape, mode, a, h->L.nodes, st));
        }
    } else {
        a.tile_base = sp.t0;
        a.ntiles = sp.nt;
        HIPCALL(h, launch_step(h->storage, h->shape, mode, a, h->L.nodes, st));
    }
    if (mode == kCheck)
        HIPCALL(h, launch_finalize(h->d_desc(), h->d_groups(), sp.g0, sp.ng, h->d_ref(), h->d_ref_prev(), sp.i0,
                                   sp.ni, h->d_part(), h->d_gpart(), h->d_res(), 0, st));
    return LBM_OK;
}

// Cheapest cover of r steps by plain launches of 1 .. kmax steps: g[n] for
// n = 0 .. r, and first[n], the length of a first launch of an optimal cover.
static void plain_covers(const double* cost, int kmax, int r, double* g, int* first) {
    g[0] = 0.0;
    first[0] = 0;
    for (int n = 1; n <= r; ++n) {
        g[n] = 1e300;
        first[n] = 1;
        for (int k = 1; k <= std::min(kmax, n); ++k) {
            const double v = cost[k] + g[n - k];
            if (v < g[n]) {
                g[n] = v;
                first[n] = k;
            }
        }
    }
}

// Steps the launch that starts at step m covers, in a sequence of steps that
// ends at step `last`.  The sequence is cut into segments that end on a check
// step (whose residual and totals the fused kernel then forms: *end =
// kEndCheck) or on `last`; a segment is covered by launches of at most
// h->fuse steps, the one that reaches a check step last, chosen to minimise
// the summed launch costs (cost_plain, cost_check) over the segment's last
// few launches; longer segments start with launches of h->fuse steps.  A run
// that ends on the snapshot step before a check step (a call ending there)
// writes the snapshot for the single check step that follows: *end =
// kEndSnap.  Returns 1 for a single-step launch.
static int plan_launch(const lbm_ctx* h, int64_t m, int64_t last, int* end) {
    *end = kEndPlain;
    const int kmax = h->fuse;
    if (kmax < 2) return 1;
    int64_t seg = last;
    bool to_check = false;
    if (h->K) {
        const int64_t c = (m + h->K - 1) / h->K * h->K;     // first check step >= m
        if (c <= seg) {
            seg = c;
            to_check = true;
        }
    }
    const int64_t r64 = seg - m + 1;
    int k = kmax;
    const int tail = 8 * kmax;        // the last steps of a segment are planned exactly
    if (r64 <= tail) {
        const int r = (int)r64;
        double g[8 * 8 + 1];
        int first[8 * 8 + 1];
        plain_covers(h->cost_plain, kmax, r, g, first);
        if (!to_check || r < 2) {
            k = first[r];
        } else {
            // the launch that reaches the check step is a fused check launch
            double best = 1e300;
            int klast = 2;
            for (int kl = 2; kl <= std::min(kmax, r); ++kl) {
                const double v = h->cost_check[kl] + g[r - kl];
                if (v < best) {
                    best = v;
                    klast = kl;
                }
            }
            k = (r == klast) ? klast : first[r - klast];
        }
    }
    if (k < 2) return 1;
    const int mode = mode_of(h, m + k - 1);
    *end = mode == kCheck ? kEndCheck : (mode == kSnap ? kEndSnap : kEndPlain);
    return k;
}

static int issue_fused(lbm_ctx* h, int64_t m, int nsteps, int end, int src_k, hipStream_t st,
                       const lbm_ctx::Span& sp) {
    StepArgs a;
    a.desc = h->d_desc();
    a.tile_inst = h->d_ptiles();
    a.src = h->buf(src_k);
    a.dst = h->buf(1 - src_k);
    a.snap = h->d_snap();
    a.partials = h->d_part();
    a.ctr_in = h->d_ctr() + sp.ctr + src_k;
    a.ctr_out = h->d_ctr() + sp.ctr + (1 - src_k);
    a.seed = h->seed;
    a.sr = h->sr;
    a.ref = h->d_ref();
    a.apply_shift = (h->K > 0 && (m - 1) % h->K == 0) ? 1 : 0;
    a.tile_base = sp.pt0;
    a.ntiles = sp.pnt;
    HIPCALL(h, launch_fused(h->storage, h->shape, a, nsteps, end, h->layout == LBM_LAYOUT_CHUNKED,
                            h->every_step ? kRoundEvery : kRoundLast, h->L.nodes, st));
    if (end == kEndCheck)
        HIPCALL(h, launch_finalize(h->d_desc(), h->d_pgroups(), sp.pg0, sp.png, h->d_ref(), h->d_ref_prev(), sp.i0,
                                   sp.ni, h->d_part(), h->d_gpart(), h->d_res(), 1, st));
    return LBM_OK;
}

// Stream `side` (the second part's) waits for everything issued on `main`
// so far, its step counters starting from the handle's; join: `main` waits
// for everything issued on `side`.  The events and `side` are created at first
// use.  Also used under graph capture (with a stream and events of its own).
static int fork_parts(lbm_ctx* h, hipStream_t main, hipStream_t* side, hipEvent_t* fork, hipEvent_t* join) {
    if (!*side) HIPCALL(h, hipStreamCreateWithFlags(side, hipStreamNonBlocking));
    if (!*fork) HIPCALL(h, hipEventCreateWithFlags(fork, hipEventDisableTiming));
    if (!*join) HIPCALL(h, hipEventCreateWithFlags(join, hipEventDisableTiming));
    HIPCALL(h, launch_copy_u32(h->d_ctr() + h->part[1].ctr, h->d_ctr(), 2, main));
    HIPCALL(h, hipEventRecord(*fork, main));
    HIPCALL(h, hipStreamWaitEvent(*side, *fork, 0));
    return LBM_OK;
}

static int join_parts(lbm_ctx* h, hipStream_t main, hipStream_t side, hipEvent_t join) {
    HIPCALL(h, hipEventRecord(join, side));
    HIPCALL(h, hipStreamWaitEvent(main, join, 0));
    return LBM_OK;
}

static int chunk_of(const lbm_ctx* h) { return h->K ? h->K : 64; }

// Capture one chunk of steps starting at a multiple of the chunk with
// buffer parity `par` (the index of the buffer holding the current state).
static int capture(lbm_ctx* h, int par) {
    const int C = chunk_of(h);
    // the parts of the batched schedule become two branches of the graph
    const bool multi = h->nparts > 1;
    if (multi) {
        // created before the capture begins (fork_parts finds them)
        if (!h->cap_part_stream) HIPCALL(h, hipStreamCreateWithFlags(&h->cap_part_stream, hipStreamNonBlocking));
        if (!h->cap_fork) HIPCALL(h, hipEventCreateWithFlags(&h->cap_fork, hipEventDisableTiming));
        if (!h->cap_join) HIPCALL(h, hipEventCreateWithFlags(&h->cap_join, hipEventDisableTiming));
    }
    HIPCALL(h, hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal));
    int src = par;
    int rc = LBM_OK;
    if (multi) rc = fork_parts(h, h->capture_stream, &h->cap_part_stream, &h->cap_fork, &h->cap_join);
    const int np = multi ? h->nparts : 1;
    int flips = 0;
    lbm_ctx::Tail tail;
    int tail_flip = 0;
    for (int s = 1; s <= C && rc == LBM_OK;) {
        int end = kEndPlain;
        const int k = plan_launch(h, s, C, &end);
        tail = lbm_ctx::Tail();
        tail_flip = flips & 1;
        for (int p = 0; p < np && rc == LBM_OK; ++p) {
            hipStream_t st = p == 0 ? h->capture_stream : h->cap_part_stream;
            const lbm_ctx::Span& sp = multi ? h->part[p] : h->all;
            rc = k >= 2 ? issue_fused(h, (int64_t)s, k, end, src, st, sp)
                        : issue_step(h, (int64_t)s, src, st, LBM_SCHED_BATCHED, sp);
        }
        if (k >= 2) {
            tail.k = k;
            tail.apply_shift = (h->K > 0 && (s - 1) % h->K == 0) ? 1 : 0;
            tail.checked = end == kEndCheck ? 1 : 0;
        }
        s += k;
        src = 1 - src;
        ++flips;
    }
    if (multi && rc == LBM_OK) rc = join_parts(h, h->capture_stream, h->cap_part_stream, h->cap_join);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->capture_stream, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return h->hip_fail(e, "hipStreamEndCapture");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return h->hip_fail(e, "hipGraphInstantiate");
    }
    h->graph[par] = g;
    h->gexec[par] = x;
    h->graph_chunk = C;
    h->graph_flips = flips;
    h->graph_tail = tail;
    h->graph_tail_flip = tail_flip;
    return LBM_OK;
}

static int step_loop(lbm_ctx* h, int64_t nsteps, bool multi) {
    const int np = multi ? h->nparts : 1;
    auto stream_of = [&](int p) { return p == 0 ? h->stream : h->part_stream; };
    auto span_of_part = [&](int p) -> const lbm_ctx::Span& { return multi ? h->part[p] : h->all; };
    int64_t left = nsteps;
    while (left > 0) {
        const int C = chunk_of(h);
        if (h->sched == LBM_SCHED_GRAPH && h->steps % C == 0 && left >= C) {
            const int par = h->cur;
            if (!h->gexec[par]) {
                int rc = capture(h, par);
                if (rc) return rc;
            }
            HIPCALL(h, hipGraphLaunch(h->gexec[par], h->stream));
            h->steps += C;
            if (h->graph_flips & 1) h->cur = 1 - h->cur;
            if (h->K) h->last_check = h->steps;
            h->tail = h->graph_tail;
            h->tail.src = par ^ h->graph_tail_flip;
            left -= C;
            continue;
        }
        const int64_t m = h->steps + 1;
        const int sched = h->sched == LBM_SCHED_PER_INSTANCE ? LBM_SCHED_PER_INSTANCE : LBM_SCHED_BATCHED;
        // the per-instance schedule issues single steps: one instance's fused
        // launch holds too few wavefronts to hide the marching latency
        // (Knudsen sweep: 4.0k MLUPS at five steps per launch, 17.1k single)
        int end = kEndPlain;
        const int k = sched == LBM_SCHED_PER_INSTANCE ? 1 : plan_launch(h, m, h->steps + left, &end);
        h->tail = lbm_ctx::Tail();
        if (k >= 2) {
            for (int p = 0; p < np; ++p) {
                int rc = issue_fused(h, m, k, end, h->cur, stream_of(p), span_of_part(p));
                if (rc) return rc;
            }
            h->tail.k = k;
            h->tail.src = h->cur;
            h->tail.apply_shift = (h->K > 0 && (m - 1) % h->K == 0) ? 1 : 0;
            h->tail.checked = end == kEndCheck ? 1 : 0;
            if (end == kEndCheck) h->last_check = m + k - 1;
            h->cur = 1 - h->cur;
            h->steps = m + k - 1;
            left -= k;
            continue;
        }
        for (int p = 0; p < np; ++p) {
            int rc = issue_step(h, m, h->cur, stream_of(p), sched, span_of_part(p));
            if (rc) return rc;
        }
        if (mode_of(h, m) == kCheck) h->last_check = m;
        h->cur = 1 - h->cur;
        h->steps = m;
        --left;
    }
    return LBM_OK;
}

int lbm_step(lbm_handle h, int64_t nsteps) {
    if (!valid(h)) return LBM_EINVAL;
    if (nsteps < 0) return h->fail(LBM_EINVAL, "nsteps < 0");
    if (!h->base) return h->fail(LBM_ESTATE, "no device memory bound");
    for (char c : h->inited)
        if (!c) return h->fail(LBM_ESTATE, "every instance must be initialised before lbm_step");
    if (nsteps > 0) {
        // the readout buffer and the descriptor copy describe the last step so far
        h->replayed = false;
        h->desc_saved = false;
    }
    if (nsteps > 0 && !h->preloaded) {
        HIPCALL(h, preload_fused(h->storage, h->sr, h->layout == LBM_LAYOUT_CHUNKED, h->every_step, h->stream));
        h->preloaded = true;
    }
    // the batched schedule spreads the instances over the parts' streams
    const bool multi = nsteps > 0 && h->nparts > 1 && h->sched == LBM_SCHED_BATCHED;
    if (multi) {
        const int rc = fork_parts(h, h->stream, &h->part_stream, &h->ev_fork, &h->ev_join);
        if (rc) return rc;
    }
    int rc = step_loop(h, nsteps, multi);
    if (multi) {
        const int rj = join_parts(h, h->stream, h->part_stream, h->ev_join);
        if (!rc) rc = rj;
    }
    return rc;
}

// Rebuild, in the readout buffer, the post-relaxation state of step n - 1
// after a last launch of k >= 2 steps (see lbm_ctx::Tail): steps n - k + 1 ..
// n - 1 again from the launch's source buffer, with the descriptors and the
// reference state that launch ran with and the stochastic-rounding counter it
// started from.  Same arithmetic, so the same bits as the original steps.
// 16-bit storage rounding only the last step of a launch (kRoundLast): that
// launch's state of step n - 1 never existed in the storage type, so the
// whole launch is replayed instead, ending with kEndMoments: the FP64 moments
// of its step-n nodes go to the readout buffer (as planes laid out like the
// snapshot), from the same registers the launch itself relaxed.
static int replay_tail(lbm_ctx* h) {
    const lbm_ctx::Tail& t = h->tail;
    StepArgs a;
    a.desc = h->d_desc_last();
    a.src = h->buf(t.src);
    a.dst = h->buf(lbm_ctx::kReadout);
    a.snap = nullptr;
    a.partials = nullptr;
    a.ctr_in = h->d_ctr() + t.src;
    a.ctr_out = h->d_ctr() + lbm_ctx::kReadout;
    a.seed = h->seed;
    a.sr = h->sr;
    // a launch that ended on a check step ran before the reference moved
    a.ref = t.checked ? h->d_ref_prev() : h->d_ref();
    a.apply_shift = t.apply_shift;
    a.tile_base = 0;
    if (!h->every_step) {
        a.snap = reinterpret_cast<double*>(h->buf(lbm_ctx::kReadout));
        a.tile_inst = h->d_ptiles();
        a.ntiles = (int32_t)h->ptile_inst.size();
        HIPCALL(h, launch_fused(h->storage, h->shape, a, t.k, kEndMoments, h->layout == LBM_LAYOUT_CHUNKED,
                                kRoundLast, h->L.nodes, h->stream));
    } else if (t.k - 1 >= 2) {
        a.tile_inst = h->d_ptiles();
        a.ntiles = (int32_t)h->ptile_inst.size();
        HIPCALL(h, launch_fused(h->storage, h->shape, a, t.k - 1, kEndPlain, h->layout == LBM_LAYOUT_CHUNKED,
                                kRoundEvery, h->L.nodes, h->stream));
    } else {
        a.tile_inst = h->d_tiles();
        a.ntiles = (int32_t)h->ntiles;
        HIPCALL(h, launch_step(h->storage, h->shape, kPlain, a, h->L.nodes, h->stream));
    }
    h->replayed = true;
    return LBM_OK;
}

static int run_moments(lbm_ctx* h, int32_t k, int out_kind, void* T, void* qx, void* qy, DD* partials) {
    const lbm_instance& in = h->inst[k];
    const double grad = in.bc_x == LBM_BC_GRADIENT ? in.grad_x : 0.0;
    // after a check step the reference has moved and its shift is still pending
    const int pending = (h->K > 0 && h->steps > 0 && h->steps % h->K == 0) ? 1 : 0;
    // the post-relaxation state of step n - 1: the buffer the last step read,
    // or (after a fused last launch) the readout buffer, replayed once
    int src = 1 - h->cur;
    if (h->steps > 0 && h->tail.k >= 2) {
        if (!h->replayed) {
            int rc = replay_tail(h);
            if (rc) return rc;
        }
        if (!h->every_step) {
            HIPCALL(h, launch_plane_moments(h->d_desc_last(), k, h->desc[k],
                                            reinterpret_cast<const double*>(h->buf(lbm_ctx::kReadout)), h->L.nodes,
                                            out_kind, T, qx, qy, in.t0, grad, partials, h->stream));
            return LBM_OK;
        }
        src = lbm_ctx::kReadout;
    }
    HIPCALL(h, launch_moments(h->storage, h->d_desc_last(), h->d_ref(), k, h->desc[k], h->buf(src),
                              h->steps > 0 ? 1 : 0, pending, out_kind, T, qx, qy, in.t0, grad, partials,
                              h->stream));
    return LBM_OK;
}

static int moments_common(lbm_handle h, int32_t k, int out_kind, void* T, void* qx, void* qy, int on_device) {
    if (!valid(h)) return LBM_EINVAL;
    int rc = check_inst(h, k);
    if (rc) return rc;
    if (!h->inited[k]) return h->fail(LBM_ESTATE, "instance not initialised");
    const lbm_instance& in = h->inst[k];
    const size_t n = (size_t)in.nx * in.ny;
    const size_t es = out_kind == 0 ? sizeof(float) : sizeof(double);
    if (on_device) {
        rc = run_moments(h, k, out_kind, T, qx, qy, nullptr);
        if (rc) return rc;
        HIPCALL(h, hipStreamSynchronize(h->stream));
        return LBM_OK;
    }
    rc = ensure_staging(h, 3 * n * sizeof(double));
    if (rc) return rc;
    char* st = reinterpret_cast<char*>(h->staging);
    void* dv[3] = {T ? st : nullptr, qx ? st + n * es : nullptr, qy ? st + 2 * n * es : nullptr};
    rc = run_moments(h, k, out_kind, dv[0], dv[1], dv[2], nullptr);
    if (rc) return rc;
    void* hv[3] = {T, qx, qy};
    for (int c = 0; c < 3; ++c)
        if (hv[c]) HIPCALL(h, hipMemcpyAsync(hv[c], dv[c], n * es, hipMemcpyDeviceToHost, h->stream));
    HIPCALL(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm_moments(lbm_handle h, int32_t k, float* T, float* qx, float* qy, int32_t on_device) {
    return moments_common(h, k, 0, T, qx, qy, on_device);
}

int lbm_moments_f64(lbm_handle h, int32_t k, double* dT, double* qx, double* qy, int32_t on_device) {
    return moments_common(h, k, 1, dT, qx, qy, on_device);
}

int lbm_moments_f64_noalloc(lbm_handle h, int32_t k, double* dT, double* qx, double* qy) {
    if (!valid(h)) return LBM_EINVAL;
    int rc = check_inst(h, k);
    if (rc) return rc;
    if (!h->inited[k]) return h->fail(LBM_ESTATE, "instance not initialised");
    const lbm_instance& in = h->inst[k];
    const int64_t n = (int64_t)in.nx * in.ny;
    if (n > kNoAllocNodes)
        return h->fail(LBM_EINVAL, "instance of " + std::to_string(n) + " nodes: lbm_moments_f64_noalloc reads out "
                                   "at most " + std::to_string(kNoAllocNodes) + " nodes (use lbm_moments_f64)");
    double* sp = scratch_ptr(h->device);
    if (!sp) return h->fail(LBM_EUNSUPPORTED, "no readout scratch on this device");
    double* dv[3] = {dT ? sp : nullptr, qx ? sp + n : nullptr, qy ? sp + 2 * n : nullptr};
    rc = run_moments(h, k, 1, dv[0], dv[1], dv[2], nullptr);
    if (rc) return rc;
    double* hv[3] = {dT, qx, qy};
    for (int c = 0; c < 3; ++c)
        if (hv[c]) HIPCALL(h, hipMemcpyAsync(hv[c], dv[c], (size_t)n * sizeof(double), hipMemcpyDeviceToHost,
                                             h->stream));
    HIPCALL(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm_totals(lbm_handle h, int32_t k, double out[3]) {
    if (!valid(h)) return LBM_EINVAL;
    int rc = check_inst(h, k);
    if (rc) return rc;
    if (!out) return h->fail(LBM_EINVAL, "out is NULL");
    if (!h->inited[k]) return h->fail(LBM_ESTATE, "instance not initialised");
    rc = run_moments(h, k, 1, nullptr, nullptr, nullptr, h->d_mpart());
    if (rc) return rc;
    const InstDesc& d = h->desc[k];
    const int nparts = ((d.nx + 255) / 256) * d.ny;
    HIPCALL(h, launch_finalize_range(h->d_mpart(), nparts, h->d_gpart(), h->d_mres(), h->stream));
    DD r[kPartials];
    HIPCALL(h, hipMemcpyAsync(r, h->d_mres(), sizeof r, hipMemcpyDeviceToHost, h->stream));
    HIPCALL(h, hipStreamSynchronize(h->stream));
    for (int c = 0; c < 3; ++c) out[c] = r[c].hi;
    for (int c = 0; c < 3; ++c)
        if (!std::isfinite(out[c])) return h->fail(LBM_ENONFINITE, "non-finite total");
    return LBM_OK;
}

int lbm_last_check(lbm_handle h, int32_t k, lbm_check_info* out) {
    if (!valid(h)) return LBM_EINVAL;
    int rc = check_inst(h, k);
    if (rc) return rc;
    if (!out) return h->fail(LBM_EINVAL, "out is NULL");
    if (h->last_check < 0) return h->fail(LBM_ESTATE, "no check step yet");
    double r[kPartials];
    HIPCALL(h, hipMemcpyAsync(r, h->d_res() + (size_t)k * kPartials, sizeof r, hipMemcpyDeviceToHost, h->stream));
    HIPCALL(h, hipStreamSynchronize(h->stream));
    out->step = h->last_check;
    out->totals[0] = r[0];
    out->totals[1] = r[1];
    out->totals[2] = r[2];
    out->residual = r[4] > 0.0 ? std::sqrt(r[3] / r[4]) : (r[3] == 0.0 ? 0.0 : INFINITY);
    for (double v : r)
        if (!std::isfinite(v)) return h->fail(LBM_ENONFINITE, "non-finite value in the check reduction");
    return LBM_OK;
}

int lbm_residual(lbm_handle h, int32_t k, double* r) {
    if (!valid(h)) return LBM_EINVAL;
    if (!r) return h->fail(LBM_EINVAL, "r is NULL");
    lbm_check_info ci;
    int rc = lbm_last_check(h, k, &ci);
    if (rc && rc != LBM_ENONFINITE) return rc;
    *r = ci.residual;
    return rc;
}

int lbm_coefficients(lbm_handle h, int32_t k, double out[6]) {
    if (!valid(h)) return LBM_EINVAL;
    if (k < 0 || k >= (int32_t)h->inst.size()) return h->fail(LBM_EINVAL, "instance index out of range");
    if (!out) return h->fail(LBM_EINVAL, "out is NULL");
    const InstDesc& d = h->desc[k];
    const Coeffs& c = h->co[k];
    out[0] = d.inv_tau;
    out[1] = (float)c.beta;
    out[2] = d.sigma;
    out[3] = d.s;
    out[4] = c.tau;
    out[5] = c.rho;
    return LBM_OK;
}

int lbm_set_wall_flux(lbm_handle h, int32_t k, int32_t wall, double q0) {
    if (!valid(h)) return LBM_EINVAL;
    int rc = check_inst(h, k);
    if (rc) return rc;
    if (wall < 0 || wall > 3) return h->fail(LBM_EINVAL, "wall must be 0..3 (x=0, x=nx-1, y=0, y=ny-1)");
    const lbm_instance& in = h->inst[k];
    if (wall_kind(in, wall) != LBM_BC_HEATFLUX)
        return h->fail(LBM_EINVAL, "wall is not a HEATFLUX wall");
    if (!std::isfinite(q0)) return h->fail(LBM_EINVAL, "q0 must be finite");
    // readouts of the current time keep the descriptors its last step ran with
    if (h->steps > 0 && !h->desc_saved) {
        HIPCALL(h, hipMemcpyAsync(h->d_desc_prev(), h->d_desc(), h->desc.size() * sizeof(InstDesc),
                                  hipMemcpyDeviceToDevice, h->stream));
        h->wall_q_last.resize(h->desc.size());
        for (size_t j = 0; j < h->desc.size(); ++j)
            for (int w = 0; w < 4; ++w) h->wall_q_last[j][w] = h->desc[j].wall_q[w];
        h->desc_saved = true;
    }
    h->qwall[k][wall] = q0;
    InstDesc& d = h->desc[k];
    d.wall_q[wall] = (float)(q0 / (h->co[k].beta * d.s));
    HIPCALL(h, launch_set_float(&h->d_desc()[k].wall_q[wall], d.wall_q[wall], h->stream));
    return LBM_OK;
}

int lbm_set_step_fusion(lbm_handle h, int32_t steps) {
    if (!valid(h)) return LBM_EINVAL;
    if (steps < 1 || steps > h->fuse_cap())
        return h->fail(LBM_EINVAL, "steps per launch must be 1 .. " + std::to_string(h->fuse_cap()) +
                                       " for this storage kind");
    h->fuse = steps;
    h->drop_graphs();
    return LBM_OK;
}

int32_t lbm_get_step_fusion(lbm_handle h) { return valid(h) ? h->fuse : -1; }

int32_t lbm_max_step_fusion(int32_t storage) {
    return (storage >= LBM_F32 && storage <= LBM_BF16_SPLIT) ? fuse_max(storage) : -1;
}

int lbm_set_schedule(lbm_handle h, int32_t schedule) {
    if (!valid(h)) return LBM_EINVAL;
    if (schedule < 0 || schedule > 2) return h->fail(LBM_EINVAL, "unknown schedule");
    h->sched = schedule;
    return LBM_OK;
}

int lbm_set_streams(lbm_handle h, int32_t n) {
    if (!valid(h)) return LBM_EINVAL;
    if (n < 0 || n > lbm_ctx::kMaxParts) return h->fail(LBM_EINVAL, "streams must be 0, 1 or 2");
    h->streams_req = n;
    make_parts(h);
    h->drop_graphs();
    return LBM_OK;
}

int32_t lbm_get_streams(lbm_handle h) { return valid(h) ? h->nparts : -1; }

static Status shape_ok(const lbm_launch_shape* s) {
    if (!s) return {LBM_EINVAL, "shape is NULL"};
    if (s->vec != 1 && s->vec != 2 && s->vec != 4) return {LBM_EINVAL, "vec must be 1, 2 or 4"};
    if (s->block_x < 64 || s->block_x % 64 || s->block_x > kMaxBlock)
        return {LBM_EINVAL, "block_x must be a multiple of 64 in [64, 512]"};
    if (s->block_y < 1 || s->block_x * s->block_y > kMaxBlock)
        return {LBM_EINVAL, "block_y >= 1 with block_x * block_y <= 512"};
    return {LBM_OK, ""};
}

int lbm_set_launch_shape(lbm_handle h, const lbm_launch_shape* s) {
    if (!valid(h)) return LBM_EINVAL;
    Status st = shape_ok(s);
    if (st.code) return h->fail(st.code, st.msg);
    if (h->sr && s->vec != 1) return h->fail(LBM_EINVAL, "stochastic rounding needs vec = 1");
    if (is_split(h->storage) && s->vec != 1) return h->fail(LBM_EINVAL, "split storage needs vec = 1");
    h->shape.vec = s->vec;
    h->shape.bx = s->block_x;
    h->shape.by = s->block_y;
    h->shape.xcd = s->xcd_remap ? 1 : 0;
    h->shape.nt = s->nontemporal ? 1 : 0;
    build_tiles(h);
    h->drop_graphs();
    if (h->base) return upload_tables(h);
    return LBM_OK;
}

int lbm_get_launch_shape(lbm_handle h, lbm_launch_shape* s) {
    if (!valid(h)) return LBM_EINVAL;
    if (!s) return h->fail(LBM_EINVAL, "shape is NULL");
    s->vec = h->shape.vec;
    s->block_x = h->shape.bx;
    s->block_y = h->shape.by;
    s->xcd_remap = h->shape.xcd;
    s->nontemporal = h->shape.nt;
    return LBM_OK;
}


// ------------------------------------------------------------------ autotuner

static std::string tune_key(lbm_ctx* h) {
    hipDeviceProp_t p;
    std::string dev = "unknown";
    if (hipGetDeviceProperties(&p, h->device) == hipSuccess) dev = std::string(p.gcnArchName);
    uint64_t f = 1469598103934665603ull;   // FNV-1a over the instance shapes
    auto mix = [&f](int64_t v) {
        for (int b = 0; b < 8; ++b) {
            f ^= (uint64_t)((v >> (8 * b)) & 0xff);
            f *= 1099511628211ull;
        }
    };
    for (auto& in : h->inst) {
        mix(in.nx);
        mix(in.ny);
        mix(in.bc_x * 4 + in.bc_y);
    }
    char b[160];
    snprintf(b, sizeof b, "%s|s%d%s|n%zu|%016llx", dev.c_str(), h->storage,
             (h->storage != LBM_F32 && h->every_step) ? "e" : "", h->inst.size(), (unsigned long long)f);
    for (char* c = b; *c; ++c)
        if (*c == ' ' || *c == '"') *c = '_';
    return b;
}

static bool cache_lookup(const char* path, const std::string& key, Shape* out, int* fuse) {
    FILE* fp = fopen(path, "r");
    if (!fp) return false;
    char line[512];
    bool found = false;
    while (fgets(line, sizeof line, fp)) {
        char k[200];
        Shape s;
        if (sscanf(line, "{\"key\": \"%199[^\"]\", \"vec\": %d, \"block_x\": %d, \"block_y\": %d, "
                         "\"xcd\": %d, \"nt\": %d",
                   k, &s.vec, &s.bx, &s.by, &s.xcd, &s.nt) == 6 &&
            key == k) {
            *out = s;
            const char* f = strstr(line, "\"fuse\": ");
            *fuse = (f && f[8] >= '1' && f[8] <= '9') ? f[8] - '0' : 1;   // the digit after '"fuse": '
            found = true;   // the last matching line wins
        }
    }
    fclose(fp);
    return found;
}

static int time_shape(lbm_ctx* h, const Shape& s, int steps, hipEvent_t e0, hipEvent_t e1, float* us) {
    h->shape = s;
    build_tiles(h);
    int rc = upload_tables(h);
    if (rc) return rc;
    StepArgs a;
    a.desc = h->d_desc();
    a.tile_inst = h->d_tiles();
    a.snap = nullptr;
    a.partials = nullptr;
    a.tile_base = 0;
    a.ntiles = (int32_t)h->ntiles;
    a.seed = h->seed;
    a.sr = h->sr;
    a.ref = h->d_ref();
    a.apply_shift = 0;
    int src = 0;
    for (int w = 0; w < 3 + steps; ++w) {
        if (w == 3) HIPCALL(h, hipEventRecord(e0, h->stream));
        a.src = h->buf(src);
        a.dst = h->buf(1 - src);
        a.ctr_in = h->d_ctr() + src;
        a.ctr_out = h->d_ctr() + (1 - src);
        HIPCALL(h, launch_step(h->storage, s, kPlain, a, h->L.nodes, h->stream));
        src = 1 - src;
    }
    HIPCALL(h, hipEventRecord(e1, h->stream));
    HIPCALL(h, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCALL(h, hipEventElapsedTime(&ms, e0, e1));
    *us = 1000.0f * ms / steps;
    return LBM_OK;
}

// Average time per step of k-step launches (the launch shape's XCD remap and
// store hint), on scratch contents.
static int time_fused(lbm_ctx* h, int k, int launches, hipEvent_t e0, hipEvent_t e1, float* us) {
    StepArgs a;
    a.desc = h->d_desc();
    a.tile_inst = h->d_ptiles();
    a.snap = nullptr;
    a.partials = nullptr;
    a.tile_base = 0;
    a.ntiles = (int32_t)h->ptile_inst.size();
    a.seed = h->seed;
    a.sr = h->sr;
    a.ref = h->d_ref();
    a.apply_shift = 0;
    int src = 0;
    for (int w = 0; w < 2 + launches; ++w) {
        if (w == 2) HIPCALL(h, hipEventRecord(e0, h->stream));
        a.src = h->buf(src);
        a.dst = h->buf(1 - src);
        a.ctr_in = h->d_ctr() + src;
        a.ctr_out = h->d_ctr() + (1 - src);
        HIPCALL(h, launch_fused(h->storage, h->shape, a, k, 0, h->layout == LBM_LAYOUT_CHUNKED,
                                h->every_step ? kRoundEvery : kRoundLast, 0, h->stream));
        src = 1 - src;
    }
    HIPCALL(h, hipEventRecord(e1, h->stream));
    HIPCALL(h, hipEventSynchronize(e1));
    float ms = 0.0f;
    HIPCALL(h, hipEventElapsedTime(&ms, e0, e1));
    *us = 1000.0f * ms / (k * launches);
    return LBM_OK;
}

int lbm_autotune(lbm_handle h, int32_t steps, char* report, size_t report_len) {
    if (!valid(h)) return LBM_EINVAL;
    if (!h->base) return h->fail(LBM_ESTATE, "no device memory bound");
    for (char c : h->inited)
        if (c) return h->fail(LBM_ESTATE, "lbm_autotune must run before lbm_init");
    if (steps <= 0) steps = 20;
    const std::string key = tune_key(h);
    const char* path = getenv("LBM_AUTOTUNE_CACHE");
    Shape cached;
    int cached_fuse = 1;
    if (path && *path && cache_lookup(path, key, &cached, &cached_fuse)) {
        lbm_launch_shape ls = {cached.vec, cached.bx, cached.by, cached.xcd, cached.nt};
        if (report && report_len) snprintf(report, report_len, "{\"key\": \"%s\", \"cached\": true}", key.c_str());
        const int rc = lbm_set_launch_shape(h, &ls);
        if (!rc) h->fuse = std::min(std::max(cached_fuse, 1), h->fuse_cap());
        return rc;
    }
    // scratch contents: a fixed pattern of moderate finite values with
    // changing bits (zero-filled buffers run faster than real contents, which
    // biases the choice between single and fused launches)
    HIPCALL(h, launch_fill(h->buf(0), h->L.buf_bytes & ~(size_t)3, 1u, h->stream));
    HIPCALL(h, launch_fill(h->buf(1), h->L.buf_bytes & ~(size_t)3, 2u, h->stream));
    hipEvent_t e0, e1;
    HIPCALL(h, hipEventCreate(&e0));
    HIPCALL(h, hipEventCreate(&e1));
    const int vecs[3] = {1, 2, 4};
    const int blocks[9][2] = {{64, 1}, {128, 1}, {256, 1}, {512, 1}, {64, 2}, {64, 4}, {128, 2}, {128, 4}, {256, 2}};
    std::string rep = "{\"key\": \"" + key + "\", \"cached\": false, \"timings_us\": [";
    Shape best;
    float best_us = 1e30f;
    int rc = LBM_OK;
    bool first = true;
    auto try_shape = [&](const Shape& s) {
        if (rc) return;
        float us = 0.0f;
        rc = time_shape(h, s, steps, e0, e1, &us);
        if (rc) return;
        char b[160];
        snprintf(b, sizeof b, "%s[%d, %d, %d, %d, %d, %.2f]", first ? "" : ", ", s.vec, s.bx, s.by, s.xcd,
                 s.nt, us);
        first = false;
        rep += b;
        if (us < best_us) {
            best_us = us;
            best = s;
        }
    };
    for (int v : vecs)
        for (auto& b : blocks) {
            // stochastic rounding and split storage run one node per lane
            if ((h->sr || is_split(h->storage)) && v != 1) continue;
            Shape s;
            s.vec = v;
            s.bx = b[0];
            s.by = b[1];
            s.xcd = 1;
            s.nt = 0;
            try_shape(s);
        }
    const Shape base_best = best;
    for (int xcd = 0; xcd < 2; ++xcd)
        for (int nt = 0; nt < 2; ++nt) {
            if (xcd == 1 && nt == 0) continue;
            Shape s = base_best;
            s.xcd = xcd;
            s.nt = nt;
            try_shape(s);
        }
    // steps per launch: the fused kernel at every number of steps up to the
    // kind's most (with the best shape's XCD remap and store hint) against the
    // best single-step shape; small lattices hold few strips and may prefer
    // fewer steps per launch
    float fused_us = 1e30f;
    int fused_k = h->fuse_cap();
    std::string fused_rep;
    double launch_us[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // measured per-launch times, k = 1 .. kmax
    if (!rc) {
        h->shape = best;
        build_tiles(h);
        rc = upload_tables(h);
        for (int k = 2; k <= h->fuse_cap() && !rc; ++k) {
            float us = 0.0f;
            rc = time_fused(h, k, (steps + k - 1) / k, e0, e1, &us);
            launch_us[k] = (double)us * k;
            char b[64];
            snprintf(b, sizeof b, "%s[%d, %.2f]", k == 2 ? "" : ", ", k, us);
            fused_rep += b;
            if (!rc && us < fused_us) {
                fused_us = us;
                fused_k = k;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    const int fuse = fused_us < best_us ? fused_k : 1;
    // the planner's launch costs: the measured plain launches, the check
    // launches scaled from the built-in figures by the same ratio
    {
        double dp[8], dc[8];
        default_costs(h->storage, h->every_step, dp, dc);
        launch_us[1] = best_us;
        for (int k = 1; k <= h->fuse_cap(); ++k) {
            if (!(launch_us[k] > 0.0)) continue;
            h->cost_plain[k] = launch_us[k];
            if (k >= 2 && dp[k] > 0.0) h->cost_check[k] = dc[k] * launch_us[k] / dp[k];
        }
    }
    char b[320];
    snprintf(b, sizeof b, "], \"best\": [%d, %d, %d, %d, %d, %.2f], \"fused_us_per_step\": %.2f, ", best.vec,
             best.bx, best.by, best.xcd, best.nt, best_us, fused_us);
    rep += b;
    rep += "\"fused_timings_us\": [" + fused_rep + "], ";
    snprintf(b, sizeof b, "\"steps_per_launch\": %d}", fuse);
    rep += b;
    if (report && report_len) snprintf(report, report_len, "%s", rep.c_str());
    if (path && *path) {
        FILE* fp = fopen(path, "a");
        if (fp) {
            fprintf(fp, "{\"key\": \"%s\", \"vec\": %d, \"block_x\": %d, \"block_y\": %d, \"xcd\": %d, \"nt\": %d, "
                        "\"us\": %.2f, \"fuse\": %d}\n",
                    key.c_str(), best.vec, best.bx, best.by, best.xcd, best.nt, best_us, fuse);
            fclose(fp);
        }
    }
    lbm_launch_shape ls = {best.vec, best.bx, best.by, best.xcd, best.nt};
    rc = lbm_set_launch_shape(h, &ls);
    if (!rc) h->fuse = fuse;
    return rc;
}

}  // extern "C"
