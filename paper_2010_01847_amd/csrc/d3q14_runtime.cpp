// Host runtime of the D3Q14 path: the C ABI of phonon_d3q14.h.  It validates
// a box, derives the relaxation coefficients (Eq. 49, Eq. 54 and the combined
// relaxation-plus-source factor of Eqs. 13, 15, 16), lays the two population
// buffers out in device memory and issues the kernels of d3q14_device.hip on
// the caller's stream.
#include "../../include/phonon_d3q14.h"
#include "d3q14_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace plbm3;

namespace {

constexpr uint32_t kMagic3 = 0x4c424d33u;   // "LBM3"
constexpr size_t kAlign = 256;
constexpr size_t kPlanePad = 4096;          // bytes between direction planes (spreads HBM channels)
thread_local std::string g_error3;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int esize(int storage) { return storage == LBM_F32 ? 4 : 2; }

struct Layout3 {
    Geometry g;
    size_t buf_bytes;      // one population buffer
    size_t off_buf[2];
    size_t off_part;       // totals stage-1 records
    size_t off_res;        // totals result (4 doubles)
    size_t total;
};

// Layout for tiles of tile_waves segments x rows_per_tile rows.  Plane,
// chunk-array and buffer starts are 256-byte aligned; the buffers do not
// depend on the tiling.
Layout3 layout_of(const lbm3d_config& c, int rows_per_tile, int tile_waves) {
    Layout3 L;
    Geometry& g = L.g;
    const int es = esize(c.storage);
    g.nx = c.nx;
    g.ny = c.ny;
    g.nz = c.nz;
    g.layout = c.layout == LBM_LAYOUT_PLANES ? 0 : 1;     // AUTO = CHUNKED
    g.rows_per_tile = (uint32_t)rows_per_tile;
    g.tile_waves = (uint32_t)tile_waves;
    g.nseg = (c.nx + kTileX - 1) / kTileX;
    g.ntx = (uint32_t)((c.nx + kTileX * tile_waves - 1) / (kTileX * tile_waves));
    g.nty = (uint32_t)((c.ny + rows_per_tile - 1) / rows_per_tile);
    g.ntiles = g.ntx * g.nty * (uint32_t)c.nz;
    if (g.layout == 0) {
        g.pitch = (int32_t)align_up((size_t)c.nx, (size_t)kRowAlign);
        const size_t plane_bytes = align_up((size_t)g.pitch * c.ny * c.nz * es, kAlign) + kPlanePad;
        g.plane = (int64_t)(plane_bytes / es);
        L.buf_bytes = kQ * plane_bytes;
    } else {
        g.pitch = 0;
        g.plane = 0;
        L.buf_bytes = align_up((size_t)g.nseg * c.ny * c.nz * kQ * kTileX * es, kAlign) + kPlanePad;
    }
    size_t o = 0;
    L.off_buf[0] = o;
    o += L.buf_bytes;
    L.off_buf[1] = o;
    o += L.buf_bytes;
    L.off_part = o;
    o += align_up(4 * sizeof(double) * (size_t)totals_blocks(g), kAlign);
    L.off_res = o;
    o += kAlign;
    L.total = o;
    return L;
}

struct Status3 {
    int code;
    std::string msg;
};

Status3 check3(const lbm3d_config* c) {
    if (!c) return {LBM_EINVAL, "config is NULL"};
    if (c->nx < 1 || c->ny < 1 || c->nz < 1) return {LBM_EINVAL, "nx, ny, nz must be >= 1"};
    if (c->storage != LBM_F32 && c->storage != LBM_F16 && c->storage != LBM_BF16)
        return {LBM_EINVAL, "storage must be LBM_F32, LBM_F16 or LBM_BF16"};
    if (c->flags & ~(LBM_FLAG_EXTERNAL_MEMORY | LBM_FLAG_STOCHASTIC_ROUNDING | LBM_FLAG_ROUND_EVERY_STEP))
        return {LBM_EINVAL, "unknown flag bits"};
    if (!(c->tau_n > 0.0) || !std::isfinite(c->tau_n)) return {LBM_EINVAL, "tau_n must be finite and > 0"};
    if (!(c->tau_r > 0.0)) return {LBM_EINVAL, "tau_r must be > 0 (+inf allowed)"};
    if (c->cv < 0.0 || !std::isfinite(c->cv)) return {LBM_EINVAL, "cv must be finite and >= 0 (0 selects 1)"};
    if (!std::isfinite(c->t0)) return {LBM_EINVAL, "t0 must be finite"};
    if (c->scale != 0.0) {
        int ex = 0;
        if (!(c->scale > 0.0) || !std::isfinite(c->scale) || std::frexp(c->scale, &ex) != 0.5)
            return {LBM_EINVAL, "scale must be 0 or a positive power of two"};
    }
    if (c->layout != LBM_LAYOUT_AUTO && c->layout != LBM_LAYOUT_PLANES && c->layout != LBM_LAYOUT_CHUNKED)
        return {LBM_EINVAL, "layout must be LBM_LAYOUT_AUTO, LBM_LAYOUT_PLANES or LBM_LAYOUT_CHUNKED"};
    // node indices (stochastic-rounding counters, tiles) are 32-bit
    if ((int64_t)c->nx * c->ny * c->nz >= ((int64_t)1 << 32))
        return {LBM_EINVAL, "box too large: 2^32 nodes or more"};
    return {LBM_OK, ""};
}

}  // namespace

struct lbm3d_ctx {
    uint32_t magic = kMagic3;
    lbm3d_config cfg{};
    hipStream_t stream = nullptr;
    Layout3 L{};
    lbm3d_launch_shape shape{4, 1, 0, 1, 32};
    int fuse = 1;                // time steps per launch (1, or 2 with the z-marching kernel)
    // two steps per launch when the z-marching tiles fill the chip (one block
    // per CU): a launch takes about one tile's marching time, so small boxes
    // run single steps (measured FP32 us per step, single / two: 64^3 5.3 /
    // 37.1, 128^3 34.1 / 41.2 with 132 tiles, 192^3 137 / 124 with 384, 512^3
    // 2670 / 1887; 512^3 FP16-SR 1464 / 1338, BF16-SR 1493 / 1378 with the
    // window kept in 16 bits and column-and-row rounding words)
    void set_default_fuse() {
        const int64_t tiles = (int64_t)((cfg.nx + kPairW3 - 1) / kPairW3) * ((cfg.ny + kPairYO - 1) / kPairYO) *
                              ((cfg.nz + shape.zchunk - 1) / shape.zchunk);
        fuse = tiles >= kPairMinTiles ? 2 : 1;
    }
    double tau = 0, beta = 1, s = 1, cv = 1;
    Coeffs co{};
    char* base = nullptr;
    bool owned = false;
    bool inited = false;
    int cur = 0;                 // buffer holding the post-relaxation state of the last step
    int64_t steps = 0;
    std::string err;

    void* buf(int k) const { return base + L.off_buf[k]; }
    double* d_part() const { return reinterpret_cast<double*>(base + L.off_part); }
    double* d_res() const { return reinterpret_cast<double*>(base + L.off_res); }
    int fail(int code, const std::string& m) {
        err = m;
        return code;
    }
    int hip_fail(hipError_t e, const char* what) {
        err = std::string(what) + ": " + hipGetErrorString(e);
        return LBM_EHIP;
    }
};

#define HIPCALL3(h, expr)                                        \
    do {                                                         \
        hipError_t e_ = (expr);                                  \
        if (e_ != hipSuccess) return (h)->hip_fail(e_, #expr);   \
    } while (0)

static bool valid3(lbm3d_handle h) { return h && h->magic == kMagic3; }

// tau = tau_C + 1/2 (Eq. 49) with 1/tau_C = 1/tau_N + 1/tau_R; beta of Eq. 54;
// k_i = (5/3) a_i beta (1/tau - (1 - 1/(2 tau)) / tau_R): (5/3) a_i is 1/3 on
// the axis movers and 1/24 on the corner movers.
static void derive(lbm3d_ctx* h) {
    const lbm3d_config& c = h->cfg;
    const bool inf_r = std::isinf(c.tau_r);
    const double inv_tc = 1.0 / c.tau_n + (inf_r ? 0.0 : 1.0 / c.tau_r);
    h->tau = 1.0 / inv_tc + 0.5;
    h->beta = inf_r ? 1.0 : 2.0 * c.tau_r / (2.0 * c.tau_r + 1.0);
    h->cv = c.cv > 0.0 ? c.cv : 1.0;
    const double kappa = 1.0 / h->tau - (inf_r ? 0.0 : (1.0 - 0.5 / h->tau) / c.tau_r);
    h->co.inv_tau = (float)(1.0 / h->tau);
    h->co.omega_axis = (float)(1.0 / 9.0);
    h->co.omega_corner = (float)(1.0 / 24.0);
    h->co.k_axis = (float)(h->beta * kappa / 3.0);
    h->co.k_corner = (float)(h->beta * kappa / 24.0);
}

extern "C" {

const char* lbm3d_last_error(lbm3d_handle h) {
    if (!h) return g_error3.c_str();
    if (!valid3(h)) return "invalid handle";
    return h->err.c_str();
}

int lbm3d_required_bytes(const lbm3d_config* cfg, size_t* bytes) {
    Status3 s = check3(cfg);
    if (s.code) {
        g_error3 = s.msg;
        return s.code;
    }
    if (!bytes) {
        g_error3 = "bytes is NULL";
        return LBM_EINVAL;
    }
    *bytes = layout_of(*cfg, 4, 1).total;
    return LBM_OK;
}

int lbm3d_create(const lbm3d_config* cfg, lbm3d_handle* out) {
    Status3 s = check3(cfg);
    if (!s.code && !out) s = {LBM_EINVAL, "out is NULL"};
    if (s.code) {
        g_error3 = s.msg;
        return s.code;
    }
    lbm3d_ctx* h = new (std::nothrow) lbm3d_ctx();
    if (!h) {
        g_error3 = "host allocation failed";
        return LBM_ENOMEM;
    }
    h->cfg = *cfg;
    h->stream = reinterpret_cast<hipStream_t>(cfg->stream);
    // default launch shape, the fastest measured for each layout at 512^3
    // (chunked: 5.60 TB/s without, 5.50 with the XCD remap; planes: 5.39 with,
    // 4.43 without)
    h->shape = cfg->layout == LBM_LAYOUT_PLANES ? lbm3d_launch_shape{4, 1, 0, 1, 32}
                                                : lbm3d_launch_shape{4, 0, 0, 1, 32};
    h->L = layout_of(*cfg, h->shape.rows_per_tile, h->shape.tile_waves);
    h->set_default_fuse();
    derive(h);
    if (!(cfg->flags & LBM_FLAG_EXTERNAL_MEMORY)) {
        void* p = nullptr;
        hipError_t e = hipMalloc(&p, h->L.total);
        if (e != hipSuccess) {
            g_error3 = std::string("hipMalloc: ") + hipGetErrorString(e);
            delete h;
            return e == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EHIP;
        }
        h->base = static_cast<char*>(p);
        h->owned = true;
    }
    *out = h;
    return LBM_OK;
}

int lbm3d_bind(lbm3d_handle h, void* device_buf, size_t bytes) {
    if (!valid3(h)) return LBM_EINVAL;
    if (!(h->cfg.flags & LBM_FLAG_EXTERNAL_MEMORY))
        return h->fail(LBM_ESTATE, "handle owns its memory (created without LBM_FLAG_EXTERNAL_MEMORY)");
    if (h->base) return h->fail(LBM_ESTATE, "memory already bound");
    if (!device_buf || bytes < h->L.total)
        return h->fail(LBM_EINVAL, "buffer NULL or smaller than lbm3d_required_bytes (" +
                                       std::to_string(h->L.total) + ")");
    if (reinterpret_cast<uintptr_t>(device_buf) % kAlign) return h->fail(LBM_EINVAL, "buffer must be 256-byte aligned");
    h->base = static_cast<char*>(device_buf);
    return LBM_OK;
}

// Device copies of host arrays for the duration of one call.
struct Staging {
    double* p = nullptr;
    ~Staging() {
        if (p) (void)hipFree(p);
    }
};

int lbm3d_init(lbm3d_handle h, const double* T, const double* qx, const double* qy, const double* qz,
               int32_t on_device) {
    if (!valid3(h)) return LBM_EINVAL;
    if (!h->base) return h->fail(LBM_ESTATE, "no device memory bound");
    const lbm3d_config& c = h->cfg;
    const size_t n = (size_t)c.nx * c.ny * c.nz;
    double s = c.scale;
    if (s == 0.0) {
        if (c.storage == LBM_F16) {
            if (on_device) return h->fail(LBM_EINVAL, "FP16 storage with device init needs an explicit scale");
            double amp = 0.0;
            for (size_t k = 0; k < n; ++k) {
                const double a = std::max({T ? std::fabs(T[k] - c.t0) : 0.0, qx ? std::fabs(qx[k]) : 0.0,
                                           qy ? std::fabs(qy[k]) : 0.0, qz ? std::fabs(qz[k]) : 0.0});
                if (!std::isfinite(a)) return h->fail(LBM_EINVAL, "non-finite initial field");
                amp = std::max(amp, a);
            }
            s = amp > 0.0 ? std::ldexp(1.0, (int)std::ceil(std::log2(amp)) - 13) : 1.0;
        } else {
            s = 1.0;
        }
    }
    const double* in[4] = {T, qx, qy, qz};
    const double* dev[4] = {nullptr, nullptr, nullptr, nullptr};
    Staging stg;
    if (on_device) {
        for (int k = 0; k < 4; ++k) dev[k] = in[k];
    } else {
        int cnt = 0;
        for (int k = 0; k < 4; ++k) cnt += in[k] != nullptr;
        if (cnt) {
            HIPCALL3(h, hipMalloc(reinterpret_cast<void**>(&stg.p), cnt * n * sizeof(double)));
            int j = 0;
            for (int k = 0; k < 4; ++k)
                if (in[k]) {
                    dev[k] = stg.p + (size_t)j * n;
                    HIPCALL3(h, hipMemcpyAsync(const_cast<double*>(dev[k]), in[k], n * sizeof(double),
                                               hipMemcpyHostToDevice, h->stream));
                    ++j;
                }
        }
    }
    // the first step pulls from buffer `cur`
    h->cur = 0;
    HIPCALL3(h, launch_init(c.storage, h->L.g, h->buf(0), dev[0], dev[1], dev[2], dev[3], c.t0, h->cv,
                            1.0 / h->beta, 1.0 / s, h->stream));
    HIPCALL3(h, hipStreamSynchronize(h->stream));
    h->s = s;
    h->steps = 0;
    h->inited = true;
    return LBM_OK;
}

int lbm3d_step(lbm3d_handle h, int64_t nsteps) {
    if (!valid3(h)) return LBM_EINVAL;
    if (nsteps < 0) return h->fail(LBM_EINVAL, "nsteps < 0");
    if (!h->inited) return h->fail(LBM_ESTATE, "not initialised");
    StepArgs a;
    a.g = h->L.g;
    a.c = h->co;
    a.seed = h->cfg.seed;
    a.xcd_remap = h->shape.xcd_remap;
    a.nontemporal = h->shape.nontemporal;
    const int sr = (h->cfg.flags & LBM_FLAG_STOCHASTIC_ROUNDING) ? 1 : 0;
    PairArgs p;
    p.g = a.g;
    p.c = a.c;
    p.seed = a.seed;
    // the z-marching kernel always hands each XCD a contiguous range of tiles:
    // measured 71.1 vs 56.9 GLUPS without (512^3 FP32, 32-plane ranges)
    p.xcd_remap = 1;
    p.nontemporal = a.nontemporal;
    p.zchunk = h->shape.zchunk;
    p.ptx = (uint32_t)((h->cfg.nx + kPairW3 - 1) / kPairW3);
    p.pty = (uint32_t)((h->cfg.ny + kPairYO - 1) / kPairYO);
    p.ptz = (uint32_t)((h->cfg.nz + p.zchunk - 1) / p.zchunk);
    p.ntiles = p.ptx * p.pty * p.ptz;
    for (int64_t k = 0; k < nsteps;) {
        if (h->fuse == 2 && nsteps - k >= 2) {
            p.src = h->buf(h->cur);
            p.dst = h->buf(1 - h->cur);
            p.step = (uint32_t)h->steps;
            HIPCALL3(h, launch_pair(h->cfg.storage, sr, (h->cfg.flags & LBM_FLAG_ROUND_EVERY_STEP) ? 1 : 0, p,
                                    h->stream));
            h->cur = 1 - h->cur;
            h->steps += 2;
            k += 2;
            continue;
        }
        a.src = h->buf(h->cur);
        a.dst = h->buf(1 - h->cur);
        a.step = (uint32_t)h->steps;
        HIPCALL3(h, launch_step(h->cfg.storage, sr, a, h->stream));
        h->cur = 1 - h->cur;
        ++h->steps;
        ++k;
    }
    return LBM_OK;
}

int64_t lbm3d_steps_done(lbm3d_handle h) { return valid3(h) ? h->steps : -1; }

int lbm3d_moments(lbm3d_handle h, double* dT, double* qx, double* qy, double* qz, int32_t on_device) {
    if (!valid3(h)) return LBM_EINVAL;
    if (!h->inited) return h->fail(LBM_ESTATE, "not initialised");
    const lbm3d_config& c = h->cfg;
    const size_t n = (size_t)c.nx * c.ny * c.nz;
    double* out[4] = {dT, qx, qy, qz};
    double* dev[4] = {nullptr, nullptr, nullptr, nullptr};
    Staging stg;
    if (on_device) {
        for (int k = 0; k < 4; ++k) dev[k] = out[k];
    } else {
        int cnt = 0;
        for (int k = 0; k < 4; ++k) cnt += out[k] != nullptr;
        if (!cnt) return LBM_OK;
        HIPCALL3(h, hipMalloc(reinterpret_cast<void**>(&stg.p), cnt * n * sizeof(double)));
        int j = 0;
        for (int k = 0; k < 4; ++k)
            if (out[k]) dev[k] = stg.p + (size_t)(j++) * n;
    }
    HIPCALL3(h, launch_moments(c.storage, h->L.g, h->buf(h->cur), h->s / h->cv, h->s * h->beta, dev[0], dev[1],
                               dev[2], dev[3], h->stream));
    if (!on_device)
        for (int k = 0; k < 4; ++k)
            if (out[k])
                HIPCALL3(h, hipMemcpyAsync(out[k], dev[k], n * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCALL3(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm3d_sample(lbm3d_handle h, const int64_t* nodes, int64_t count, double* out, int32_t on_device) {
    if (!valid3(h)) return LBM_EINVAL;
    if (!h->inited) return h->fail(LBM_ESTATE, "not initialised");
    if (count < 0) return h->fail(LBM_EINVAL, "count < 0");
    if (count == 0) return LBM_OK;
    if (!nodes || !out) return h->fail(LBM_EINVAL, "nodes or out is NULL");
    const lbm3d_config& c = h->cfg;
    const int64_t n = (int64_t)c.nx * c.ny * c.nz;
    const int64_t* dn = nodes;
    double* dout = out;
    Staging stg;
    if (!on_device) {
        for (int64_t k = 0; k < count; ++k)
            if (nodes[k] < 0 || nodes[k] >= n) return h->fail(LBM_EINVAL, "node index out of range");
        HIPCALL3(h, hipMalloc(reinterpret_cast<void**>(&stg.p), (size_t)count * (4 * sizeof(double) + sizeof(int64_t))));
        dout = stg.p;
        int64_t* pn = reinterpret_cast<int64_t*>(stg.p + 4 * count);
        HIPCALL3(h, hipMemcpyAsync(pn, nodes, (size_t)count * sizeof(int64_t), hipMemcpyHostToDevice, h->stream));
        dn = pn;
    }
    HIPCALL3(h, launch_sample(c.storage, h->L.g, h->buf(h->cur), h->s / h->cv, h->s * h->beta, dn, count, dout,
                              h->stream));
    if (!on_device)
        HIPCALL3(h, hipMemcpyAsync(out, dout, (size_t)count * 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIPCALL3(h, hipStreamSynchronize(h->stream));
    return LBM_OK;
}

int lbm3d_totals(lbm3d_handle h, double out[4]) {
    if (!valid3(h)) return LBM_EINVAL;
    if (!out) return h->fail(LBM_EINVAL, "out is NULL");
    if (!h->inited) return h->fail(LBM_ESTATE, "not initialised");
    HIPCALL3(h, launch_totals(h->cfg.storage, h->L.g, h->buf(h->cur), h->d_part(), h->d_res(), h->stream));
    double r[4];
    HIPCALL3(h, hipMemcpyAsync(r, h->d_res(), sizeof r, hipMemcpyDeviceToHost, h->stream));
    HIPCALL3(h, hipStreamSynchronize(h->stream));
    out[0] = r[0] * h->s;
    for (int k = 1; k < 4; ++k) out[k] = r[k] * h->s * h->beta;
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(out[k])) return h->fail(LBM_ENONFINITE, "non-finite total");
    return LBM_OK;
}

int lbm3d_set_launch_shape(lbm3d_handle h, const lbm3d_launch_shape* shape) {
    if (!valid3(h)) return LBM_EINVAL;
    if (!shape) return h->fail(LBM_EINVAL, "shape is NULL");
    const int r = shape->rows_per_tile, tw = shape->tile_waves;
    if (r != 1 && r != 2 && r != 4) return h->fail(LBM_EINVAL, "rows_per_tile must be 1, 2 or 4");
    if (tw != 1 && tw != 2 && tw != 4 && tw != 8) return h->fail(LBM_EINVAL, "tile_waves must be 1, 2, 4 or 8");
    if (r * tw > 8) return h->fail(LBM_EINVAL, "rows_per_tile * tile_waves must be <= 8 (512 threads)");
    if ((shape->xcd_remap & ~1) || (shape->nontemporal & ~1))
        return h->fail(LBM_EINVAL, "xcd_remap and nontemporal must be 0 or 1");
    if (shape->zchunk < 1) return h->fail(LBM_EINVAL, "zchunk must be >= 1");
    h->shape = *shape;
    // the tiling changes, the buffers (which do not depend on it) stay
    const Layout3 L = layout_of(h->cfg, r, tw);
    h->L.g = L.g;
    return LBM_OK;
}

int lbm3d_set_step_fusion(lbm3d_handle h, int32_t steps) {
    if (!valid3(h)) return LBM_EINVAL;
    if (steps != 1 && steps != 2) return h->fail(LBM_EINVAL, "steps per launch must be 1 or 2");
    h->fuse = steps;
    return LBM_OK;
}

int32_t lbm3d_get_step_fusion(lbm3d_handle h) { return valid3(h) ? h->fuse : -1; }

int lbm3d_get_launch_shape(lbm3d_handle h, lbm3d_launch_shape* shape) {
    if (!valid3(h)) return LBM_EINVAL;
    if (!shape) return h->fail(LBM_EINVAL, "shape is NULL");
    *shape = h->shape;
    return LBM_OK;
}

int lbm3d_autotune(lbm3d_handle h, int32_t steps, char* report, size_t report_len) {
    if (!valid3(h)) return LBM_EINVAL;
    if (!h->base) return h->fail(LBM_ESTATE, "no device memory bound");
    if (h->inited) return h->fail(LBM_ESTATE, "lbm3d_autotune must run before lbm3d_init");
    if (steps <= 0) steps = 20;
    // scratch contents: a fixed pattern of moderate finite values with
    // changing bits (zero-filled buffers run the single-step kernel about 8%
    // faster than real contents: FP16-SR 512^3 1343 against 1464 us per step)
    HIPCALL3(h, launch_fill(h->buf(0), h->L.buf_bytes & ~(size_t)3, 1u, h->stream));
    HIPCALL3(h, launch_fill(h->buf(1), h->L.buf_bytes & ~(size_t)3, 2u, h->stream));
    hipEvent_t e0, e1;
    HIPCALL3(h, hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return h->hip_fail(e, "hipEventCreate");
    }
    std::string rep = "{\"timings_us\": [";
    lbm3d_launch_shape best = h->shape;
    float best_us = 1e30f;
    int rc = LBM_OK;
    h->inited = true;                 // let lbm3d_step run on the zeroed buffers
    bool first = true;
    auto try_shape = [&](const lbm3d_launch_shape& sh) {
        if (rc) return;
        rc = lbm3d_set_launch_shape(h, &sh);
        if (!rc) rc = lbm3d_step(h, 2);   // warm-up
        if (!rc && (e = hipEventRecord(e0, h->stream)) != hipSuccess) rc = h->hip_fail(e, "hipEventRecord");
        if (!rc) rc = lbm3d_step(h, steps);
        if (!rc && (e = hipEventRecord(e1, h->stream)) != hipSuccess) rc = h->hip_fail(e, "hipEventRecord");
        if (!rc && (e = hipEventSynchronize(e1)) != hipSuccess) rc = h->hip_fail(e, "hipEventSynchronize");
        float ms = 0.0f;
        if (!rc && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) rc = h->hip_fail(e, "hipEventElapsedTime");
        if (rc) return;
        const float us = 1e3f * ms / (float)steps;
        char b[96];
        snprintf(b, sizeof b, "%s[%d, %d, %d, %d, %.2f]", first ? "" : ", ", sh.rows_per_tile, sh.xcd_remap,
                 sh.nontemporal, sh.tile_waves, us);
        first = false;
        rep += b;
        if (us < best_us) {
            best_us = us;
            best = sh;
        }
    };
    // every tile shape with and without the XCD remap, then streaming stores on the best
    h->fuse = 1;
    for (int r : {1, 2, 4})
        for (int tw : {1, 2, 4, 8})
            for (int xcd = 0; xcd < 2; ++xcd)
                if (r * tw <= 8) try_shape(lbm3d_launch_shape{r, xcd, 0, tw, h->shape.zchunk});
    if (!rc) {
        lbm3d_launch_shape sh = best;
        sh.nontemporal = 1;
        try_shape(sh);
    }
    // two steps per launch over z ranges of 16, 32 and 64 planes, with and
    // without streaming stores (per-step time over the same number of steps,
    // rounded up to pairs); the two-step kernel's tile is fixed, so the
    // single-step kernel's best store kind need not be its best
    const float single_us = best_us;
    float pair_us = 1e30f;
    int best_z = best.zchunk, best_nt = best.nontemporal;
    std::string prep;
    steps += steps & 1;
    for (int zc : {16, 32, 64}) {
        for (int nt = 0; nt < 2; ++nt) {
            if (rc) break;
            lbm3d_launch_shape sh = best;
            sh.zchunk = zc;
            sh.nontemporal = nt;
            rc = lbm3d_set_launch_shape(h, &sh);
            h->fuse = 2;
            if (!rc) rc = lbm3d_step(h, 2);
            if (!rc && (e = hipEventRecord(e0, h->stream)) != hipSuccess) rc = h->hip_fail(e, "hipEventRecord");
            if (!rc) rc = lbm3d_step(h, steps);
            if (!rc && (e = hipEventRecord(e1, h->stream)) != hipSuccess) rc = h->hip_fail(e, "hipEventRecord");
            if (!rc && (e = hipEventSynchronize(e1)) != hipSuccess) rc = h->hip_fail(e, "hipEventSynchronize");
            float ms = 0.0f;
            if (!rc && (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
                rc = h->hip_fail(e, "hipEventElapsedTime");
            if (rc) break;
            const float us = 1e3f * ms / (float)steps;
            char b[64];
            snprintf(b, sizeof b, "%s[%d, %d, %.2f]", prep.empty() ? "" : ", ", zc, nt, us);
            prep += b;
            if (us < pair_us) {
                pair_us = us;
                best_z = zc;
                best_nt = nt;
            }
        }
    }
    best.zchunk = best_z;
    h->fuse = pair_us < single_us ? 2 : 1;
    if (h->fuse == 2) best.nontemporal = best_nt;
    h->inited = false;
    h->steps = 0;
    h->cur = 0;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
        h->set_default_fuse();
        return rc;
    }
    rc = lbm3d_set_launch_shape(h, &best);
    if (rc) return rc;
    char b[128];
    snprintf(b, sizeof b, "], \"best\": [%d, %d, %d, %d, %.2f], \"pair_us_per_step\": [", best.rows_per_tile,
             best.xcd_remap, best.nontemporal, best.tile_waves, single_us);
    rep += b;
    rep += prep;
    snprintf(b, sizeof b, "], \"zchunk\": %d, \"steps_per_launch\": %d}", best.zchunk, h->fuse);
    rep += b;
    if (report && report_len) {
        strncpy(report, rep.c_str(), report_len - 1);
        report[report_len - 1] = 0;
    }
    return LBM_OK;
}

void lbm3d_destroy(lbm3d_handle h) {
    if (!valid3(h)) return;
    if (h->owned && h->base) (void)hipFree(h->base);
    h->magic = 0;
    delete h;
}

}  // extern "C"
