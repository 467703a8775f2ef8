// Drives the host-side validation and sizing paths of the C ABI
// (phonon_lbm.h, phonon_d3q14.h) for the AddressSanitizer /
// UndefinedBehaviorSanitizer build of the CPU tests: every configuration error
// the library reports, device-memory sizes from the smallest lattices to
// ones near the node-count limit, the calls that accept NULL handles, and
// lbm_create / lbm3d_create on a host without a usable GPU (they must fail
// cleanly with LBM_EHIP).  Exit status 0 when every return code is the
// expected one.
#include "phonon_d3q14.h"
#include "phonon_lbm.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

static int failures = 0;

static void expect(bool ok, const char* what) {
    if (!ok) {
        std::printf("FAILED: %s\n", what);
        ++failures;
    }
}

static lbm_instance inst(int nx, int ny, int bcx = LBM_BC_PERIODIC, int bcy = LBM_BC_PERIODIC) {
    lbm_instance in;
    std::memset(&in, 0, sizeof in);
    in.nx = nx;
    in.ny = ny;
    in.bc_x = bcx;
    in.bc_y = bcy;
    in.tau_n = 0.6;
    in.tau_r = 5.0;
    in.cv = 1.0;
    in.t0 = 1.0;
    in.grad_x = bcx == LBM_BC_GRADIENT ? 1e-3 : 0.0;
    for (int w = 0; w < 4; ++w) in.t_wall[w] = 1.0;
    return in;
}

static lbm_config config(const std::vector<lbm_instance>& v, int storage = LBM_F32) {
    lbm_config c;
    std::memset(&c, 0, sizeof c);
    c.n_instances = (int32_t)v.size();
    c.storage = storage;
    c.inst = v.data();
    return c;
}

static int required(const lbm_config& c, size_t* b) { return lbm_required_bytes(&c, b); }

int main() {
    size_t bytes = 0;
    expect(std::strlen(lbm_version()) > 0, "lbm_version");
    expect(lbm_last_error(nullptr) != nullptr, "lbm_last_error(NULL)");
    expect(lbm_required_bytes(nullptr, &bytes) == LBM_EINVAL, "NULL config");
    // valid sizes: every storage kind and layout, single and batched
    for (int st = LBM_F32; st <= LBM_BF16_SPLIT; ++st)
        for (int layout = 0; layout <= 2; ++layout)
            for (int check : {0, -1, 2, 100}) {
              for (int32_t flags : {0, (int32_t)LBM_FLAG_ROUND_EVERY_STEP}) {
                std::vector<lbm_instance> v = {inst(2, 2), inst(65, 3, LBM_BC_ISOTHERMAL), inst(513, 77, LBM_BC_GRADIENT,
                                                                                               LBM_BC_DIFFUSE)};
                lbm_config c = config(v, st);
                c.layout = layout;
                c.check_interval = check;
                c.flags = flags;
                const int split = st == LBM_F16_SPLIT || st == LBM_BF16_SPLIT;
                const int rc = required(c, &bytes);
                if (split && layout == LBM_LAYOUT_PLANES) expect(rc == LBM_EUNSUPPORTED, "split planes refused");
                else expect(rc == LBM_OK && bytes > 0, "valid config sized");
              }
            }
    // near the node-count limit (2^31 nodes): sizes must not overflow
    {
        std::vector<lbm_instance> v = {inst(46340, 46340)};
        lbm_config c = config(v);
        expect(required(c, &bytes) == LBM_OK && bytes > (size_t)46340 * 46340 * 64, "large lattice sized");
        v[0] = inst(65536, 32769);
        c = config(v);
        expect(required(c, &bytes) == LBM_EINVAL, "more than 2^31 nodes refused");
    }
    // configuration errors
    {
        std::vector<lbm_instance> v = {inst(1, 5)};
        lbm_config c = config(v);
        expect(required(c, &bytes) == LBM_EINVAL, "nx < 2");
        v[0] = inst(8, 8);
        v[0].tau_n = 0.0;
        expect(required(c, &bytes) == LBM_EINVAL, "tau_n = 0");
        v[0].tau_n = NAN;
        expect(required(c, &bytes) == LBM_EINVAL, "tau_n NaN");
        v[0] = inst(8, 8);
        v[0].tau_r = -1.0;
        expect(required(c, &bytes) == LBM_EINVAL, "tau_r < 0");
        v[0] = inst(8, 8);
        v[0].tau_r = INFINITY;
        expect(required(c, &bytes) == LBM_OK, "tau_r infinite accepted");
        v[0] = inst(8, 8);
        v[0].scale = 3.0;
        expect(required(c, &bytes) == LBM_EINVAL, "scale not a power of two");
        v[0] = inst(8, 8, LBM_BC_PERIODIC, LBM_BC_GRADIENT);
        expect(required(c, &bytes) == LBM_EINVAL, "gradient along y");
        v[0] = inst(8, 8, LBM_BC_DIFFUSE, LBM_BC_DIFFUSE);
        expect(required(c, &bytes) == LBM_EUNSUPPORTED, "corners of two diffuse axes");
        v[0] = inst(8, 8, LBM_BC_GRADIENT, LBM_BC_ISOTHERMAL);
        expect(required(c, &bytes) == LBM_EUNSUPPORTED, "isothermal across a gradient seam");
        v[0] = inst(8, 8, 7, 0);
        expect(required(c, &bytes) == LBM_EINVAL, "unknown boundary kind");
        v[0] = inst(8, 8);
        v[0].wall_bc[2] = LBM_BC_ISOTHERMAL;
        expect(required(c, &bytes) == LBM_EINVAL, "wall kind on a periodic axis");
        v[0] = inst(8, 8);
        c.storage = 9;
        expect(required(c, &bytes) == LBM_EINVAL, "bad storage");
        c.storage = LBM_F32;
        c.check_interval = 1;
        expect(required(c, &bytes) == LBM_EINVAL, "check interval 1");
        c.check_interval = 0;
        c.flags = 0x100;
        expect(required(c, &bytes) == LBM_EINVAL, "unknown flags");
        c.flags = 0;
        c.n_instances = 0;
        expect(required(c, &bytes) == LBM_EINVAL, "no instances");
        c.n_instances = 1;
        expect(lbm_required_bytes(&c, nullptr) == LBM_EINVAL, "NULL bytes");
        lbm_handle h = nullptr;
        c.storage = 9;
        expect(lbm_create(&c, &h) == LBM_EINVAL && h == nullptr, "create refuses a bad config");
        expect(std::strlen(lbm_last_error(nullptr)) > 0, "create error message");
    }
    // a valid config on a host whose GPU is missing fails with LBM_EHIP (or
    // succeeds where a GPU is present) and leaves nothing behind
    {
        std::vector<lbm_instance> v = {inst(70, 33, LBM_BC_GRADIENT, LBM_BC_DIFFUSE)};
        lbm_config c = config(v);
        lbm_handle h = nullptr;
        const int rc = lbm_create(&c, &h);
        expect(rc == LBM_EHIP || rc == LBM_OK || rc == LBM_ENOMEM, "create on this host");
        if (rc == LBM_OK) lbm_destroy(h);
    }
    lbm_destroy(nullptr);
    expect(lbm_step(nullptr, 1) == LBM_EINVAL, "step(NULL)");
    expect(lbm_steps_done(nullptr) == -1, "steps_done(NULL)");
    expect(lbm_get_step_fusion(nullptr) == -1, "get_step_fusion(NULL)");
    expect(lbm_set_streams(nullptr, 2) == LBM_EINVAL, "set_streams(NULL)");
    expect(lbm_get_streams(nullptr) == -1, "get_streams(NULL)");
    expect(lbm_max_step_fusion(LBM_F32) == 7 && lbm_max_step_fusion(LBM_BF16_SPLIT) == 6, "max step fusion");
    expect(lbm_max_step_fusion(7) == -1, "max step fusion of a bad kind");
    double out[3];
    expect(lbm_totals(nullptr, 0, out) == LBM_EINVAL, "totals(NULL)");
    expect(lbm_moments_f64_noalloc(nullptr, 0, out, nullptr, nullptr) == LBM_EINVAL, "noalloc(NULL)");

    // D3Q14
    lbm3d_config c3;
    std::memset(&c3, 0, sizeof c3);
    c3.nx = 5;
    c3.ny = 3;
    c3.nz = 2;
    c3.storage = LBM_F32;
    c3.tau_n = 0.6;
    c3.tau_r = 5.0;
    c3.t0 = 1.0;
    for (int st = LBM_F32; st <= LBM_BF16; ++st)
        for (int layout = 0; layout <= 2; ++layout) {
            c3.storage = st;
            c3.layout = layout;
            expect(lbm3d_required_bytes(&c3, &bytes) == LBM_OK && bytes > 0, "D3Q14 sized");
        }
    c3.storage = LBM_F16_SPLIT;
    expect(lbm3d_required_bytes(&c3, &bytes) != LBM_OK, "D3Q14 split refused");
    c3.storage = LBM_F32;
    c3.nx = 0;
    expect(lbm3d_required_bytes(&c3, &bytes) == LBM_EINVAL, "D3Q14 nx = 0");
    c3.nx = 5;
    c3.tau_n = -1.0;
    expect(lbm3d_required_bytes(&c3, &bytes) == LBM_EINVAL, "D3Q14 tau_n < 0");
    c3.tau_n = 0.6;
    lbm3d_handle h3 = nullptr;
    const int rc3 = lbm3d_create(&c3, &h3);
    expect(rc3 == LBM_EHIP || rc3 == LBM_OK || rc3 == LBM_ENOMEM, "D3Q14 create on this host");
    if (rc3 == LBM_OK) lbm3d_destroy(h3);
    lbm3d_destroy(nullptr);
    expect(lbm3d_last_error(nullptr) != nullptr, "lbm3d_last_error(NULL)");

    std::printf("runtime sanitizer checks: %s\n", failures ? "FAILED" : "ok");
    return failures ? 1 : 0;
}
