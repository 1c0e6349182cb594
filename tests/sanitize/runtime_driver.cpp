// Drives the host-side paths of libclaw that run before any device work
// (descriptor validation, workspace plans, size limits, error strings, the
// learned correction's host arithmetic), for a build whose host code runs
// under AddressSanitizer and UndefinedBehaviorSanitizer (test infrastructure;
// see tests/test_sanitizers.py).  Exits nonzero if a call returns a status
// other than the one expected.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "../../include/claw.h"

static int g_fail = 0;
static void expect(claw_status got, claw_status want, const char* what) {
    if (got != want) {
        fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, claw_last_error());
        ++g_fail;
    }
}

static claw_desc sw(int64_t n) {
    claw_desc d;
    claw_desc_init(&d);
    d.n[0] = d.n[1] = n;
    d.riemann = CLAW_RP_SHALLOW_WATER;
    d.meqn = d.mwaves = 3;
    d.dtype = CLAW_FP32;
    for (int k = 0; k < 3; ++k) d.bc_lo[k] = d.bc_hi[k] = CLAW_BC_WALL;
    return d;
}

int main() {
    size_t bytes = 0;
    claw_desc d = sw(64);
    expect(claw_workspace_bytes(&d, &bytes), CLAW_OK, "workspace sw");
    expect(claw_workspace_bytes(nullptr, &bytes), CLAW_E_INVALID, "null desc");
    // every validation rule, one bad field at a time
    struct Bad { const char* what; void (*edit)(claw_desc*); claw_status want; };
    const Bad bad[] = {
        {"ndim", [](claw_desc* x) { x->ndim = 4; }, CLAW_E_INVALID},
        {"n<1", [](claw_desc* x) { x->n[1] = 0; }, CLAW_E_INVALID},
        {"n huge", [](claw_desc* x) { x->n[0] = (int64_t)1 << 40; }, CLAW_E_UNSUPPORTED},
        {"upper", [](claw_desc* x) { x->upper[0] = x->lower[0]; }, CLAW_E_INVALID},
        {"bc", [](claw_desc* x) { x->bc_hi[1] = 7; }, CLAW_E_INVALID},
        {"2d nz", [](claw_desc* x) { x->n[2] = 2; }, CLAW_E_INVALID},
        {"ghost", [](claw_desc* x) { x->num_ghost = 3; }, CLAW_E_INVALID},
        {"flags", [](claw_desc* x) { x->flags = 64; }, CLAW_E_INVALID},
        {"dtype", [](claw_desc* x) { x->dtype = 9; }, CLAW_E_INVALID},
        {"limiter", [](claw_desc* x) { x->limiter = 9; }, CLAW_E_INVALID},
        {"cfl", [](claw_desc* x) { x->cfl_max = 0.5; }, CLAW_E_INVALID},
        {"dt_max", [](claw_desc* x) { x->dt_max = 0; }, CLAW_E_INVALID},
        {"too many cells", [](claw_desc* x) { x->n[0] = x->n[1] = 40000; }, CLAW_E_UNSUPPORTED},
        {"sw 3d", [](claw_desc* x) { x->ndim = 3; }, CLAW_E_UNSUPPORTED},
        {"sw meqn", [](claw_desc* x) { x->meqn = 4; }, CLAW_E_INVALID},
        {"sw aux", [](claw_desc* x) { x->maux = 2; }, CLAW_E_INVALID},
        {"grav", [](claw_desc* x) { x->grav = -1; }, CLAW_E_INVALID},
        {"riemann", [](claw_desc* x) { x->riemann = 9; }, CLAW_E_INVALID},
        {"plugin id", [](claw_desc* x) { x->riemann = 40; }, CLAW_E_INVALID},
        {"plugin meqn", [](claw_desc* x) { x->riemann = CLAW_RP_BURGERS; }, CLAW_E_INVALID},
        {"plugin param", [](claw_desc* x) { x->riemann = CLAW_RP_SHALLOW_WATER_GENERIC; x->param[2] = NAN; },
         CLAW_E_INVALID},
        {"acoustics meqn", [](claw_desc* x) { x->riemann = CLAW_RP_ACOUSTICS; x->mwaves = 2; x->meqn = 4; },
         CLAW_E_INVALID},
        {"acoustics rho", [](claw_desc* x) { x->riemann = CLAW_RP_ACOUSTICS; x->mwaves = 2; x->meqn = 3; x->rho = 0; },
         CLAW_E_INVALID},
    };
    for (const Bad& b : bad) {
        claw_desc x = sw(64);
        b.edit(&x);
        expect(claw_workspace_bytes(&x, &bytes), b.want, b.what);
    }
    // create / static run refuse bad arguments before any device work
    claw_solver* h = nullptr;
    expect(claw_create(&d, nullptr, nullptr, nullptr, 0, nullptr, &h), CLAW_E_INVALID, "create null q");
    alignas(256) static float fake[16];
    expect(claw_create(&d, fake, nullptr, fake, 16, nullptr, &h), CLAW_E_INVALID, "create small workspace");
    double t = 0;
    int64_t nrej = 0;
    expect(claw_advance(nullptr, 1, 0.0, &t, &nrej), CLAW_E_INVALID, "advance null");
    // batches
    claw_desc ds[3] = {sw(100), sw(131), sw(77)};
    expect(claw_batch_workspace_bytes(ds, 3, &bytes), CLAW_OK, "batch bytes");
    ds[1].riemann = CLAW_RP_ACOUSTICS;
    ds[1].mwaves = 2;
    expect(claw_batch_workspace_bytes(ds, 3, &bytes), CLAW_E_UNSUPPORTED, "batch mixed");
    expect(claw_batch_workspace_bytes(ds, 0, &bytes), CLAW_E_INVALID, "batch empty");
    // learned correction: sizes and host arithmetic
    claw_lc_desc ld;
    memset(&ld, 0, sizeof ld);
    ld.nx = 48;
    ld.ny = 40;
    ld.mu_h = 1.0f;
    for (int c = 0; c < 3; ++c) ld.sl[c] = ld.sd1[c] = ld.sd2[c] = ld.sd3[c] = ld.s_out[c] = 1.0f;
    size_t pb = 0, wb = 0;
    expect(claw_lc_sizes(&ld, &pb, &wb), CLAW_OK, "lc sizes");
    ld.nx = 1;
    expect(claw_lc_sizes(&ld, &pb, &wb), CLAW_E_INVALID, "lc small");
    const double r2[3] = {1e-6, 2e-6, 0.0};
    float so[3];
    double w[3];
    expect(claw_lc_scales(r2, 64, 0.5, 1, so, w), CLAW_OK, "lc scales");
    expect(claw_lc_scales(r2, 0, 0.5, 1, so, w), CLAW_E_INVALID, "lc scales ncell");
    // plug-in registry and strings
    int32_t me = 0, mw = 0, nd = 0, vf = 0;
    const char* name = nullptr;
    expect(claw_plugin_info(CLAW_RP_BURGERS, &me, &mw, &nd, &vf, &name), CLAW_OK, "plugin info");
    expect(claw_plugin_info(99, &me, &mw, &nd, &vf, &name), CLAW_E_INVALID, "plugin unknown");
    for (int s = 0; s < 8; ++s) (void)strlen(claw_status_string((claw_status)s));
    (void)strlen(claw_last_error());
    printf("runtime host paths: %d unexpected statuses\n", g_fail);
    return g_fail ? 1 : 0;
}
