// runtime.hip -- the C ABI of include/claw.h: descriptor validation,
// workspace plan, the step sequence of section 4.1 (sweeps x, y (, z), then
// the CFL control kernel) enqueued on the caller's stream, and the captured
// HIP graph that runs many adaptive steps without host round trips.
#include <math.h>
#include <stdarg.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/claw.h"
#include "claw_launch.h"

using namespace claw;

namespace {

thread_local char g_err[512] = "";

claw_status fail(claw_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
claw_status fail(claw_status s, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return s;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(CLAW_E_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                        __LINE__);                                                             \
    } while (0)

constexpr size_t kAlign = 4096;
constexpr int kGraphSteps = 32;  // trial steps per captured graph (batched ensembles)
// Trial counts of the captured single-grid graphs: a call replays a
// decomposition of the trials it needs (greedy, largest first), so a short
// advance dispatches no trial beyond its step count.
constexpr int kLadder[4] = {32, 8, 2, 1};

size_t round_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Plan {
    int64_t ncell;
    size_t elem;
    size_t state_bytes;
    size_t off_ctrl, off_b1, off_b2, off_zc, total;
};

claw_status validate(const claw_desc* d) {
    if (!d) return fail(CLAW_E_INVALID, "descriptor is NULL");
    if (d->ndim != 2 && d->ndim != 3) return fail(CLAW_E_INVALID, "ndim must be 2 or 3 (got %d)", d->ndim);
    for (int k = 0; k < 3; ++k) {
        if (d->n[k] < 1) return fail(CLAW_E_INVALID, "n[%d] = %lld must be >= 1", k, (long long)d->n[k]);
        if (d->n[k] >= ((int64_t)1 << 31))  // keeps the cell count below from overflowing
            return fail(CLAW_E_UNSUPPORTED, "n[%d] = %lld is too large", k, (long long)d->n[k]);
        if (k < d->ndim && !(d->upper[k] > d->lower[k]))
            return fail(CLAW_E_INVALID, "upper[%d] must exceed lower[%d]", k, k);
        if (d->bc_lo[k] < 0 || d->bc_lo[k] > 2 || d->bc_hi[k] < 0 || d->bc_hi[k] > 2)
            return fail(CLAW_E_INVALID, "boundary condition of direction %d out of range", k);
    }
    if (d->ndim == 2 && d->n[2] != 1) return fail(CLAW_E_INVALID, "2D grids need n[2] = 1");
    if (d->num_ghost != 2) return fail(CLAW_E_INVALID, "num_ghost must be 2 (got %d)", d->num_ghost);
    if (d->flags & ~(CLAW_FLAG_FUSED_STEP | CLAW_FLAG_STRANG | CLAW_FLAG_SPLIT_STEP))
        return fail(CLAW_E_INVALID, "unknown flags 0x%x", (unsigned)d->flags);
    if ((d->flags & CLAW_FLAG_FUSED_STEP) && (d->flags & CLAW_FLAG_SPLIT_STEP))
        return fail(CLAW_E_INVALID, "CLAW_FLAG_FUSED_STEP and CLAW_FLAG_SPLIT_STEP exclude each other");
    if (d->dtype != CLAW_FP32 && d->dtype != CLAW_FP64) return fail(CLAW_E_INVALID, "unknown dtype");
    if (d->limiter < 0 || d->limiter > 5) return fail(CLAW_E_INVALID, "unknown limiter");
    if (!(d->cfl_desired > 0) || !(d->cfl_max >= d->cfl_desired))
        return fail(CLAW_E_INVALID, "need 0 < cfl_desired <= cfl_max");
    if (!(d->dt_max > 0)) return fail(CLAW_E_INVALID, "dt_max must be positive");
    const int64_t ncell = d->n[0] * d->n[1] * d->n[2];
    if (ncell * (int64_t)(d->meqn > 2 ? d->meqn : 2) >= ((int64_t)1 << 31) || d->n[1] > 65535 * 4 ||
        d->n[2] > 65535)
        return fail(CLAW_E_UNSUPPORTED, "grid too large for 32-bit element offsets");
    // the sweeps address each field with 32-bit byte offsets
    if ((uint64_t)ncell * (d->dtype == CLAW_FP64 ? 8u : 4u) > 0xffffffffull)
        return fail(CLAW_E_UNSUPPORTED, "grid too large: a field must stay below 4 GiB");
    if (d->riemann == CLAW_RP_ACOUSTICS) {
        if (d->meqn != 1 + d->ndim) return fail(CLAW_E_INVALID, "acoustics needs meqn = 1 + ndim");
        if (d->mwaves != 2) return fail(CLAW_E_INVALID, "acoustics has mwaves = 2");
        if (d->maux != 0 && d->maux != 2) return fail(CLAW_E_INVALID, "acoustics takes maux 0 or 2");
        if (d->maux == 0 && !(d->rho > 0 && d->bulk > 0))
            return fail(CLAW_E_INVALID, "acoustics needs rho > 0 and bulk > 0");
    } else if (d->riemann == CLAW_RP_SHALLOW_WATER) {
        if (d->ndim != 2) return fail(CLAW_E_UNSUPPORTED, "shallow water is 2D");
        if (d->meqn != 3 || d->mwaves != 3) return fail(CLAW_E_INVALID, "shallow water has meqn = mwaves = 3");
        if (d->maux != 0) return fail(CLAW_E_INVALID, "shallow water takes no aux");
        if (!(d->grav > 0)) return fail(CLAW_E_INVALID, "grav must be positive");
    } else if (d->riemann >= CLAW_RP_PLUGIN_BASE) {
        int32_t meqn = 0, mwaves = 0, ndim_max = 0;
        if (claw_plugin_info(d->riemann, &meqn, &mwaves, &ndim_max, nullptr, nullptr) != CLAW_OK)
            return fail(CLAW_E_INVALID, "unknown Riemann solver %d", d->riemann);
        if (d->meqn != meqn || d->mwaves != mwaves)
            return fail(CLAW_E_INVALID, "plug-in %d has meqn = %d, mwaves = %d", d->riemann, meqn, mwaves);
        if (d->ndim > ndim_max) return fail(CLAW_E_UNSUPPORTED, "plug-in %d runs up to %dD", d->riemann, ndim_max);
        if (d->maux != 0) return fail(CLAW_E_INVALID, "plug-in solvers take no aux");
        for (int k = 0; k < 4; ++k)
            if (!isfinite(d->param[k])) return fail(CLAW_E_INVALID, "param[%d] is not finite", k);
    } else {
        return fail(CLAW_E_INVALID, "unknown Riemann solver %d", d->riemann);
    }
    return CLAW_OK;
}

Plan make_plan(const claw_desc* d) {
    Plan p;
    p.ncell = d->n[0] * d->n[1] * d->n[2];
    p.elem = d->dtype == CLAW_FP64 ? 8 : 4;
    p.state_bytes = (size_t)p.ncell * (size_t)d->meqn * p.elem;
    p.off_ctrl = 0;
    p.off_b1 = round_up(sizeof(Ctrl));
    p.off_b2 = p.off_b1 + round_up(p.state_bytes);
    p.off_zc = p.off_b2 + round_up(p.state_bytes);
    p.total = p.off_zc + (d->maux ? round_up((size_t)p.ncell * 2 * p.elem) : 0);
    return p;
}

}  // namespace

struct claw_solver {
    claw_desc d;
    Plan plan;
    int sys;
    bool fp32;
    bool fused;   // one fused kernel per 2D step (fused.hip) instead of an x and a y sweep
    bool fused3;  // 3D acoustics: one fused x and y kernel (fused.hip), then the z sweep
    bool strang;  // Strang splitting: half-step sweeps around a full step of the last direction
    hipStream_t stream;
    hipStream_t cap_stream;
    void* buf[3];
    void* zc;
    Ctrl* ctrl;
    double dx[3];
    int parity;                  // parity of the next trial; copy parity ^ 1 is the committed state
    hipGraphExec_t gexec[4][2];  // captured trial sequences, by ladder rung and starting parity
    hipGraph_t graph[4][2];
    std::vector<hipEvent_t> events;
    hipGraphExec_t lc_exec;  // captured learned steps and the arguments they were captured with
    hipGraph_t lc_graph;
    unsigned char lc_key[128];
};

namespace {

int result_offset(int ndim) { return ndim == 2 ? 2 : 1; }

int col_chunk(int64_t m, int64_t nx, int64_t nlines_o) {
    // cells along the sweep per wavefront: the shortest chunks (least
    // redundant halo work) that still give every SIMD at most three
    // wavefronts, so no SIMD marches a fourth chunk (measured at 2048^2 FP32:
    // 22 rows, 3008 wavefronts on 1024 SIMDs; 24 rows 5 % slower, 20 rows
    // 20 % slower); at least 16 rows.  Tuning overrides from the environment:
    // CLAW_COL_WAVES (target wavefronts per column sweep) and CLAW_COL_CHUNK
    // (rows per chunk, used as given up to m); values <= 0 are ignored.
    static const int64_t target_waves = [] {
        const char* e = getenv("CLAW_COL_WAVES");
        if (e && atoll(e) > 0) return (int64_t)atoll(e);
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        return (int64_t)3 * 4 * cus;
    }();
    static const int64_t forced = [] {
        const char* e = getenv("CLAW_COL_CHUNK");
        return e ? (int64_t)atoll(e) : (int64_t)0;
    }();
    const int64_t nstrip = (nx + 63) / 64;
    int64_t chunk = forced > 0 ? forced : (m * nstrip * nlines_o + target_waves - 1) / target_waves;
    if (forced <= 0) {
        if (chunk < 16) chunk = 16;
        if (chunk > 1024) chunk = 1024;
    }
    if (chunk > m) chunk = m;
    if (chunk < 1) chunk = 1;
    return (int)chunk;
}

// Sweep arguments of one grid.  chunk <= 0 picks the column chunk from the
// grid size (col_chunk).
template <typename R>
SweepArgs<R> grid_args(const claw_desc& d, int sys, int64_t ncell, void* const* buf, const void* zc,
                       Ctrl* ctrl, int dir, int src_off, int dst_off, int chunk) {
    SweepArgs<R> a;
    memset(&a, 0, sizeof a);
    for (int i = 0; i < 3; ++i) a.buf[i] = (R*)buf[i];
    a.zc = (const R*)zc;
    a.ctrl = ctrl;
    a.ncell = (int32_t)ncell;
    const int64_t nx = d.n[0], ny = d.n[1], nz = d.n[2];
    a.nx = (int32_t)nx;
    a.dir = dir;
    a.src_off = src_off;
    a.dst_off = dst_off;
    a.bc_lo = d.bc_lo[dir];
    a.bc_hi = d.bc_hi[dir];
    a.limiter = d.limiter;
    a.efix = d.efix;
    a.grav = (R)d.grav;
    a.sqrt_grav = (R)sqrt(d.grav);
    if (sys == SYS_AC) {
        a.Z0 = (R)sqrt(d.rho * d.bulk);
        a.c0 = (R)sqrt(d.bulk / d.rho);
    }
    for (int k = 0; k < 4; ++k) a.prm[k] = (R)d.param[k];
    if (dir == 0) {
        a.m = (int32_t)nx;
        a.stride = 1;
        a.nrows = (int32_t)(ny * nz);
    } else {
        a.m = (int32_t)(dir == 1 ? ny : nz);
        a.stride = (int32_t)(dir == 1 ? nx : nx * ny);
        a.nlines_o = (int32_t)(dir == 1 ? nz : ny);
        a.ostride = (int32_t)(dir == 1 ? nx * ny : nx);
        a.chunk = chunk > 0 ? (int32_t)(chunk < a.m ? chunk : a.m) : col_chunk(a.m, nx, a.nlines_o);
    }
    return a;
}

template <typename R>
SweepArgs<R> sweep_args(const claw_solver* h, int dir, int src_off, int dst_off) {
    return grid_args<R>(h->d, h->sys, h->plan.ncell, h->buf, h->zc, h->ctrl, dir, src_off, dst_off, 0);
}

// One sweep launch.  speeds: speed-only pass; parity: step-state copy and
// speed slots; first / last: the sweep opens / closes a trial.
hipError_t enqueue_sweep(claw_solver* h, int dir, int src_off, int dst_off, bool speeds, int parity,
                         bool first, bool last, hipStream_t s) {
    if (h->fp32) {
        SweepArgs<float> a = sweep_args<float>(h, dir, src_off, dst_off);
        a.parity = parity;
        a.first = first ? 1 : 0;
        a.last = last ? 1 : 0;
        return launch_sweep<float>(a, h->sys, h->d.meqn, speeds, s);
    }
    SweepArgs<double> a = sweep_args<double>(h, dir, src_off, dst_off);
    a.parity = parity;
    a.first = first ? 1 : 0;
    a.last = last ? 1 : 0;
    return launch_sweep<double>(a, h->sys, h->d.meqn, speeds, s);
}

int committed(const claw_solver* h) { return h->parity ^ 1; }

// Sweeps of one trial: direction, dt fraction implied by the control block,
// source and destination buffer offsets (relative to the current buffer).
// Offsets run 0 -> 1 -> 2 -> 1 -> 2 ..., so Q^n (offset 0) is never written;
// Godunov 2D x: 0->1, y: 1->2; 3D adds z: 2->1; Strang 2D x/2: 0->1,
// y: 1->2, x/2: 2->1.
int trial_sweeps(const claw_solver* h, int* dirs, int* so, int* dof) {
    const int nd = h->d.ndim;
    const int k = h->strang ? 2 * nd - 1 : nd;
    for (int i = 0; i < k; ++i) {
        dirs[i] = i < nd ? i : k - 1 - i;
        so[i] = i == 0 ? 0 : (i % 2 ? 1 : 2);
        dof[i] = (i + 1) % 2 ? 1 : 2;
    }
    return k;
}

// Buffer offset of a step's result: the fused 2D step writes cur + 1; the
// fused 3D x and y step writes cur + 1 and the z sweep cur + 2.
int result_offset_of(const claw_solver* h) {
    if (h->fused) return 1;
    if (h->fused3) return 2;
    int dirs[5], so[5], dof[5];
    const int k = trial_sweeps(h, dirs, so, dof);
    return dof[k - 1];
}

// Rows per workgroup of the fused 2D step: about four rounds of the
// workgroups a device holds at once (four per CU: one wavefront per SIMD each,
// four wavefronts per SIMD), so the last round leaves few CUs idle, and at
// least 24 rows so the four halo rows a chunk sweeps twice stay a small share
// (measured at 4096^2 FP32: 16 / 24 / 32 / 48 rows give 165.8 / 154.4 / 158.4 /
// 169.6 us per step; at 8192^2 the rule's 68 rows 551 us, 32 / 64 / 96 rows
// 559 / 544 / 551 us).
// CLAW_FUSED_CHUNK overrides the choice for tuning (read once per process;
// values <= 0 are ignored).
int fused_chunk(int64_t nx, int64_t ny, bool fp32) {
    static const int64_t target = [] {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        return (int64_t)16 * cus;
    }();
    static const int64_t forced = [] {
        const char* e = getenv("CLAW_FUSED_CHUNK");
        return e ? (int64_t)atoll(e) : (int64_t)0;
    }();
    const int64_t w = fp32 ? 248 : 124;
    const int64_t strips = (nx + w - 1) / w;
    int64_t chunk = forced > 0 ? forced : (strips * ny + target - 1) / target;
    if (forced <= 0 && chunk < 24) chunk = 24;
    if (chunk > ny) chunk = ny;
    if (chunk < 1) chunk = 1;
    return (int)chunk;
}

// Rows of one z plane per workgroup of the fused 3D acoustics x and y step:
// the planes split into as many chunks as three workgroups per CU allow, at
// least 16 rows each (measured at 256^3 FP32: 24 / 32 / 52 / 64 / 86 rows
// give 142.3 / 141.5 / 146.9 / 139.6 / 136.4 us per launch; 86 rows are three
// chunks per plane, 768 workgroups).  CLAW_FUSED_CHUNK overrides it as for
// the 2D step.
int fused3_chunk(int64_t ny, int64_t nz) {
    static const int64_t cus = [] {
        int dev = 0, n = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0)
            n = 256;
        return (int64_t)n;
    }();
    static const int64_t forced = [] {
        const char* e = getenv("CLAW_FUSED_CHUNK");
        return e ? (int64_t)atoll(e) : (int64_t)0;
    }();
    int64_t per_plane = 3 * cus / (nz > 0 ? nz : 1);
    if (per_plane < 1) per_plane = 1;
    int64_t chunk = forced > 0 ? forced : (ny + per_plane - 1) / per_plane;
    if (forced <= 0 && chunk < 16) chunk = 16;
    if (chunk > ny) chunk = ny;
    if (chunk < 1) chunk = 1;
    return (int)chunk;
}

template <typename R>
Fused3Args<R> fused3_args(const claw_solver* h, int parity) {
    Fused3Args<R> F;
    memset(&F, 0, sizeof F);
    F.a = sweep_args<R>(h, 0, 0, 1);
    F.a.parity = parity;
    F.ny = (int32_t)h->d.n[1];
    F.nz = (int32_t)h->d.n[2];
    F.bcy_lo = h->d.bc_lo[1];
    F.bcy_hi = h->d.bc_hi[1];
    F.chunk = fused3_chunk(h->d.n[1], h->d.n[2]);
    return F;
}

template <typename R>
FusedArgs<R> fused_args(const claw_solver* h, int parity) {
    FusedArgs<R> F;
    memset(&F, 0, sizeof F);
    F.a = sweep_args<R>(h, 0, 0, 1);
    F.a.parity = parity;
    F.ny = (int32_t)h->d.n[1];
    F.bcy_lo = h->d.bc_lo[1];
    F.bcy_hi = h->d.bc_hi[1];
    F.chunk = fused_chunk(h->d.n[0], h->d.n[1], h->fp32);
    return F;
}

// One trial step: the sweeps x, y (, z).  The first decides the previous
// trial on the device; the trial itself is decided by the next trial's first
// sweep or by a commit.  ev (optional) receives an event before each sweep and
// one after the last.
claw_status enqueue_trial(claw_solver* h, hipStream_t s, hipEvent_t* ev) {
    if (h->fused) {
        HIP_TRY(launch_open(h->ctrl, h->parity, h->fp32, s));
        if (ev) HIP_TRY(hipEventRecord(ev[0], s));
        if (h->fp32) HIP_TRY(launch_step2d<float>(fused_args<float>(h, h->parity), s));
        else HIP_TRY(launch_step2d<double>(fused_args<double>(h, h->parity), s));
        if (ev) HIP_TRY(hipEventRecord(ev[1], s));
        h->parity ^= 1;
        return CLAW_OK;
    }
    if (h->fused3) {  // opened by the x and y kernel, closed by the z sweep
        if (ev) HIP_TRY(hipEventRecord(ev[0], s));
        if (h->fp32) HIP_TRY(launch_step_xy3<float>(fused3_args<float>(h, h->parity), h->sys, s));
        else HIP_TRY(launch_step_xy3<double>(fused3_args<double>(h, h->parity), h->sys, s));
        if (ev) HIP_TRY(hipEventRecord(ev[1], s));
        HIP_TRY(enqueue_sweep(h, 2, 1, 2, false, h->parity, false, true, s));
        if (ev) HIP_TRY(hipEventRecord(ev[2], s));
        h->parity ^= 1;
        return CLAW_OK;
    }
    int dirs[5], so[5], dof[5];
    const int k = trial_sweeps(h, dirs, so, dof);
    for (int i = 0; i < k; ++i) {
        if (ev) HIP_TRY(hipEventRecord(ev[i], s));
        HIP_TRY(enqueue_sweep(h, dirs[i], so[i], dof[i], false, h->parity, i == 0, i == k - 1, s));
    }
    if (ev) HIP_TRY(hipEventRecord(ev[k], s));
    h->parity ^= 1;
    return CLAW_OK;
}

// Applies the decision of the last trial (if any) to the committed copy.
claw_status commit(claw_solver* h) {
    HIP_TRY(launch_commit(h->ctrl, committed(h), h->fp32, h->stream));
    return CLAW_OK;
}

claw_status read_ctrl(claw_solver* h, Ctrl* out) {
    HIP_TRY(hipMemcpyAsync(out, h->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CLAW_OK;
}

// The committed step state only (one small copy and one stream synchronisation).
claw_status read_state(claw_solver* h, StepState* out) {
    HIP_TRY(hipMemcpyAsync(out, &h->ctrl->st[committed(h)], sizeof(StepState), hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return CLAW_OK;
}

claw_status sync_state(claw_solver* h) {
    if (h->fp32)
        HIP_TRY(launch_sync_state<float>(h->ctrl, committed(h), (float*)h->buf[0], (float*)h->buf[1],
                                         (float*)h->buf[2], h->plan.ncell * h->d.meqn, h->stream));
    else
        HIP_TRY(launch_sync_state<double>(h->ctrl, committed(h), (double*)h->buf[0], (double*)h->buf[1],
                                          (double*)h->buf[2], h->plan.ncell * h->d.meqn, h->stream));
    return CLAW_OK;
}

// Speed-only pass on the committed state into the committed copy's slots
// (call after commit()).  auto_dt: the pass skips its work when the committed
// copy already holds a next step (dt_next > 0).
claw_status speed_pass(claw_solver* h, bool auto_dt = false) {
    const int q = committed(h);
    HIP_TRY(launch_zero_speeds(h->ctrl, q, h->stream));
    for (int dir = 0; dir < h->d.ndim; ++dir) {
        if (h->fp32) {
            SweepArgs<float> a = sweep_args<float>(h, dir, 0, 0);
            a.parity = q;
            a.auto_dt = auto_dt ? 1 : 0;
            HIP_TRY(launch_sweep<float>(a, h->sys, h->d.meqn, true, h->stream));
        } else {
            SweepArgs<double> a = sweep_args<double>(h, dir, 0, 0);
            a.parity = q;
            a.auto_dt = auto_dt ? 1 : 0;
            HIP_TRY(launch_sweep<double>(a, h->sys, h->d.meqn, true, h->stream));
        }
    }
    return CLAW_OK;
}

// max |s| of parity q and direction dir: the largest of the slots (the bit
// patterns of non-negative values order like the values)
double smax_value(const claw_solver* h, const Ctrl& c, int q, int dir) {
    if (h->fp32) {
        unsigned m = 0u;
        for (int k = 0; k < SMAX_SLOTS; ++k) m = c.smax[q][dir][k].v32 > m ? c.smax[q][dir][k].v32 : m;
        float f;
        memcpy(&f, &m, 4);
        return f;
    }
    unsigned long long m = 0ull;
    for (int k = 0; k < SMAX_SLOTS; ++k) m = c.smax[q][dir][k].v64 > m ? c.smax[q][dir][k].v64 : m;
    double v;
    memcpy(&v, &m, 8);
    return v;
}

// First trial step of an adaptive run (call after commit()): dt0, else the
// dt_next of a previous run, else cfl_desired / sigma of a speed pass.  The
// choice between the last two is made on the device (no host round trip).
claw_status begin_adaptive(claw_solver* h, double dt0) {
    const int q = committed(h);
    const int roff = result_offset_of(h);
    if (dt0 > 0) {
        HIP_TRY(launch_begin(h->ctrl, q, dt0, MODE_ADAPT, roff, h->stream));
        return CLAW_OK;
    }
    claw_status st = speed_pass(h, true);
    if (st) return st;
    HIP_TRY(launch_init_dt(h->ctrl, q, h->fp32, MODE_ADAPT, roff, true, h->stream));
    return CLAW_OK;
}

claw_status ctrl_status(const StepState& c) {
    if (c.err == 5) return fail(CLAW_E_NONPHYSICAL, "non-physical state (depth <= 0 or not finite)");
    if (c.err == 6) return fail(CLAW_E_STATE, "step control failed (no usable time step)");
    if (c.err) return fail(CLAW_E_STATE, "step control error %d", c.err);
    return CLAW_OK;
}

// Graph of kLadder[r] trials starting at the current parity (captured once
// per rung and starting parity).
claw_status ensure_graph(claw_solver* h, int r) {
    const int p = h->parity;
    if (h->gexec[r][p]) return CLAW_OK;
    HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
    claw_status st = CLAW_OK;
    for (int k = 0; k < kLadder[r] && st == CLAW_OK; ++k) st = enqueue_trial(h, h->cap_stream, nullptr);
    h->parity = p;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(CLAW_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&h->gexec[r][p], g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        h->gexec[r][p] = nullptr;
        return fail(CLAW_E_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    h->graph[r][p] = g;
    return CLAW_OK;
}

// Fills the handle for a validated descriptor d over the state q and a
// workspace laid out by plan p at ws; no device work.
void bind_solver(claw_solver* h, const claw_desc* d, const Plan& p, void* q, char* ws, hipStream_t stream) {
    h->d = *d;
    h->plan = p;
    h->fp32 = d->dtype == CLAW_FP32;
    h->sys = d->riemann >= CLAW_RP_PLUGIN_BASE ? d->riemann
             : (d->riemann == CLAW_RP_SHALLOW_WATER ? SYS_SW : (d->maux ? SYS_ACV : SYS_AC));
    h->strang = (d->flags & CLAW_FLAG_STRANG) != 0;
    const bool fusable = !h->strang && h->sys == SYS_SW && d->ndim == 2;
    const bool big = d->dtype == CLAW_FP32 && (uint64_t)p.state_bytes >= (uint64_t)CLAW_FUSED_AUTO_BYTES;
    const bool want = (d->flags & CLAW_FLAG_FUSED_STEP) || (big && !(d->flags & CLAW_FLAG_SPLIT_STEP));
    h->fused = fusable && want;
    // 3D acoustics with rows of one wavefront's cells and extrapolation at both x ends
    const bool fusable3 = !h->strang && (h->sys == SYS_AC || h->sys == SYS_ACV) && d->ndim == 3 &&
                          d->n[0] == (d->dtype == CLAW_FP32 ? 256 : 128) && d->n[2] <= 65535 &&
                          d->bc_lo[0] == CLAW_BC_EXTRAP && d->bc_hi[0] == CLAW_BC_EXTRAP;
    h->fused3 = fusable3 && want;
    h->stream = stream;
    h->ctrl = (Ctrl*)(ws + p.off_ctrl);
    h->buf[0] = q;
    h->buf[1] = ws + p.off_b1;
    h->buf[2] = ws + p.off_b2;
    h->zc = d->maux ? (void*)(ws + p.off_zc) : nullptr;
    for (int k = 0; k < 3; ++k) h->dx[k] = k < d->ndim ? (d->upper[k] - d->lower[k]) / (double)d->n[k] : 1.0;
    h->parity = 0;
}

// Set-up kernels on the handle's stream: control block, derived acoustic
// coefficients.
hipError_t setup_kernels(claw_solver* h, const void* aux) {
    hipError_t e = launch_ctrl_init(h->ctrl, h->dx, h->d.ndim, h->d.cfl_desired, h->d.cfl_max, h->d.dt_max,
                                    h->strang, result_offset_of(h), h->stream);
    if (e == hipSuccess && h->d.maux) {
        if (h->fp32) e = launch_derive_zc<float>((const float*)aux, (float*)h->zc, h->plan.ncell, h->stream);
        else e = launch_derive_zc<double>((const double*)aux, (double*)h->zc, h->plan.ncell, h->stream);
    }
    return e;
}

// Enqueues exactly `trials` trial steps as replays of the captured graphs.
claw_status replay_trials(claw_solver* h, int64_t trials) {
    for (int r = 0; r < 4; ++r) {
        while (trials >= kLadder[r]) {
            claw_status st = ensure_graph(h, r);
            if (st) return st;
            HIP_TRY(hipGraphLaunch(h->gexec[r][h->parity], h->stream));
            h->parity ^= kLadder[r] & 1;
            trials -= kLadder[r];
        }
    }
    return CLAW_OK;
}

// The adaptive loop of claw_advance: trials from the graph ladder (graphs)
// or enqueued one by one (no graph objects, nothing allocated).
claw_status run_adaptive(claw_solver* h, int64_t nsteps, double dt0, bool graphs, double* t,
                         int64_t* nreject) {
    claw_status st = commit(h);
    if (st) return st;
    if (nsteps > 0) {
        st = begin_adaptive(h, dt0);
        if (st) return st;
    }
    HIP_TRY(launch_set_target(h->ctrl, committed(h), nsteps, h->stream));
    int64_t remaining = nsteps;
    StepState S;
    for (int round = 0; round < 1000; ++round) {
        if (graphs) {
            st = replay_trials(h, remaining);
        } else {
            for (int64_t k = 0; k < remaining && st == CLAW_OK; ++k) st = enqueue_trial(h, h->stream, nullptr);
        }
        if (!st) st = commit(h);
        if (!st) st = read_state(h, &S);
        if (st) return st;
        if (S.err) {  // the state stays the last accepted one
            st = sync_state(h);
            return st ? st : ctrl_status(S);
        }
        remaining = S.target - S.accepted;
        if (S.done || remaining <= 0) break;
    }
    // the caller's array receives the state once, after the last round (no
    // copy when the last step already wrote it)
    st = sync_state(h);
    if (st) return st;
    if (t) *t = S.t;
    if (nreject) *nreject = S.rejected - S.base_rejected;
    if (S.accepted - S.base_accepted != nsteps) return fail(CLAW_E_STATE, "advance stopped early");
    return CLAW_OK;
}

}  // namespace

#ifdef CLAW_DEBUG
namespace claw {
namespace {
DebugTake g_debug_take[16];  // one reader per kernel file, filled during static initialisation
int g_debug_n = 0;
}  // namespace
void debug_register(DebugTake take) {
    if (g_debug_n < 16) g_debug_take[g_debug_n++] = take;
}
}  // namespace claw
#endif

extern "C" {

claw_status claw_plugin_info(int32_t id, int32_t* meqn, int32_t* mwaves, int32_t* ndim_max,
                             int32_t* vec_field, const char** name) {
#define CLAW_PLUGIN_INFO(pid, P)                             \
    if (id == pid) {                                         \
        if (meqn) *meqn = P<double>::MEQN;                   \
        if (mwaves) *mwaves = P<double>::MWAVES;             \
        if (ndim_max) *ndim_max = P<double>::NDIM_MAX;       \
        if (vec_field) *vec_field = P<double>::VEC;          \
        if (name) *name = P<double>::name();                 \
        return CLAW_OK;                                      \
    }
    CLAW_PLUGINS(CLAW_PLUGIN_INFO)
#undef CLAW_PLUGIN_INFO
    return fail(CLAW_E_INVALID, "no plug-in solver with id %d", id);
}

void claw_desc_init(claw_desc* d) {
    if (!d) return;
    memset(d, 0, sizeof *d);
    d->ndim = 2;
    d->n[0] = d->n[1] = d->n[2] = 1;
    d->upper[0] = d->upper[1] = d->upper[2] = 1.0;
    d->limiter = CLAW_LIM_MC;
    d->dtype = CLAW_FP64;
    d->efix = 1;
    d->num_ghost = 2;
    d->rho = d->bulk = d->grav = 1.0;
    d->cfl_desired = 0.9;
    d->cfl_max = 1.0;
    d->dt_max = INFINITY;
}

claw_status claw_workspace_bytes(const claw_desc* d, size_t* bytes) {
    claw_status st = validate(d);
    if (st) return st;
    if (!bytes) return fail(CLAW_E_INVALID, "bytes is NULL");
    *bytes = make_plan(d).total;
    return CLAW_OK;
}

claw_status claw_create(const claw_desc* d, void* q, const void* aux, void* workspace,
                        size_t workspace_bytes, void* stream, claw_solver** out) {
    claw_status st = validate(d);
    if (st) return st;
    if (!out) return fail(CLAW_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!q) return fail(CLAW_E_INVALID, "q is NULL");
    if (!workspace) return fail(CLAW_E_INVALID, "workspace is NULL");
    if ((d->maux != 0) != (aux != nullptr)) return fail(CLAW_E_INVALID, "aux must be given iff maux = 2");
    Plan p = make_plan(d);
    if (workspace_bytes < p.total)
        return fail(CLAW_E_INVALID, "workspace too small: %zu < %zu bytes", workspace_bytes, p.total);
    if (((uintptr_t)q % 256) || ((uintptr_t)workspace % 256) || (aux && ((uintptr_t)aux % 16)))
        return fail(CLAW_E_INVALID, "q and workspace must be 256-byte aligned");
    claw_solver* h = new (std::nothrow) claw_solver();
    if (!h) return fail(CLAW_E_HIP, "out of host memory");
    bind_solver(h, d, p, q, (char*)workspace, (hipStream_t)stream);
    hipError_t e = hipStreamCreateWithFlags(&h->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete h;
        return fail(CLAW_E_HIP, "stream create failed: %s", hipGetErrorString(e));
    }
    e = setup_kernels(h, aux);
    if (e != hipSuccess) {
        (void)hipStreamDestroy(h->cap_stream);
        delete h;
        return fail(CLAW_E_HIP, "set-up kernels failed: %s", hipGetErrorString(e));
    }
    *out = h;
    return CLAW_OK;
}

claw_status claw_cfl(claw_solver* h, double* sigma, double* smax) {
    if (!h) return fail(CLAW_E_INVALID, "solver is NULL");
    claw_status st = commit(h);
    if (!st) st = speed_pass(h);
    if (st) return st;
    Ctrl c;
    st = read_ctrl(h, &c);
    if (st) return st;
    const int q = committed(h);
    if (c.nonphys[q]) return fail(CLAW_E_NONPHYSICAL, "non-physical state (depth <= 0 or not finite)");
    double sg = 0;
    for (int k = 0; k < 3; ++k) {
        double v = 0;
        if (k < h->d.ndim) {
            v = smax_value(h, c, q, k);
            if (v / h->dx[k] > sg) sg = v / h->dx[k];
        }
        if (smax) smax[k] = v;
    }
    if (sigma) *sigma = sg;
    return CLAW_OK;
}

claw_status claw_step(claw_solver* h, double dt, double* cfl) {
    if (!h) return fail(CLAW_E_INVALID, "solver is NULL");
    if (!(dt > 0) || !isfinite(dt)) return fail(CLAW_E_INVALID, "dt must be positive and finite");
    claw_status st = commit(h);
    if (st) return st;
    HIP_TRY(launch_begin(h->ctrl, committed(h), dt, MODE_STEP, result_offset_of(h), h->stream));
    st = enqueue_trial(h, h->stream, nullptr);
    if (!st) st = commit(h);
    if (st || !cfl) return st;
    StepState S;
    st = read_state(h, &S);
    if (st) return st;
    *cfl = S.cfl;
    st = ctrl_status(S);
    if (st) return st;
    if (!S.last_accepted) return fail(CLAW_E_CFL, "step rejected: Courant number %.6g > %.6g", S.cfl, h->d.cfl_max);
    return CLAW_OK;
}

claw_status claw_sweep(claw_solver* h, int32_t dir, double dt, double* smax) {
    if (!h) return fail(CLAW_E_INVALID, "solver is NULL");
    if (dir < 0 || dir >= h->d.ndim) return fail(CLAW_E_INVALID, "direction %d out of range", dir);
    if (!(dt >= 0) || !isfinite(dt)) return fail(CLAW_E_INVALID, "dt must be finite and >= 0");
    claw_status st = commit(h);
    if (st) return st;
    HIP_TRY(launch_begin(h->ctrl, committed(h), dt, MODE_FIXED, 1, h->stream));
    HIP_TRY(enqueue_sweep(h, dir, 0, 1, false, h->parity, true, true, h->stream));
    h->parity ^= 1;
    st = commit(h);
    if (st || !smax) return st;
    Ctrl c;
    st = read_ctrl(h, &c);
    if (st) return st;
    const int q = committed(h);
    if (c.nonphys[q]) return fail(CLAW_E_NONPHYSICAL, "non-physical state (depth <= 0 or not finite)");
    *smax = smax_value(h, c, q, dir);
    return CLAW_OK;
}

// The adaptive loop: one speed pass (skipped when a previous run left the
// next step), then as many trials as steps are asked for, replayed from the
// graph ladder; the state is copied back into q and the committed step state
// read once.  A rejected trial leaves one step to do, so the loop repeats with
// that many trials (each repetition costs one more read).
claw_status claw_advance(claw_solver* h, int64_t nsteps, double dt0, double* t, int64_t* nreject) {
    if (!h) return fail(CLAW_E_INVALID, "solver is NULL");
    if (nsteps < 0) return fail(CLAW_E_INVALID, "nsteps must be >= 0");
    return run_adaptive(h, nsteps, dt0, true, t, nreject);
}

claw_status claw_advance_fixed(claw_solver* h, int64_t nsteps, const double* dts, double* cfl_log) {
    if (!h) return fail(CLAW_E_INVALID, "solver is NULL");
    if (nsteps < 0 || (nsteps > 0 && !dts)) return fail(CLAW_E_INVALID, "bad step list");
    for (int64_t k = 0; k < nsteps; ++k)
        if (!(dts[k] > 0) || !isfinite(dts[k])) return fail(CLAW_E_INVALID, "dts[%lld] not positive", (long long)k);
    claw_status st = CLAW_OK;
    bool uniform = !cfl_log && nsteps >= kGraphSteps;
    for (int64_t k = 1; k < nsteps && uniform; ++k) uniform = dts[k] == dts[0];
    if (uniform) {
        // one begin, then captured trials: a fixed-dt trial keeps its dt and is
        // accepted by the next trial's first sweep
        st = commit(h);
        if (st) return st;
        HIP_TRY(launch_begin(h->ctrl, committed(h), dts[0], MODE_FIXED, result_offset_of(h), h->stream));
        st = replay_trials(h, nsteps);
        if (!st) st = commit(h);
        if (!st) st = sync_state(h);
        if (st) return st;
        StepState S;
        st = read_state(h, &S);
        if (st) return st;
        return ctrl_status(S);
    }
    for (int64_t k = 0; k < nsteps; ++k) {
        st = commit(h);
        if (st) return st;
        HIP_TRY(launch_begin(h->ctrl, committed(h), dts[k], MODE_FIXED, result_offset_of(h), h->stream));
        st = enqueue_trial(h, h->stream, nullptr);
        if (!st) st = commit(h);
        if (st) return st;
        if (cfl_log)
            HIP_TRY(hipMemcpyAsync(&cfl_log[k], &h->ctrl->st[committed(h)].cfl, sizeof(double),
                                   hipMemcpyDeviceToHost, h->stream));
    }
    st = sync_state(h);
    if (st) return st;
    StepState S;
    st = read_state(h, &S);
    if (st) return st;
    return ctrl_status(S);
}

claw_status claw_advance_timed(claw_solver* h, int64_t nsteps, double* kernel_ms, int64_t* launches) {
    if (!h) return fail(CLAW_E_INVALID, "solver is NULL");
    if (nsteps < 0) return fail(CLAW_E_INVALID, "nsteps must be >= 0");
    double ms[4] = {0, 0, 0, 0};
    int64_t cnt[4] = {0, 0, 0, 0};
    const int per = 2 * h->d.ndim;  // events per trial: one before each sweep and one after the last
    const int batch = 64;
    while ((int)h->events.size() < batch * per) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        h->events.push_back(e);
    }
    claw_status st = commit(h);
    if (st) return st;
    if (nsteps > 0) {
        st = begin_adaptive(h, 0.0);
        if (st) return st;
        HIP_TRY(launch_set_target(h->ctrl, committed(h), nsteps, h->stream));
        int64_t remaining = nsteps;
        while (remaining > 0) {
            const int64_t n = remaining < batch ? remaining : batch;
            for (int64_t k = 0; k < n; ++k) {
                st = enqueue_trial(h, h->stream, &h->events[k * per]);
                if (st) return st;
            }
            st = commit(h);
            if (st) return st;
            HIP_TRY(hipStreamSynchronize(h->stream));
            int dirs[5], so[5], dof[5];
            // timed kernels per trial (the fused 3D x and y step counts in slot 0)
            const int nk = h->fused ? 1 : (h->fused3 ? 2 : trial_sweeps(h, dirs, so, dof));
            for (int64_t k = 0; k < n; ++k) {
                hipEvent_t* ev = &h->events[k * per];
                for (int j = 0; j < nk; ++j) {
                    float v = 0;
                    HIP_TRY(hipEventElapsedTime(&v, ev[j], ev[j + 1]));
                    const int slot = h->fused ? 0 : (h->fused3 ? 2 * j : dirs[j]);
                    ms[slot] += v;
                    cnt[slot] += 1;
                }
            }
            Ctrl c;
            st = read_ctrl(h, &c);
            if (st) return st;
            const StepState& S = c.st[committed(h)];
            if (S.err) return ctrl_status(S);
            if (S.done) break;
            remaining = S.target - S.accepted;
        }
    }
    st = sync_state(h);
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(h->stream));
    for (int k = 0; k < 4; ++k) {
        if (kernel_ms) kernel_ms[k] = ms[k];
        if (launches) launches[k] = cnt[k];
    }
    return CLAW_OK;
}

claw_status claw_sync_state(claw_solver* h) {
    if (!h) return fail(CLAW_E_INVALID, "solver is NULL");
    claw_status st = commit(h);
    if (st) return st;
    return sync_state(h);
}

claw_status claw_get_control(claw_solver* h, double* t, double* dt_next, int64_t* accepted, int64_t* rejected) {
    if (!h) return fail(CLAW_E_INVALID, "solver is NULL");
    claw_status st = commit(h);
    if (st) return st;
    StepState S;
    st = read_state(h, &S);
    if (st) return st;
    if (t) *t = S.t;
    if (dt_next) *dt_next = S.dt_next;
    if (accepted) *accepted = S.accepted;
    if (rejected) *rejected = S.rejected;
    return CLAW_OK;
}

claw_status claw_set_control(claw_solver* h, double t, double dt_next) {
    if (!h) return fail(CLAW_E_INVALID, "solver is NULL");
    if (!isfinite(t) || !(dt_next >= 0)) return fail(CLAW_E_INVALID, "bad control values");
    claw_status st = commit(h);
    if (st) return st;
    HIP_TRY(launch_set_control(h->ctrl, committed(h), t, dt_next, h->stream));
    return CLAW_OK;
}

claw_status claw_destroy(claw_solver* h) {
    if (!h) return CLAW_OK;
    hipError_t e = hipStreamSynchronize(h->stream);
    for (int r = 0; r < 4; ++r)
        for (int p = 0; p < 2; ++p) {
            if (h->gexec[r][p]) (void)hipGraphExecDestroy(h->gexec[r][p]);
            if (h->graph[r][p]) (void)hipGraphDestroy(h->graph[r][p]);
        }
    if (h->lc_exec) (void)hipGraphExecDestroy(h->lc_exec);
    if (h->lc_graph) (void)hipGraphDestroy(h->lc_graph);
    for (hipEvent_t ev : h->events) (void)hipEventDestroy(ev);
    if (h->cap_stream) (void)hipStreamDestroy(h->cap_stream);
    delete h;
    if (e != hipSuccess) return fail(CLAW_E_HIP, "stream sync failed: %s", hipGetErrorString(e));
    return CLAW_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Sweep without allocation: the control block and the derived acoustic
// coefficients of claw_sweep_noalloc live in `scratch`, a static device array
// each GPU holds for the life of the process.  Host code never passes the
// array's name to a kernel (in host code it is only a stand-in for the symbol):
// its device address is looked up once per device with hipGetSymbolAddress
// and kept in g_scratch_ptr.  Calls that overlap on one GPU share the array.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchCtrlBytes = 32768;  // the control block, rounded up
static_assert(sizeof(Ctrl) <= kScratchCtrlBytes, "control block exceeds its scratch slot");
constexpr size_t kScratchBytes = kScratchCtrlBytes + ((size_t)CLAW_NOALLOC_ZC_BYTES);
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];

// Device address of the current device's scratch array (looked up on the
// first call on that device).
claw_status scratch_of_current_device(char** out) {
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CLAW_E_UNSUPPORTED, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(CLAW_E_HIP, "scratch symbol lookup failed on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = (char*)g_scratch_ptr[dev];
    return CLAW_OK;
}

}  // namespace

extern "C" {

claw_status claw_sweep_noalloc(const claw_desc* d, const void* src, void* dst, const void* aux, int32_t dir,
                               double dt, double* smax_dev, void* stream) {
    claw_status st = validate(d);
    if (st) return st;
    if (!src || !dst) return fail(CLAW_E_INVALID, "src and dst must be device pointers");
    if (src == dst) return fail(CLAW_E_INVALID, "src and dst must not alias");
    if (dir < 0 || dir >= d->ndim) return fail(CLAW_E_INVALID, "direction %d out of range", dir);
    if (!(dt >= 0) || !isfinite(dt)) return fail(CLAW_E_INVALID, "dt must be finite and >= 0");
    if ((d->maux != 0) != (aux != nullptr)) return fail(CLAW_E_INVALID, "aux must be given iff maux = 2");
    if (d->flags & CLAW_FLAG_STRANG) return fail(CLAW_E_INVALID, "a single sweep takes no splitting flag");
    if (((uintptr_t)src % 16) || ((uintptr_t)dst % 16) || (aux && ((uintptr_t)aux % 16)))
        return fail(CLAW_E_INVALID, "src, dst and aux must be 16-byte aligned");
    const Plan p = make_plan(d);
    const size_t zc_bytes = d->maux ? (size_t)p.ncell * 2 * p.elem : 0;
    if (zc_bytes > (size_t)CLAW_NOALLOC_ZC_BYTES)
        return fail(CLAW_E_UNSUPPORTED,
                    "claw_sweep_noalloc: %zu bytes of derived coefficients exceed the %zu-byte scratch "
                    "limit (use claw_create with a workspace)",
                    zc_bytes, (size_t)CLAW_NOALLOC_ZC_BYTES);
    char* sp = nullptr;
    st = scratch_of_current_device(&sp);
    if (st) return st;
    // a handle on the stack over the scratch array: control block first, then
    // the coefficient fields; rotation buffers 0 = src, 1 = dst (2 unused)
    claw_solver h{};
    claw_desc dd = *d;
    dd.flags = CLAW_FLAG_SPLIT_STEP;
    bind_solver(&h, &dd, p, const_cast<void*>(src), sp, (hipStream_t)stream);
    h.ctrl = (Ctrl*)sp;
    h.buf[1] = dst;
    h.buf[2] = dst;
    h.zc = d->maux ? (void*)(sp + kScratchCtrlBytes) : nullptr;
    // fresh control block (speed slots and flags cleared by the kernel: no
    // memset node for a caller that captures this call), then the trial
    HIP_TRY(setup_kernels(&h, aux));
    const int q = committed(&h);
    HIP_TRY(launch_begin(h.ctrl, q, dt, MODE_FIXED, 1, h.stream));
    HIP_TRY(enqueue_sweep(&h, dir, 0, 1, false, h.parity, true, true, h.stream));
    h.parity ^= 1;
    HIP_TRY(launch_commit(h.ctrl, committed(&h), h.fp32, h.stream));
    if (smax_dev) HIP_TRY(launch_report_smax(h.ctrl, committed(&h), dir, h.fp32, smax_dev, h.stream));
    return CLAW_OK;
}

claw_status claw_debug_take(uint64_t* count, uint32_t* first_line) {
#ifdef CLAW_DEBUG
    if (hipDeviceSynchronize() != hipSuccess) return fail(CLAW_E_HIP, "device synchronisation failed");
    uint64_t n = 0;
    uint32_t first = 0;
    for (int k = 0; k < g_debug_n; ++k) {
        unsigned line = 0;
        n += g_debug_take[k](&line);
        if (!first && line) first = line;
    }
    if (count) *count = n;
    if (first_line) *first_line = first;
    return CLAW_OK;
#else
    if (count) *count = 0;
    if (first_line) *first_line = 0;
    return fail(CLAW_E_UNSUPPORTED, "not a debug build: the range checks are in libclaw_debug.so (CLAW_DEBUG)");
#endif
}

const char* claw_status_string(claw_status s) {
    switch (s) {
        case CLAW_OK: return "ok";
        case CLAW_E_INVALID: return "invalid argument";
        case CLAW_E_UNSUPPORTED: return "unsupported";
        case CLAW_E_HIP: return "HIP runtime error";
        case CLAW_E_CFL: return "step rejected (CFL)";
        case CLAW_E_NONPHYSICAL: return "non-physical state";
        case CLAW_E_STATE: return "step control failed";
    }
    return "unknown status";
}

const char* claw_last_error(void) { return g_err; }

}  // extern "C"

// ===========================================================================
// Batched ensembles of independent shallow-water grids (claw_batch_*)
// ===========================================================================

struct claw_batch {
    int count;
    bool fp32;
    std::vector<claw_desc> d;
    std::vector<Plan> plan;
    hipStream_t stream;
    hipStream_t cap_stream;
    char* ws;
    size_t off_ptrs, off_args, off_rows, off_cols, off_fused, off_fargs, off_bufs;
    size_t args_stride;  // bytes per SweepArgs of the dtype
    bool fused;          // one fused step kernel per trial for every instance (fused.hip)
    Ctrl** ctrl_ptrs;    // device array of the instances' control blocks
    std::vector<Ctrl*> ctrl;
    std::vector<std::array<void*, 3>> buf;
    int n_row_blocks, n_col_blocks, max_col_blocks, n_fused_blocks, max_fused_blocks;
    int chunk, schedule, rpw;
    double tuned_us;
    bool have_dt_next;
    int parity;
    hipGraphExec_t gexec[2];
    hipGraph_t graph[2];
};

namespace {

constexpr int kBatchChunkMin = 8;
const int kTuneChunks[] = {16, 32, 64, 128};
const int kTuneRpw[] = {2, 4, 8};
// fused batches: rows per fused workgroup (the column chunk of their speed passes too)
constexpr int kFusedChunkMin = 16;
const int kTuneFusedChunks[] = {16, 24, 32, 48, 64};

int inst_row_blocks(const claw_desc& d, bool fp32);
int inst_col_blocks(const claw_desc& d, int chunk);
int inst_fused_blocks(const claw_desc& d, bool fp32, int chunk);

// A batch takes the fused 2D step under the single grid's rule applied to
// its whole state: asked for (CLAW_FLAG_FUSED_STEP), or FP32 with at least
// CLAW_FUSED_AUTO_BYTES of state and not CLAW_FLAG_SPLIT_STEP.
bool batch_is_fused(const claw_desc* d, int count) {
    if (d[0].flags & CLAW_FLAG_FUSED_STEP) return true;
    if ((d[0].flags & CLAW_FLAG_SPLIT_STEP) || d[0].dtype != CLAW_FP32) return false;
    uint64_t bytes = 0;
    for (int i = 0; i < count; ++i) bytes += (uint64_t)d[i].n[0] * (uint64_t)d[i].n[1] * 3u * 4u;
    return bytes >= (uint64_t)CLAW_FUSED_AUTO_BYTES;
}

claw_status batch_validate(const claw_desc* d, int32_t count) {
    if (!d || count < 1 || count > 65535) return fail(CLAW_E_INVALID, "need 1..65535 descriptors");
    for (int i = 0; i < count; ++i) {
        claw_status st = validate(&d[i]);
        if (st) return st;
        if (d[i].riemann != CLAW_RP_SHALLOW_WATER || d[i].ndim != 2)
            return fail(CLAW_E_UNSUPPORTED, "batches hold 2D shallow-water instances (instance %d)", i);
        if (d[i].dtype != d[0].dtype) return fail(CLAW_E_INVALID, "all instances need the same dtype");
        if (d[i].flags & ~(CLAW_FLAG_FUSED_STEP | CLAW_FLAG_SPLIT_STEP))
            return fail(CLAW_E_UNSUPPORTED, "batches run the split or the fused 2D step (instance %d)", i);
        if ((d[i].flags & (CLAW_FLAG_FUSED_STEP | CLAW_FLAG_SPLIT_STEP)) !=
            (d[0].flags & (CLAW_FLAG_FUSED_STEP | CLAW_FLAG_SPLIT_STEP)))
            return fail(CLAW_E_INVALID, "all instances need the same step flags (instance %d)", i);
        if ((d[i].flags & CLAW_FLAG_FUSED_STEP) && (d[i].flags & CLAW_FLAG_SPLIT_STEP))
            return fail(CLAW_E_INVALID, "fused and split step both asked for (instance %d)", i);
    }
    // a batched sweep is one 1-D launch of 256-thread workgroups, and a
    // dispatch counts its work-items in 32 bits: at most 2^24 - 1 workgroups
    int64_t rows = 0, cols = 0, fused = 0;
    const bool is_fused = batch_is_fused(d, count);
    for (int i = 0; i < count; ++i) {
        rows += inst_row_blocks(d[i], d[0].dtype == CLAW_FP32);
        cols += inst_col_blocks(d[i], kBatchChunkMin);
        if (is_fused) fused += inst_fused_blocks(d[i], d[0].dtype == CLAW_FP32, kFusedChunkMin);
    }
    const int64_t max_blocks = ((int64_t)1 << 24) - 1;
    if (rows > max_blocks || cols > max_blocks || fused > max_blocks)
        return fail(CLAW_E_UNSUPPORTED, "batch too large for one launch (%lld row blocks, %lld column blocks)",
                    (long long)rows, (long long)cols);
    return CLAW_OK;
}

struct BatchPlan {
    size_t ctrl_stride, off_ptrs, off_args, off_rows, off_cols, off_fused, off_fargs, off_bufs, total, args_stride;
    int max_row_blocks, max_col_blocks, max_fused_blocks;
};

int row_cpl(bool fp32) { return fp32 ? 4 : 2; }

int inst_row_blocks(const claw_desc& d, bool fp32) {
    const int P = 62 * row_cpl(fp32);
    return (int)(((d.n[0] + P - 1) / P) * ((d.n[1] + 3) / 4));
}
int inst_col_blocks(const claw_desc& d, int chunk) {
    const int64_t sg = ((d.n[0] + 63) / 64 + 3) / 4;
    const int64_t c = chunk < d.n[1] ? chunk : d.n[1];
    return (int)(sg * ((d.n[1] + c - 1) / c));
}
// fused step: strips of 62 CPL columns times chunks of rows
int inst_fused_blocks(const claw_desc& d, bool fp32, int chunk) {
    const int64_t W = 62 * row_cpl(fp32);
    const int64_t c = chunk < d.n[1] ? chunk : d.n[1];
    return (int)(((d.n[0] + W - 1) / W) * ((d.n[1] + c - 1) / c));
}

BatchPlan batch_plan(const claw_desc* d, int count) {
    BatchPlan p;
    const bool fp32 = d[0].dtype == CLAW_FP32;
    p.ctrl_stride = (sizeof(Ctrl) + 255) / 256 * 256;
    p.args_stride = fp32 ? sizeof(SweepArgs<float>) : sizeof(SweepArgs<double>);
    p.off_ptrs = round_up(p.ctrl_stride * count);
    p.off_args = p.off_ptrs + round_up(sizeof(Ctrl*) * count);
    p.off_rows = p.off_args + round_up(p.args_stride * 2 * count);
    p.max_row_blocks = 0;
    p.max_col_blocks = 0;
    p.max_fused_blocks = 0;
    const bool fused = batch_is_fused(d, count);
    for (int i = 0; i < count; ++i) {
        p.max_row_blocks += inst_row_blocks(d[i], fp32);
        p.max_col_blocks += inst_col_blocks(d[i], kBatchChunkMin);
        if (fused) p.max_fused_blocks += inst_fused_blocks(d[i], fp32, kFusedChunkMin);
    }
    p.off_cols = p.off_rows + round_up(sizeof(BatchBlock) * p.max_row_blocks);
    p.off_fused = p.off_cols + round_up(sizeof(BatchBlock) * p.max_col_blocks);
    p.off_fargs = p.off_fused + round_up(sizeof(BatchBlock) * p.max_fused_blocks);
    p.off_bufs = p.off_fargs + (fused ? round_up((fp32 ? sizeof(FusedArgs<float>) : sizeof(FusedArgs<double>)) *
                                                 count) : 0);
    p.total = p.off_bufs;
    for (int i = 0; i < count; ++i) p.total += 2 * round_up(make_plan(&d[i]).state_bytes);
    return p;
}

// Block tables and per-instance sweep arguments for column chunk `chunk`,
// schedule 0 (largest instances first) or 1 (round-robin over instances) and
// rpw rows per row-sweep wavefront.
claw_status batch_tables(claw_batch* b, int chunk, int schedule, int rpw) {
    const int n = b->count;
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
        return b->plan[x].ncell > b->plan[y].ncell;
    });
    std::vector<std::vector<BatchBlock>> rows(n), cols(n), fus(n);
    const int P = 62 * row_cpl(b->fp32);
    for (int i = 0; i < n; ++i) {
        const claw_desc& d = b->d[i];
        const int segs = (int)((d.n[0] + P - 1) / P), groups = (int)((d.n[1] + 4 * rpw - 1) / (4 * rpw));
        const int nfull = (int)(d.n[0] / P), S = row_tail((int)d.n[0], row_cpl(b->fp32)).rows;
        for (int y = 0; y < groups; ++y)
            for (int x = 0; x < segs; ++x)
                if (x < nfull || (int64_t)y * 4 * rpw * S < d.n[1]) rows[i].push_back({i, x, y, 0});
        const int sg = (int)(((d.n[0] + 63) / 64 + 3) / 4);
        const int c = chunk < d.n[1] ? chunk : (int)d.n[1];
        const int nch = (int)((d.n[1] + c - 1) / c);
        for (int y = 0; y < nch; ++y)
            for (int x = 0; x < sg; ++x) cols[i].push_back({i, x, y, 0});
        if (b->fused) {  // the fused step's chunks are the columns' chunks
            const int strips = (int)((d.n[0] + 62 * row_cpl(b->fp32) - 1) / (62 * row_cpl(b->fp32)));
            for (int y = 0; y < nch; ++y)
                for (int x = 0; x < strips; ++x) fus[i].push_back({i, x, y, 0});
        }
    }
    auto flatten = [&](std::vector<std::vector<BatchBlock>>& per) {
        std::vector<BatchBlock> out;
        if (schedule == 0) {
            for (int i : order) out.insert(out.end(), per[i].begin(), per[i].end());
        } else {
            size_t k = 0;
            bool any = true;
            while (any) {
                any = false;
                for (int i : order)
                    if (k < per[i].size()) {
                        out.push_back(per[i][k]);
                        any = true;
                    }
                ++k;
            }
        }
        return out;
    };
    std::vector<BatchBlock> rt = flatten(rows), ct = flatten(cols), ft = flatten(fus);
    if ((int)ct.size() > b->max_col_blocks) return fail(CLAW_E_INVALID, "column chunk too small");
    if ((int)ft.size() > b->max_fused_blocks) return fail(CLAW_E_INVALID, "fused chunk too small");
    // per-instance arguments (x: cur -> cur+1, y: cur+1 -> cur+2)
    std::vector<char> args(b->args_stride * 2 * n);
    for (int i = 0; i < n; ++i) {
        void* bufs[3] = {b->buf[i][0], b->buf[i][1], b->buf[i][2]};
        for (int dir = 0; dir < 2; ++dir) {
            char* dst = args.data() + b->args_stride * (2 * i + dir);
            if (b->fp32) {
                SweepArgs<float> a = grid_args<float>(b->d[i], SYS_SW, b->plan[i].ncell, bufs, nullptr,
                                                      b->ctrl[i], dir, dir, dir + 1, chunk);
                memcpy(dst, &a, sizeof a);
            } else {
                SweepArgs<double> a = grid_args<double>(b->d[i], SYS_SW, b->plan[i].ncell, bufs, nullptr,
                                                        b->ctrl[i], dir, dir, dir + 1, chunk);
                memcpy(dst, &a, sizeof a);
            }
        }
    }
    HIP_TRY(hipMemcpyAsync(b->ws + b->off_args, args.data(), args.size(), hipMemcpyHostToDevice, b->stream));
    if (b->fused) {  // per-instance fused-step arguments: x sweep from cur to cur + 1, rows per chunk
        const size_t fs = b->fp32 ? sizeof(FusedArgs<float>) : sizeof(FusedArgs<double>);
        std::vector<char> fargs(fs * n);
        for (int i = 0; i < n; ++i) {
            void* bufs[3] = {b->buf[i][0], b->buf[i][1], b->buf[i][2]};
            const int c = chunk < b->d[i].n[1] ? chunk : (int)b->d[i].n[1];
            if (b->fp32) {
                FusedArgs<float> F;
                memset(&F, 0, sizeof F);
                F.a = grid_args<float>(b->d[i], SYS_SW, b->plan[i].ncell, bufs, nullptr, b->ctrl[i], 0, 0, 1, 0);
                F.ny = (int32_t)b->d[i].n[1];
                F.bcy_lo = b->d[i].bc_lo[1];
                F.bcy_hi = b->d[i].bc_hi[1];
                F.chunk = c;
                memcpy(fargs.data() + fs * i, &F, sizeof F);
            } else {
                FusedArgs<double> F;
                memset(&F, 0, sizeof F);
                F.a = grid_args<double>(b->d[i], SYS_SW, b->plan[i].ncell, bufs, nullptr, b->ctrl[i], 0, 0, 1, 0);
                F.ny = (int32_t)b->d[i].n[1];
                F.bcy_lo = b->d[i].bc_lo[1];
                F.bcy_hi = b->d[i].bc_hi[1];
                F.chunk = c;
                memcpy(fargs.data() + fs * i, &F, sizeof F);
            }
        }
        HIP_TRY(hipMemcpyAsync(b->ws + b->off_fargs, fargs.data(), fargs.size(), hipMemcpyHostToDevice, b->stream));
        HIP_TRY(hipMemcpyAsync(b->ws + b->off_fused, ft.data(), ft.size() * sizeof(BatchBlock),
                               hipMemcpyHostToDevice, b->stream));
    }
    HIP_TRY(hipMemcpyAsync(b->ws + b->off_rows, rt.data(), rt.size() * sizeof(BatchBlock), hipMemcpyHostToDevice,
                           b->stream));
    HIP_TRY(hipMemcpyAsync(b->ws + b->off_cols, ct.data(), ct.size() * sizeof(BatchBlock), hipMemcpyHostToDevice,
                           b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    b->n_row_blocks = (int)rt.size();
    b->n_col_blocks = (int)ct.size();
    b->n_fused_blocks = (int)ft.size();
    b->chunk = chunk;
    b->schedule = schedule;
    b->rpw = rpw;
    for (int p = 0; p < 2; ++p) {  // launch sizes changed: recapture
        if (b->gexec[p]) (void)hipGraphExecDestroy(b->gexec[p]);
        if (b->graph[p]) (void)hipGraphDestroy(b->graph[p]);
        b->gexec[p] = nullptr;
        b->graph[p] = nullptr;
    }
    return CLAW_OK;
}

template <typename R>
hipError_t batch_sweep(claw_batch* b, int dir, bool speeds, int parity, bool first, bool last, hipStream_t s) {
    BatchLaunch<R> L;
    L.blocks = (const BatchBlock*)(b->ws + (dir == 0 ? b->off_rows : b->off_cols));
    L.args = (const SweepArgs<R>*)(b->ws + b->off_args);
    L.parity = parity;
    L.first = first ? 1 : 0;
    L.last = last ? 1 : 0;
    L.limiter = b->d[0].limiter;
    L.rpw = b->rpw;
    for (const claw_desc& d : b->d)
        if (d.limiter != L.limiter) L.limiter = -1;
    return launch_batch_sweep<R>(L, SYS_SW, dir, dir == 0 ? b->n_row_blocks : b->n_col_blocks, speeds, s);
}

hipError_t batch_sweep_any(claw_batch* b, int dir, bool speeds, int parity, bool first, bool last, hipStream_t s) {
    return b->fp32 ? batch_sweep<float>(b, dir, speeds, parity, first, last, s)
                   : batch_sweep<double>(b, dir, speeds, parity, first, last, s);
}

template <typename R>
hipError_t batch_step2d(claw_batch* b, hipStream_t s) {
    BatchFusedLaunch<R> L;
    L.blocks = (const BatchBlock*)(b->ws + b->off_fused);
    L.args = (const FusedArgs<R>*)(b->ws + b->off_fargs);
    L.parity = b->parity;
    L.limiter = b->d[0].limiter;
    for (const claw_desc& d : b->d)
        if (d.limiter != L.limiter) L.limiter = -1;
    return launch_batch_step2d<R>(L, b->n_fused_blocks, s);
}

// Result buffer offset of a trial: the fused step writes cur + 1, the x and y
// sweeps cur + 2.
int batch_result_off(const claw_batch* b) { return b->fused ? 1 : 2; }

claw_status batch_trial(claw_batch* b, hipStream_t s) {
    if (b->fused) {  // every instance's opening (one thread each), then one fused launch
        HIP_TRY(launch_batch_ctrl(b->ctrl_ptrs, b->count, BOP_OPEN, b->parity, 0.0, 0, batch_result_off(b), 0,
                                  b->fp32, s));
        HIP_TRY(b->fp32 ? batch_step2d<float>(b, s) : batch_step2d<double>(b, s));
        b->parity ^= 1;
        return CLAW_OK;
    }
    HIP_TRY(batch_sweep_any(b, 0, false, b->parity, true, false, s));
    HIP_TRY(batch_sweep_any(b, 1, false, b->parity, false, true, s));
    b->parity ^= 1;
    return CLAW_OK;
}

claw_status batch_ctrl(claw_batch* b, int op, double dt = 0, int mode = 0, long long nsteps = 0) {
    HIP_TRY(launch_batch_ctrl(b->ctrl_ptrs, b->count, op, b->parity ^ 1, dt, mode, batch_result_off(b), nsteps,
                              b->fp32, b->stream));
    return CLAW_OK;
}

claw_status batch_read(claw_batch* b, std::vector<Ctrl>& out) {
    out.resize(b->count);
    for (int i = 0; i < b->count; ++i)
        HIP_TRY(hipMemcpyAsync(&out[i], b->ctrl[i], sizeof(Ctrl), hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return CLAW_OK;
}

claw_status batch_graph(claw_batch* b) {
    const int p = b->parity;
    if (b->gexec[p]) return CLAW_OK;
    HIP_TRY(hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
    claw_status st = CLAW_OK;
    for (int k = 0; k < kGraphSteps && st == CLAW_OK; ++k) st = batch_trial(b, b->cap_stream);
    b->parity = p;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(CLAW_E_HIP, "batch graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->gexec[p], g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        b->gexec[p] = nullptr;
        return fail(CLAW_E_HIP, "batch graph instantiate failed: %s", hipGetErrorString(e));
    }
    b->graph[p] = g;
    return CLAW_OK;
}

std::string tune_key(const claw_batch* b) {
    int64_t cells = 0;
    for (int i = 0; i < b->count; ++i) cells += b->plan[i].ncell;
    int lg = 0;
    while ((int64_t(1) << (lg + 1)) <= cells) ++lg;
    char key[128];
    snprintf(key, sizeof key, "gfx950/%s/sw%s/n%d/cells2^%d", b->fp32 ? "f32" : "f64", b->fused ? "-fused" : "",
             b->count, lg);
    return key;
}

bool cache_lookup(const char* path, const std::string& key, int* chunk, int* schedule, int* rpw, double* us) {
    FILE* f = path ? fopen(path, "r") : nullptr;
    if (!f) return false;
    char line[512];
    bool found = false;
    const std::string pat = "\"" + key + "\"";
    while (fgets(line, sizeof line, f)) {
        const char* p = strstr(line, pat.c_str());
        if (!p) continue;
        const char* c = strstr(p, "\"chunk\":");
        const char* s = strstr(p, "\"schedule\":");
        const char* r = strstr(p, "\"rows_per_wave\":");
        const char* u = strstr(p, "\"us_per_step\":");
        if (c && s && r && u && sscanf(c + 8, "%d", chunk) == 1 && sscanf(s + 11, "%d", schedule) == 1 &&
            sscanf(r + 16, "%d", rpw) == 1 && sscanf(u + 14, "%lf", us) == 1)
            found = true;
    }
    fclose(f);
    return found;
}

void cache_store(const char* path, const std::string& key, int chunk, int schedule, int rpw, double us) {
    if (!path) return;
    std::vector<std::string> keep;
    if (FILE* f = fopen(path, "r")) {
        char line[512];
        const std::string pat = "\"" + key + "\"";
        while (fgets(line, sizeof line, f)) {
            std::string l(line);
            if (l.find("\"gfx") != std::string::npos && l.find(pat) == std::string::npos) {
                while (!l.empty() && (l.back() == '\n' || l.back() == ',')) l.pop_back();
                keep.push_back(l);
            }
        }
        fclose(f);
    }
    char entry[512];
    snprintf(entry, sizeof entry,
             "  \"%s\": {\"chunk\": %d, \"schedule\": %d, \"rows_per_wave\": %d, \"us_per_step\": %.3f}",
             key.c_str(), chunk, schedule, rpw, us);
    keep.push_back(entry);
    FILE* f = fopen(path, "w");
    if (!f) return;
    fprintf(f, "{\n");
    for (size_t i = 0; i < keep.size(); ++i) fprintf(f, "%s%s\n", keep[i].c_str(), i + 1 < keep.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
}

}  // namespace

extern "C" {

claw_status claw_batch_workspace_bytes(const claw_desc* descs, int32_t count, size_t* bytes) {
    claw_status st = batch_validate(descs, count);
    if (st) return st;
    if (!bytes) return fail(CLAW_E_INVALID, "bytes is NULL");
    *bytes = batch_plan(descs, count).total;
    return CLAW_OK;
}

claw_status claw_batch_create(const claw_desc* descs, int32_t count, void* const* q, void* workspace,
                              size_t workspace_bytes, void* stream, claw_batch** out) {
    claw_status st = batch_validate(descs, count);
    if (st) return st;
    if (!out || !q || !workspace) return fail(CLAW_E_INVALID, "NULL argument");
    *out = nullptr;
    const BatchPlan bp = batch_plan(descs, count);
    if (workspace_bytes < bp.total)
        return fail(CLAW_E_INVALID, "workspace too small: %zu < %zu bytes", workspace_bytes, bp.total);
    if ((uintptr_t)workspace % 256) return fail(CLAW_E_INVALID, "workspace must be 256-byte aligned");
    for (int i = 0; i < count; ++i)
        if (!q[i] || (uintptr_t)q[i] % 256) return fail(CLAW_E_INVALID, "q[%d] NULL or not 256-byte aligned", i);
    claw_batch* b = new (std::nothrow) claw_batch();
    if (!b) return fail(CLAW_E_HIP, "out of host memory");
    b->count = count;
    b->fp32 = descs[0].dtype == CLAW_FP32;
    b->d.assign(descs, descs + count);
    b->stream = (hipStream_t)stream;
    b->ws = (char*)workspace;
    b->off_ptrs = bp.off_ptrs;
    b->off_args = bp.off_args;
    b->off_rows = bp.off_rows;
    b->off_cols = bp.off_cols;
    b->off_fused = bp.off_fused;
    b->off_fargs = bp.off_fargs;
    b->off_bufs = bp.off_bufs;
    b->fused = batch_is_fused(descs, count);
    b->max_fused_blocks = bp.max_fused_blocks;
    b->args_stride = bp.args_stride;
    b->max_col_blocks = bp.max_col_blocks;
    b->ctrl_ptrs = (Ctrl**)(b->ws + bp.off_ptrs);
    size_t off = bp.off_bufs;
    for (int i = 0; i < count; ++i) {
        b->plan.push_back(make_plan(&descs[i]));
        b->ctrl.push_back((Ctrl*)(b->ws + bp.ctrl_stride * i));
        std::array<void*, 3> bufs;
        bufs[0] = q[i];
        bufs[1] = b->ws + off;
        off += round_up(b->plan[i].state_bytes);
        bufs[2] = b->ws + off;
        off += round_up(b->plan[i].state_bytes);
        b->buf.push_back(bufs);
    }
    hipError_t e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete b;
        return fail(CLAW_E_HIP, "stream create failed: %s", hipGetErrorString(e));
    }
    auto bail = [&](claw_status s) {
        (void)hipStreamDestroy(b->cap_stream);
        delete b;
        return s;
    };
    for (int i = 0; i < count; ++i) {
        double dx[3];
        for (int k = 0; k < 3; ++k) dx[k] = k < 2 ? (descs[i].upper[k] - descs[i].lower[k]) / (double)descs[i].n[k] : 1.0;
        e = launch_ctrl_init(b->ctrl[i], dx, 2, descs[i].cfl_desired, descs[i].cfl_max, descs[i].dt_max, false,
                             batch_result_off(b), b->stream);
        if (e != hipSuccess) return bail(fail(CLAW_E_HIP, "control init failed: %s", hipGetErrorString(e)));
    }
    e = hipMemcpyAsync(b->ctrl_ptrs, b->ctrl.data(), sizeof(Ctrl*) * count, hipMemcpyHostToDevice, b->stream);
    if (e != hipSuccess) return bail(fail(CLAW_E_HIP, "upload failed: %s", hipGetErrorString(e)));
    b->parity = 0;
    st = batch_tables(b, 32, 0, ROW_RPW_BATCH_DEFAULT);
    if (st) return bail(st);
    *out = b;
    return CLAW_OK;
}

claw_status claw_batch_tune(claw_batch* b, const char* cache_path, int32_t* chunk_out, int32_t* schedule_out,
                            int32_t* rows_per_wave_out, double* us_per_step) {
    if (!b) return fail(CLAW_E_INVALID, "batch is NULL");
    const std::string key = tune_key(b);
    int chunk = 0, schedule = 0, rpw = 0;
    double best = 0;
    bool cached = cache_lookup(cache_path, key, &chunk, &schedule, &rpw, &best);
    // an entry that is no valid tile choice (an edited or damaged file) counts as a miss
    const int chunk_min = b->fused ? kFusedChunkMin : kBatchChunkMin;
    if (cached && (chunk < chunk_min || chunk > 4096 || (schedule != 0 && schedule != 1) ||
                   !batch_rpw_ok(rpw) || !(best > 0)))
        cached = false;
    if (!cached) {
        // time a few state-preserving trials (dt = 0, always accepted) per candidate
        claw_status st = batch_ctrl(b, BOP_COMMIT);
        if (st) return st;
        std::vector<Ctrl> saved;
        st = batch_read(b, saved);
        if (st) return st;
        hipEvent_t e0, e1;
        HIP_TRY(hipEventCreate(&e0));
        HIP_TRY(hipEventCreate(&e1));
        best = 1e300;
        // candidates: schedule x column chunk x rows per row wavefront
        // (fused batches: schedule x rows per fused workgroup; the row table
        // serves only their speed passes)
        std::vector<std::array<int, 3>> cand;
        for (int sched = 0; sched < 2; ++sched) {
            if (b->fused) {
                for (int c : kTuneFusedChunks) cand.push_back({sched, c, ROW_RPW_BATCH_DEFAULT});
            } else {
                for (int c : kTuneChunks)
                    for (int r : kTuneRpw) cand.push_back({sched, c, r});
            }
        }
        for (const auto& cd : cand) {
            st = batch_tables(b, cd[1], cd[0], cd[2]);
            if (st) break;
            const int reps = 6;
            for (int k = 0; k < 2 + reps && st == CLAW_OK; ++k) {
                if (k == 2) HIP_TRY(hipEventRecord(e0, b->stream));
                st = batch_ctrl(b, BOP_BEGIN_FIXED, 0.0, MODE_FIXED);
                if (!st) st = batch_trial(b, b->stream);
                if (!st) st = batch_ctrl(b, BOP_COMMIT);
            }
            if (st) break;
            HIP_TRY(hipEventRecord(e1, b->stream));
            HIP_TRY(hipEventSynchronize(e1));
            float ms = 0;
            HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
            const double us = ms * 1e3 / reps;
            if (us < best) {
                best = us;
                schedule = cd[0];
                chunk = cd[1];
                rpw = cd[2];
            }
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st) return st;
        for (int i = 0; i < b->count; ++i)  // restore the control state the trials advanced
            HIP_TRY(hipMemcpyAsync(b->ctrl[i], &saved[i], sizeof(Ctrl), hipMemcpyHostToDevice, b->stream));
        HIP_TRY(hipStreamSynchronize(b->stream));
        cache_store(cache_path, key, chunk, schedule, rpw, best);
    }
    claw_status st = batch_tables(b, chunk, schedule, rpw);
    if (st) return st;
    b->tuned_us = best;
    if (chunk_out) *chunk_out = chunk;
    if (schedule_out) *schedule_out = schedule;
    if (rows_per_wave_out) *rows_per_wave_out = rpw;
    if (us_per_step) *us_per_step = best;
    return CLAW_OK;
}

claw_status claw_batch_set_tiles(claw_batch* b, int32_t chunk, int32_t schedule, int32_t rows_per_wave) {
    if (!b) return fail(CLAW_E_INVALID, "batch is NULL");
    if (chunk < (b->fused ? kFusedChunkMin : kBatchChunkMin) || (schedule != 0 && schedule != 1) ||
        !batch_rpw_ok(rows_per_wave))
        return fail(CLAW_E_INVALID, "bad tile choice");
    return batch_tables(b, chunk, schedule, rows_per_wave);
}

claw_status claw_batch_advance(claw_batch* b, int64_t nsteps, double* t, int64_t* nreject) {
    if (!b) return fail(CLAW_E_INVALID, "batch is NULL");
    if (nsteps < 0) return fail(CLAW_E_INVALID, "nsteps must be >= 0");
    claw_status st = batch_ctrl(b, BOP_COMMIT);
    if (st) return st;
    std::vector<Ctrl> c0;
    st = batch_read(b, c0);
    if (st) return st;
    if (nsteps > 0) {
        if (!b->have_dt_next) {  // first trial steps from a speed pass of every instance
            st = batch_ctrl(b, BOP_ZERO_SPEEDS);
            if (st) return st;
            for (int dir = 0; dir < 2; ++dir)
                HIP_TRY(batch_sweep_any(b, dir, true, b->parity ^ 1, false, false, b->stream));
        }
        st = batch_ctrl(b, BOP_BEGIN_ADAPT, 0.0, MODE_ADAPT, nsteps);
        if (st) return st;
        st = batch_graph(b);
        if (st) return st;
        int64_t remaining = nsteps;
        for (int round = 0; round < 1000 && remaining > 0; ++round) {
            const int64_t reps = (remaining + kGraphSteps - 1) / kGraphSteps;
            for (int64_t r = 0; r < reps; ++r) HIP_TRY(hipGraphLaunch(b->gexec[b->parity], b->stream));
            st = batch_ctrl(b, BOP_COMMIT);
            if (st) return st;
            std::vector<Ctrl> c;
            st = batch_read(b, c);
            if (st) return st;
            remaining = 0;
            for (int i = 0; i < b->count; ++i) {
                const StepState& S = c[i].st[b->parity ^ 1];
                if (S.err) return ctrl_status(S);
                if (!S.done && S.target - S.accepted > remaining) remaining = S.target - S.accepted;
            }
        }
        b->have_dt_next = true;
    }
    for (int i = 0; i < b->count; ++i) {
        hipError_t e = b->fp32 ? launch_sync_state<float>(b->ctrl[i], b->parity ^ 1, (float*)b->buf[i][0],
                                                          (float*)b->buf[i][1], (float*)b->buf[i][2],
                                                          b->plan[i].ncell * 3, b->stream)
                               : launch_sync_state<double>(b->ctrl[i], b->parity ^ 1, (double*)b->buf[i][0],
                                                           (double*)b->buf[i][1], (double*)b->buf[i][2],
                                                           b->plan[i].ncell * 3, b->stream);
        HIP_TRY(e);
    }
    std::vector<Ctrl> c;
    st = batch_read(b, c);
    if (st) return st;
    for (int i = 0; i < b->count; ++i) {
        const StepState& S = c[i].st[b->parity ^ 1];
        const StepState& S0 = c0[i].st[b->parity ^ 1];
        if (t) t[i] = S.t;
        if (nreject) nreject[i] = S.rejected - S0.rejected;
        if (S.accepted - S0.accepted != nsteps) return fail(CLAW_E_STATE, "instance %d stopped early", i);
    }
    return CLAW_OK;
}

claw_status claw_batch_destroy(claw_batch* b) {
    if (!b) return CLAW_OK;
    hipError_t e = hipStreamSynchronize(b->stream);
    for (int p = 0; p < 2; ++p) {
        if (b->gexec[p]) (void)hipGraphExecDestroy(b->gexec[p]);
        if (b->graph[p]) (void)hipGraphDestroy(b->graph[p]);
    }
    if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
    delete b;
    if (e != hipSuccess) return fail(CLAW_E_HIP, "stream sync failed: %s", hipGetErrorString(e));
    return CLAW_OK;
}

}  // extern "C"

// ===========================================================================
// Learned coarse-grid flux correction (learned.hip): parameter block and
// workspace layout, validation, and the composed learned step.
// ===========================================================================
namespace {

constexpr size_t kLcAlign = 256;
size_t lc_round(size_t v) { return (v + kLcAlign - 1) / kLcAlign * kLcAlign; }

// Parameter block: masters, Adam m, Adam v (FP32, both networks), then the
// BF16 copies W1 [2][64][16], W2 [2][64][64], W3 [2][16][64].
struct LcParamPlan {
    size_t off_m, off_v, off_w1b, off_w2b, off_w3b, total;
};
LcParamPlan lc_param_plan() {
    LcParamPlan p;
    const size_t vec = lc_round(sizeof(float) * LC_NPARAM);
    p.off_m = vec;
    p.off_v = 2 * vec;
    p.off_w1b = 3 * vec;
    p.off_w2b = p.off_w1b + lc_round(2 * 2 * LC_W1B);
    p.off_w3b = p.off_w2b + lc_round(2 * 2 * LC_W2B);
    p.total = p.off_w3b + lc_round(2 * 2 * LC_W3B);
    return p;
}

LcParams lc_params(void* base) {
    const LcParamPlan p = lc_param_plan();
    char* b = (char*)base;
    LcParams a;
    a.theta = (float*)b;
    a.m = (float*)(b + p.off_m);
    a.v = (float*)(b + p.off_v);
    a.w1b = (unsigned short*)(b + p.off_w1b);
    a.w2b = (unsigned short*)(b + p.off_w2b);
    a.w3b = (unsigned short*)(b + p.off_w3b);
    return a;
}

// Workspace: dF, dG, cell gradients, bad-cell flags, per-wavefront partial
// gradients, per-block loss partials.
struct LcWorkPlan {
    size_t off_dF, off_dG, off_g, off_bad, off_part, off_loss, total;
    int nparts, nloss;
};

LcNet lc_net_shape(const claw_lc_desc* d) {
    LcNet a;
    memset(&a, 0, sizeof a);
    a.nx = (int)d->nx;
    a.ny = (int)d->ny;
    a.ncell = a.nx * a.ny;
    a.tpr_x = (a.nx - 1 + 63) / 64;
    a.tpr_y = (a.nx + 63) / 64;
    a.ntiles_x = a.ny * a.tpr_x;
    a.ntiles = a.ntiles_x + (a.ny - 1) * a.tpr_y;
    a.nm.mu_h = d->mu_h;
    for (int c = 0; c < 3; ++c) {
        a.nm.sl[c] = d->sl[c];
        a.nm.sd1[c] = d->sd1[c];
        a.nm.sd2[c] = d->sd2[c];
        a.nm.sd3[c] = d->sd3[c];
        a.nm.s_out[c] = d->s_out[c];
    }
    return a;
}

LcWorkPlan lc_work_plan(const claw_lc_desc* d) {
    const LcNet a = lc_net_shape(d);
    const size_t nx = (size_t)d->nx, ny = (size_t)d->ny;
    LcWorkPlan w;
    w.nparts = lc_net_waves(a, 512);  // per direction
    w.nloss = lc_cell_blocks((int64_t)(nx * ny));
    w.off_dF = 0;
    w.off_dG = w.off_dF + lc_round(sizeof(float) * 3 * ny * (nx + 1));
    w.off_g = w.off_dG + lc_round(sizeof(float) * 3 * (ny + 1) * nx);
    w.off_bad = w.off_g + lc_round(sizeof(float) * 3 * ny * nx);
    w.off_part = w.off_bad + lc_round(ny * nx);
    w.off_loss = w.off_part + lc_round(sizeof(float) * 2 * (size_t)w.nparts * LC_NET);
    w.total = w.off_loss + lc_round(sizeof(double) * 4 * (size_t)w.nloss);
    return w;
}

claw_status lc_validate(const claw_lc_desc* d) {
    if (!d) return fail(CLAW_E_INVALID, "learned-correction descriptor is NULL");
    if (d->nx < 2 || d->ny < 2) return fail(CLAW_E_INVALID, "grid must be at least 2 x 2");
    if (d->nx >= ((int64_t)1 << 31) / 3 || d->ny >= ((int64_t)1 << 31) / 3 ||  // bounds the product below
        3 * d->nx * d->ny >= ((int64_t)1 << 31) || d->nx + 1 >= ((int64_t)1 << 31) / 3)
        return fail(CLAW_E_UNSUPPORTED, "grid too large for 32-bit offsets");
    for (int c = 0; c < 3; ++c)
        if (!(d->sl[c] > 0 && d->sd1[c] > 0 && d->sd2[c] > 0 && d->sd3[c] > 0) || !isfinite(d->sl[c]) ||
            !isfinite(d->sd1[c]) || !isfinite(d->sd2[c]) || !isfinite(d->sd3[c]))
            return fail(CLAW_E_INVALID, "input scales must be positive and finite");
    if (!isfinite(d->mu_h) || !isfinite(d->s_out[0]) || !isfinite(d->s_out[1]) || !isfinite(d->s_out[2]))
        return fail(CLAW_E_INVALID, "non-finite normalisation");
    return CLAW_OK;
}

LcNet lc_net(const claw_lc_desc* d, const void* params) {
    LcNet a = lc_net_shape(d);
    const LcParams p = lc_params(const_cast<void*>(params));
    a.theta = p.theta;
    a.w1b = p.w1b;
    a.w2b = p.w2b;
    a.w3b = p.w3b;
    return a;
}

LcApply lc_apply_args(const claw_lc_desc* d, const float* dF, const float* dG, void* work, double nux, double nuy,
                      double tau, double kappa) {
    const LcWorkPlan w = lc_work_plan(d);
    LcApply a;
    memset(&a, 0, sizeof a);
    a.dF = dF;
    a.dG = dG;
    a.bad = (unsigned char*)work + w.off_bad;
    a.nx = (int)d->nx;
    a.ny = (int)d->ny;
    a.ncell = a.nx * a.ny;
    a.nux = (float)nux;
    a.nuy = (float)nuy;
    a.tau = (float)tau;
    a.kappa = (float)kappa;
    for (int c = 0; c < 3; ++c) a.s_out[c] = d->s_out[c];
    return a;
}

}  // namespace

extern "C" {

claw_status claw_lc_sizes(const claw_lc_desc* d, size_t* param_bytes, size_t* work_bytes) {
    if (param_bytes) *param_bytes = lc_param_plan().total;
    if (work_bytes) {
        claw_status st = lc_validate(d);
        if (st) return st;
        *work_bytes = lc_work_plan(d).total;
    }
    return CLAW_OK;
}

claw_status claw_lc_init(void* params, void* stream) {
    if (!params) return fail(CLAW_E_INVALID, "params is NULL");
    HIP_TRY(launch_lc_init(lc_params(params), (hipStream_t)stream));
    return CLAW_OK;
}

claw_status claw_lc_forward(const claw_lc_desc* d, const void* params, const float* q, float* dF, float* dG,
                            void* stream) {
    claw_status st = lc_validate(d);
    if (st) return st;
    if (!params || !q || !dF || !dG) return fail(CLAW_E_INVALID, "NULL buffer");
    LcNet a = lc_net(d, params);
    a.q = q;
    a.dF = dF;
    a.dG = dG;
    HIP_TRY(launch_lc_forward(a, (hipStream_t)stream));
    return CLAW_OK;
}

claw_status claw_lc_loss_grad(const claw_lc_desc* d, const void* params, const float* q, const float* target,
                              const float* plain, double nux, double nuy, const double* w, void* work,
                              float* grad, double* loss, void* stream) {
    claw_status st = lc_validate(d);
    if (st) return st;
    if (!params || !q || !target || !plain || !w || !work || !grad) return fail(CLAW_E_INVALID, "NULL buffer");
    if (!(nux > 0) || !(nuy > 0)) return fail(CLAW_E_INVALID, "nu must be positive");
    const hipStream_t s = (hipStream_t)stream;
    const LcWorkPlan wp = lc_work_plan(d);
    char* ws = (char*)work;
    float* dF = (float*)(ws + wp.off_dF);
    float* dG = (float*)(ws + wp.off_dG);
    float* g = (float*)(ws + wp.off_g);
    LcNet a = lc_net(d, params);
    a.q = q;
    a.dF = dF;
    a.dG = dG;
    HIP_TRY(launch_lc_forward(a, s));
    LcCell c;
    memset(&c, 0, sizeof c);
    c.dF = dF;
    c.dG = dG;
    c.target = target;
    c.plain = plain;
    c.g = g;
    c.loss_part = (double*)(ws + wp.off_loss);
    c.nx = a.nx;
    c.ny = a.ny;
    c.ncell = a.ncell;
    c.nux = (float)nux;
    c.nuy = (float)nuy;
    const double n3 = 3.0 * (double)a.ncell;
    for (int f = 0; f < 3; ++f) {
        c.w[f] = (float)w[f];
        c.gscale[f] = (float)(2.0 * w[f] / n3);
    }
    HIP_TRY(launch_lc_cellgrad(c, s));
    a.g = g;
    a.nux = (float)nux;
    a.nuy = (float)nuy;
    a.partial = (float*)(ws + wp.off_part);
    HIP_TRY(launch_lc_backward(a, s));
    HIP_TRY(launch_lc_reduce(a.partial, wp.nparts, grad, c.loss_part, wp.nloss, 1.0 / n3, loss, s));
    return CLAW_OK;
}

claw_status claw_lc_adam(void* params, const float* grad, int64_t step, double lr, double beta1, double beta2,
                         double eps, void* stream) {
    if (!params || !grad) return fail(CLAW_E_INVALID, "NULL buffer");
    if (step < 1) return fail(CLAW_E_INVALID, "Adam steps count from 1");
    if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps >= 0))
        return fail(CLAW_E_INVALID, "bad Adam hyperparameters");
    const double c1 = 1.0 / (1.0 - pow(beta1, (double)step));
    const double c2 = 1.0 / (1.0 - pow(beta2, (double)step));
    HIP_TRY(launch_lc_adam(lc_params(params), grad, (float)lr, (float)beta1, (float)beta2, (float)eps, (float)c1,
                           (float)c2, (hipStream_t)stream));
    return CLAW_OK;
}

claw_status claw_lc_apply(const claw_lc_desc* d, const float* qn, const float* plain, const float* dF,
                          const float* dG, double nux, double nuy, double tau, double kappa, float* out,
                          uint8_t* keep_x, uint8_t* keep_y, void* work, void* stream) {
    claw_status st = lc_validate(d);
    if (st) return st;
    if (!qn || !plain || !dF || !dG || !out || !work) return fail(CLAW_E_INVALID, "NULL buffer");
    if (out != plain) {
        const size_t bytes = sizeof(float) * 3 * (size_t)d->nx * (size_t)d->ny;
        const char* o = (const char*)out;
        const char* p = (const char*)plain;
        const char* qq = (const char*)qn;
        if ((o < p + bytes && p < o + bytes) || (o < qq + bytes && qq < o + bytes))
            return fail(CLAW_E_INVALID, "out may alias plain only exactly");
    }
    LcApply a = lc_apply_args(d, dF, dG, work, nux, nuy, tau, kappa);
    a.qn = qn;
    a.plain = plain;
    a.out = out;
    a.keep_x = keep_x;
    a.keep_y = keep_y;
    HIP_TRY(launch_lc_apply(a, (hipStream_t)stream));
    return CLAW_OK;
}

claw_status claw_lc_coarsen(int64_t nx, int64_t ny, const float* fine, float* coarse, void* stream) {
    if (nx < 1 || ny < 1 || 12 * nx * ny >= ((int64_t)1 << 31)) return fail(CLAW_E_INVALID, "bad coarse grid");
    if (!fine || !coarse) return fail(CLAW_E_INVALID, "NULL buffer");
    HIP_TRY(launch_lc_coarsen(fine, coarse, (int)nx, (int)ny, (hipStream_t)stream));
    return CLAW_OK;
}

claw_status claw_lc_perturb(int64_t nx, int64_t ny, const float* q, float* out, const float* sigma, uint32_t seed,
                            uint32_t call, void* stream) {
    if (nx < 1 || ny < 1 || 3 * nx * ny >= ((int64_t)1 << 31)) return fail(CLAW_E_INVALID, "bad grid");
    if (!q || !out || !sigma) return fail(CLAW_E_INVALID, "NULL buffer");
    for (int f = 0; f < 3; ++f)
        if (!(sigma[f] >= 0.0f) || !isfinite(sigma[f])) return fail(CLAW_E_INVALID, "sigma[%d] invalid", f);
    HIP_TRY(launch_lc_perturb(q, out, (int)(nx * ny), sigma, seed, call, (hipStream_t)stream));
    return CLAW_OK;
}

claw_status claw_lc_scales(const double* r2, int64_t ncell, double nu, int32_t correct_depth, float* s_out,
                           double* w) {
    if (!r2 || !s_out || !w) return fail(CLAW_E_INVALID, "NULL argument");
    if (ncell < 1 || !(nu > 0)) return fail(CLAW_E_INVALID, "need ncell >= 1 and nu > 0");
    double rms[3];
    for (int f = 0; f < 3; ++f) {
        if (!(r2[f] >= 0)) return fail(CLAW_E_INVALID, "r2[%d] invalid", f);
        const double ms = r2[f] / (double)ncell;
        const double m = ms > 1e-30 ? ms : 1e-30;
        rms[f] = sqrt(m);
        w[f] = 1.0 / m;
    }
    const double mom = 0.5 * (rms[1] + rms[2]);
    s_out[0] = correct_depth ? (float)(rms[0] / nu) : 0.0f;
    s_out[1] = (float)(mom / nu);
    s_out[2] = (float)(mom / nu);
    return CLAW_OK;
}

claw_status claw_lc_advance(claw_solver* h, const claw_lc_desc* d, const void* params, int64_t nsteps, double dt,
                            double tau, double kappa, void* work) {
    if (!h) return fail(CLAW_E_INVALID, "solver is NULL");
    claw_status st = lc_validate(d);
    if (st) return st;
    if (!params || !work) return fail(CLAW_E_INVALID, "NULL buffer");
    if (!h->fp32 || h->d.riemann != CLAW_RP_SHALLOW_WATER || h->d.ndim != 2)
        return fail(CLAW_E_UNSUPPORTED, "the learned correction runs on FP32 2D shallow water");
    if (h->d.n[0] != d->nx || h->d.n[1] != d->ny) return fail(CLAW_E_INVALID, "grid differs from the solver's");
    for (int k = 0; k < 2; ++k)
        if (h->d.bc_lo[k] != CLAW_BC_WALL || h->d.bc_hi[k] != CLAW_BC_WALL)
            return fail(CLAW_E_UNSUPPORTED, "the learned correction assumes walls on all sides");
    if (nsteps < 0 || !(dt > 0) || !isfinite(dt)) return fail(CLAW_E_INVALID, "bad step count or dt");
    const LcWorkPlan wp = lc_work_plan(d);
    char* ws = (char*)work;
    LcNet a = lc_net(d, params);
    a.dF = (float*)(ws + wp.off_dF);
    a.dG = (float*)(ws + wp.off_dG);
    a.buf0 = (float*)h->buf[0];
    a.buf1 = (float*)h->buf[1];
    a.buf2 = (float*)h->buf[2];
    a.ctrl = h->ctrl;
    a.qsel = 0;  // Q^n is the trial's current buffer
    LcApply ap = lc_apply_args(d, a.dF, a.dG, work, dt / h->dx[0], dt / h->dx[1], tau, kappa);
    ap.buf0 = a.buf0;
    ap.buf1 = a.buf1;
    ap.buf2 = a.buf2;
    ap.ctrl = h->ctrl;
    ap.qsel = 0;
    ap.rsel = result_offset_of(h);  // the plain result, corrected in place
    // the forward pass applies the indicator test itself (zero on the faces
    // that fail it), so the application reads no depths for it
    a.mask = 1;
    a.tau = ap.tau;
    a.kappa = ap.kappa;
    ap.premasked = 1;
    // One learned step: the plain fixed-dt trial, then the corrections from
    // Q^n applied to its result before the next trial's first sweep accepts it.
    auto enqueue_step = [&](hipStream_t s) -> claw_status {
        const int cq = h->parity;
        claw_status r = enqueue_trial(h, s, nullptr);
        if (r) return r;
        a.cq = cq;
        ap.cq = cq;
        HIP_TRY(launch_lc_forward(a, s));
        HIP_TRY(launch_lc_apply(ap, s));
        return CLAW_OK;
    };
    st = commit(h);
    if (st) return st;
    HIP_TRY(launch_begin(h->ctrl, committed(h), dt, MODE_FIXED, result_offset_of(h), h->stream));
    constexpr int G = 16;  // learned steps per captured graph (even: parity returns)
    int64_t done = 0;
    if (nsteps >= G) {
        struct Key {
            const void* params;
            void* work;
            claw_lc_desc d;
            float tau, kappa, nux, nuy;
            int parity;
        } key;
        static_assert(sizeof(Key) <= sizeof(h->lc_key), "graph key too large");
        memset(&key, 0, sizeof key);
        key.params = params;
        key.work = work;
        key.d = *d;
        key.tau = ap.tau;
        key.kappa = ap.kappa;
        key.nux = ap.nux;
        key.nuy = ap.nuy;
        key.parity = h->parity;
        if (!h->lc_exec || memcmp(h->lc_key, &key, sizeof key) != 0) {
            if (h->lc_exec) (void)hipGraphExecDestroy(h->lc_exec);
            if (h->lc_graph) (void)hipGraphDestroy(h->lc_graph);
            h->lc_exec = nullptr;
            h->lc_graph = nullptr;
            HIP_TRY(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
            const int p0 = h->parity;
            claw_status cs = CLAW_OK;
            for (int k = 0; k < G && cs == CLAW_OK; ++k) cs = enqueue_step(h->cap_stream);
            h->parity = p0;
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(h->cap_stream, &g);
            if (cs) {
                if (g) (void)hipGraphDestroy(g);
                return cs;
            }
            if (e != hipSuccess) return fail(CLAW_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&h->lc_exec, g, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                (void)hipGraphDestroy(g);
                h->lc_exec = nullptr;
                return fail(CLAW_E_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
            }
            h->lc_graph = g;
            memset(h->lc_key, 0, sizeof h->lc_key);
            memcpy(h->lc_key, &key, sizeof key);
        }
        for (; done + G <= nsteps; done += G) HIP_TRY(hipGraphLaunch(h->lc_exec, h->stream));
    }
    for (; done < nsteps; ++done) {
        st = enqueue_step(h->stream);
        if (st) return st;
    }
    st = commit(h);
    if (!st) st = sync_state(h);
    if (st) return st;
    Ctrl c;
    st = read_ctrl(h, &c);
    if (st) return st;
    return ctrl_status(c.st[committed(h)]);
}

}  // extern "C"
