// control.hip -- one-thread kernels that set up and close the step state of
// the device control block (trial step, first step from a speed pass, step
// target, committing the last trial's decision) and the small element-wise
// set-up kernels (derived acoustic coefficients, copy of the state back into
// q).  The per-step CFL decision itself (section 4.1) is decide(), evaluated by
// the sweep that opens the next trial.
//
// All step-control scalars stay in the device control block, so a captured
// graph of many steps runs without any host round trip.
#include <math.h>

#include "claw_launch.h"

namespace claw {

__global__ void k_ctrl_init(Ctrl* c, double dx0, double dx1, double dx2, int ndim, double cfl_desired,
                            double cfl_max, double dt_max, int strang, int result_off) {
    for (int q = 0; q < 2; ++q) {
        StepState& s = c->st[q];
        s.t = s.dt = s.dt_next = s.cfl = 0.0;
        for (int d = 0; d < 3; ++d) {
            s.dtdx[d] = 0.0;
            s.dtdx_f[d] = 0.0f;
        }
        s.cur = s.done = s.err = s.last_accepted = s.pending = s.mode = s.pad = 0;
        s.result_off = result_off;
        s.accepted = s.rejected = s.target = s.consecutive = s.trials = 0;
        s.base_accepted = s.base_rejected = 0;
        clear_speeds(c, q);
        c->nonphys[q] = 0;
    }
    c->ndim = ndim;
    c->dx[0] = dx0;
    c->dx[1] = dx1;
    c->dx[2] = dx2;
    c->inv_dx[0] = 1.0 / dx0;
    c->inv_dx[1] = 1.0 / dx1;
    c->inv_dx[2] = 1.0 / dx2;
    for (int d = 0; d < 3; ++d) c->sweep_frac[d] = (strang && d < ndim - 1) ? 0.5 : 1.0;
    c->cfl_desired = cfl_desired;
    c->cfl_max = cfl_max;
    c->dt_max = dt_max;
}

// Applies a pending decision to copy q and clears the speed slots of the
// other parity (those the next trial will fill).
__global__ void k_commit(Ctrl* c, int q, int fp32) {
    StepState N;
    decide(c, q, fp32 != 0, N);
    c->st[q] = N;
    const int o = q ^ 1;
    clear_speeds(c, o);
    c->nonphys[o] = 0;
}

__global__ void k_begin(Ctrl* c, int q, double dt, int mode, int result_off) {
    StepState& s = c->st[q];
    set_trial_dt(c, s, dt);
    s.mode = mode;
    s.result_off = result_off;
    s.done = 0;
    s.err = 0;
    s.pending = 0;
}

__global__ void k_zero_speeds(Ctrl* c, int q) {
    clear_speeds(c, q);
    c->nonphys[q] = 0;
}

// First trial step from the speed-only pass that filled slot q; with
// use_next, the next step a previous run left (dt_next > 0) if there is one
// (the speed pass then skipped its work).
__global__ void k_init_dt(Ctrl* c, int q, int fp32, int mode, int result_off, int use_next) {
    StepState& s = c->st[q];
    s.mode = mode;
    s.result_off = result_off;
    s.pending = 0;
    s.done = 0;
    s.err = 0;
    if (use_next && s.dt_next > 0.0) {
        set_trial_dt(c, s, s.dt_next);
        return;
    }
    if (c->nonphys[q]) {
        s.err = 5;
        s.done = 1;
        return;
    }
    double dt = 0.0;
    if (!next_dt(c, sigma_of(c, q, fp32 != 0), &dt)) {
        s.err = 6;
        s.done = 1;
        return;
    }
    set_trial_dt(c, s, dt);
}

__global__ void k_set_target(Ctrl* c, int q, long long nsteps) {
    StepState& s = c->st[q];
    s.target = s.accepted + nsteps;
    s.base_accepted = s.accepted;
    s.base_rejected = s.rejected;
    s.done = nsteps <= 0 ? 1 : 0;
    s.consecutive = 0;
}

__global__ void k_set_control(Ctrl* c, int q, double t, double dt_next) {
    c->st[q].t = t;
    c->st[q].dt_next = dt_next;
}

template <typename R>
__global__ void k_derive_zc(const R* __restrict__ aux, R* __restrict__ zc, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    R rho = aux[i];
    R K = aux[n + i];
    // impedance and sound speed, correctly rounded in both precisions
    zc[i] = sqrt(rho * K);
    zc[n + i] = sqrt(K / rho);
}

// Copies the current buffer of copy q into buf[0] (the caller's q) when it is elsewhere.
template <typename R>
__global__ void k_sync_state(const Ctrl* c, int q, R* b0, const R* b1, const R* b2, int64_t n) {
    const int cur = c->st[q].cur;
    if (cur == 0) return;
    const R* src = cur == 1 ? b1 : b2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b0[i] = src[i];
}

__global__ void k_reset_cur(Ctrl* c, int q) { c->st[q].cur = 0; }

// Largest |s| of direction dir recorded in copy q, or a NaN when a sweep of
// that copy met a non-physical state.
__global__ void k_report_smax(const Ctrl* c, int q, int dir, int fp32, double* out) {
    if (c->nonphys[q]) {
        *out = __builtin_nan("");
        return;
    }
    *out = fp32 ? (double)__uint_as_float(smax32_of(c, q, dir))
                : __longlong_as_double((long long)smax64_of(c, q, dir));
}

hipError_t launch_ctrl_init(Ctrl* c, const double* dx, int ndim, double cfl_desired, double cfl_max,
                            double dt_max, bool strang, int result_off, hipStream_t s) {
    hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(1), 0, s, c, dx[0], dx[1], dx[2], ndim, cfl_desired,
                       cfl_max, dt_max, strang ? 1 : 0, result_off);
    return hipGetLastError();
}
hipError_t launch_commit(Ctrl* c, int q, bool fp32, hipStream_t s) {
    hipLaunchKernelGGL(k_commit, dim3(1), dim3(1), 0, s, c, q, fp32 ? 1 : 0);
    return hipGetLastError();
}
hipError_t launch_begin(Ctrl* c, int q, double dt, int mode, int result_off, hipStream_t s) {
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(1), 0, s, c, q, dt, mode, result_off);
    return hipGetLastError();
}
hipError_t launch_zero_speeds(Ctrl* c, int q, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_speeds, dim3(1), dim3(1), 0, s, c, q);
    return hipGetLastError();
}
hipError_t launch_init_dt(Ctrl* c, int q, bool fp32, int mode, int result_off, bool use_next, hipStream_t s) {
    hipLaunchKernelGGL(k_init_dt, dim3(1), dim3(1), 0, s, c, q, fp32 ? 1 : 0, mode, result_off,
                       use_next ? 1 : 0);
    return hipGetLastError();
}
hipError_t launch_set_target(Ctrl* c, int q, long long nsteps, hipStream_t s) {
    hipLaunchKernelGGL(k_set_target, dim3(1), dim3(1), 0, s, c, q, nsteps);
    return hipGetLastError();
}
hipError_t launch_set_control(Ctrl* c, int q, double t, double dt_next, hipStream_t s) {
    hipLaunchKernelGGL(k_set_control, dim3(1), dim3(1), 0, s, c, q, t, dt_next);
    return hipGetLastError();
}

hipError_t launch_report_smax(const Ctrl* c, int q, int dir, bool fp32, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_report_smax, dim3(1), dim3(1), 0, s, c, q, dir, fp32 ? 1 : 0, out);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_derive_zc(const R* aux, R* zc, int64_t ncell, hipStream_t s) {
    if (ncell <= 0) return hipSuccess;
    const int64_t blocks = (ncell + 255) / 256;
    hipLaunchKernelGGL((k_derive_zc<R>), dim3((unsigned)blocks), dim3(256), 0, s, aux, zc, ncell);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_sync_state(Ctrl* c, int q, R* b0, R* b1, R* b2, int64_t n, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((k_sync_state<R>), dim3((unsigned)blocks), dim3(256), 0, s, c, q, b0, b1, b2, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reset_cur, dim3(1), dim3(1), 0, s, c, q);
    return hipGetLastError();
}

template hipError_t launch_derive_zc<float>(const float*, float*, int64_t, hipStream_t);
template hipError_t launch_derive_zc<double>(const double*, double*, int64_t, hipStream_t);
template hipError_t launch_sync_state<float>(Ctrl*, int, float*, float*, float*, int64_t, hipStream_t);
template hipError_t launch_sync_state<double>(Ctrl*, int, double*, double*, double*, int64_t, hipStream_t);

}  // namespace claw
