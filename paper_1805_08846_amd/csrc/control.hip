// control.hip -- one-thread kernels that set up the device control block
// (trial step, first step from a speed pass, step target) and the small
// element-wise set-up kernels (derived acoustic coefficients, copy of the
// state back into q).  The per-step CFL decision itself (section 4.1) runs
// in the last workgroup of the sweep that closes a step (control_step).
//
// All step-control scalars stay in the device control block, so a captured
// graph of many steps runs without any host round trip.
#include <math.h>

#include "claw_launch.h"

namespace claw {

__global__ void k_ctrl_init(Ctrl* c, double dx0, double dx1, double dx2, int ndim, double cfl_desired,
                            double cfl_max, double dt_max) {
    c->t = 0.0;
    c->dt = 0.0;
    c->dt_next = 0.0;
    c->cfl = 0.0;
    c->dx[0] = dx0;
    c->dx[1] = dx1;
    c->dx[2] = dx2;
    c->ndim = ndim;
    c->cfl_desired = cfl_desired;
    c->cfl_max = cfl_max;
    c->dt_max = dt_max;
    c->mode = 0;
    c->cur = 0;
    c->done = 0;
    c->err = 0;
    c->last_accepted = 0;
    c->accepted = 0;
    c->rejected = 0;
    c->target = 0;
    c->consecutive = 0;
    c->trials = 0;
    c->blocks_done = 0u;
    set_trial_dt(c, 0.0);
}

__global__ void k_begin(Ctrl* c, double dt) {
    set_trial_dt(c, dt);
    c->done = 0;
    c->err = 0;
}

__global__ void k_begin_speeds(Ctrl* c) {
    set_trial_dt(c, c->dt);
    c->done = 0;
    c->err = 0;
}

// First trial step from the speed-only pass that ran just before.
__global__ void k_init_dt(Ctrl* c, int fp32) {
    double dt = 0.0;
    if (c->nonphys) {
        c->err = 5;
        c->done = 1;
        return;
    }
    if (!next_dt(c, sigma_of(c, fp32 != 0), &dt)) {
        c->err = 6;
        c->done = 1;
        return;
    }
    set_trial_dt(c, dt);
}

__global__ void k_set_target(Ctrl* c, long long nsteps) {
    c->target = c->accepted + nsteps;
    c->done = nsteps <= 0 ? 1 : 0;
    c->consecutive = 0;
    c->err = 0;
}

// Step control as its own one-thread kernel (used when the control is not
// fused into the last sweep).
__global__ void k_control(Ctrl* c, int result_off, int mode, int fp32) {
    control_step(c, result_off, mode, fp32 != 0, false);
}

__global__ void k_accept_sweep(Ctrl* c, int result_off) {
    if (c->done) return;
    c->cur = (c->cur + result_off) % 3;
}

__global__ void k_set_control(Ctrl* c, double t, double dt_next) {
    c->t = t;
    c->dt_next = dt_next;
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

// Copies the current buffer into buf[0] (the caller's q) when it is elsewhere.
template <typename R>
__global__ void k_sync_state(const Ctrl* c, R* b0, const R* b1, const R* b2, int64_t n) {
    const int cur = c->cur;
    if (cur == 0) return;
    const R* src = cur == 1 ? b1 : b2;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        b0[i] = src[i];
}

__global__ void k_reset_cur(Ctrl* c) { c->cur = 0; }

hipError_t launch_ctrl_init(Ctrl* c, const double* dx, int ndim, double cfl_desired, double cfl_max,
                            double dt_max, hipStream_t s) {
    hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(1), 0, s, c, dx[0], dx[1], dx[2], ndim, cfl_desired,
                       cfl_max, dt_max);
    return hipGetLastError();
}
hipError_t launch_begin(Ctrl* c, double dt, hipStream_t s) {
    hipLaunchKernelGGL(k_begin, dim3(1), dim3(1), 0, s, c, dt);
    return hipGetLastError();
}
hipError_t launch_begin_speeds(Ctrl* c, hipStream_t s) {
    hipLaunchKernelGGL(k_begin_speeds, dim3(1), dim3(1), 0, s, c);
    return hipGetLastError();
}
hipError_t launch_init_dt(Ctrl* c, bool fp32, hipStream_t s) {
    hipLaunchKernelGGL(k_init_dt, dim3(1), dim3(1), 0, s, c, fp32 ? 1 : 0);
    return hipGetLastError();
}
hipError_t launch_set_target(Ctrl* c, long long nsteps, hipStream_t s) {
    hipLaunchKernelGGL(k_set_target, dim3(1), dim3(1), 0, s, c, nsteps);
    return hipGetLastError();
}
hipError_t launch_control(Ctrl* c, int result_off, int mode, bool fp32, hipStream_t s) {
    hipLaunchKernelGGL(k_control, dim3(1), dim3(1), 0, s, c, result_off, mode, fp32 ? 1 : 0);
    return hipGetLastError();
}
hipError_t launch_accept_sweep(Ctrl* c, int result_off, hipStream_t s) {
    hipLaunchKernelGGL(k_accept_sweep, dim3(1), dim3(1), 0, s, c, result_off);
    return hipGetLastError();
}
hipError_t launch_set_control(Ctrl* c, double t, double dt_next, hipStream_t s) {
    hipLaunchKernelGGL(k_set_control, dim3(1), dim3(1), 0, s, c, t, dt_next);
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
hipError_t launch_sync_state(Ctrl* c, R* b0, R* b1, R* b2, int64_t n, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL((k_sync_state<R>), dim3((unsigned)blocks), dim3(256), 0, s, c, b0, b1, b2, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reset_cur, dim3(1), dim3(1), 0, s, c);
    return hipGetLastError();
}

template hipError_t launch_derive_zc<float>(const float*, float*, int64_t, hipStream_t);
template hipError_t launch_derive_zc<double>(const double*, double*, int64_t, hipStream_t);
template hipError_t launch_sync_state<float>(Ctrl*, float*, float*, float*, int64_t, hipStream_t);
template hipError_t launch_sync_state<double>(Ctrl*, double*, double*, double*, int64_t, hipStream_t);

}  // namespace claw
