// claw_launch.h -- host-side launch entry points of the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "claw_device.h"

namespace claw {

// One directional sweep of system sys with meqn fields; a.dir selects the
// row (0) or column (1, 2) kernel.  kind: 0 sweep, 1 speed-only pass, 2 sweep
// that closes a step (its last workgroup runs the step control with
// a.ctrl_mode and a.result_off).
template <typename R>
hipError_t launch_sweep(const SweepArgs<R>& a, int sys, int meqn, int kind, hipStream_t s);

// Step-control kernels (one thread; see control.hip).
hipError_t launch_begin(Ctrl* c, double dt, hipStream_t s);
hipError_t launch_begin_speeds(Ctrl* c, hipStream_t s);
hipError_t launch_init_dt(Ctrl* c, bool fp32, hipStream_t s);
hipError_t launch_set_target(Ctrl* c, long long nsteps, hipStream_t s);
hipError_t launch_control(Ctrl* c, int result_off, int mode, bool fp32, hipStream_t s);
hipError_t launch_accept_sweep(Ctrl* c, int result_off, hipStream_t s);
hipError_t launch_set_control(Ctrl* c, double t, double dt_next, hipStream_t s);
hipError_t launch_ctrl_init(Ctrl* c, const double* dx, int ndim, double cfl_desired,
                            double cfl_max, double dt_max, hipStream_t s);

// Element-wise set-up kernels.
template <typename R>
hipError_t launch_derive_zc(const R* aux, R* zc, int64_t ncell, hipStream_t s);
template <typename R>
hipError_t launch_sync_state(Ctrl* c, R* b0, R* b1, R* b2, int64_t n, hipStream_t s);

}  // namespace claw
