// claw_launch.h -- host-side launch entry points of the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "claw_device.h"

namespace claw {

// One directional sweep (or, with speeds, its speed-only pass) of system sys
// with meqn fields; a.dir selects the row (0) or column (1, 2) kernel.
template <typename R>
hipError_t launch_sweep(const SweepArgs<R>& a, int sys, int meqn, bool speeds, hipStream_t s);

// One-thread step-control kernels on step-state copy q (see control.hip).
hipError_t launch_ctrl_init(Ctrl* c, const double* dx, int ndim, double cfl_desired,
                            double cfl_max, double dt_max, hipStream_t s);
hipError_t launch_commit(Ctrl* c, int q, bool fp32, hipStream_t s);
hipError_t launch_begin(Ctrl* c, int q, double dt, int mode, int result_off, hipStream_t s);
hipError_t launch_zero_speeds(Ctrl* c, int q, hipStream_t s);
hipError_t launch_init_dt(Ctrl* c, int q, bool fp32, int mode, int result_off, hipStream_t s);
hipError_t launch_set_target(Ctrl* c, int q, long long nsteps, hipStream_t s);
hipError_t launch_set_control(Ctrl* c, int q, double t, double dt_next, hipStream_t s);

// Batched ensemble launches (batch.hip): blocks[i] maps workgroup i of a
// launch to an instance and its logical block; args holds two SweepArgs per
// instance (x, y).
struct BatchBlock {
    int inst, x, y, z;
};
template <typename R>
struct BatchLaunch {
    const BatchBlock* blocks;
    const SweepArgs<R>* args;
    int parity, first, last, pad;
};
enum { BOP_COMMIT = 0, BOP_ZERO_SPEEDS = 1, BOP_BEGIN_FIXED = 2, BOP_BEGIN_ADAPT = 3 };
template <typename R>
hipError_t launch_batch_sweep(const BatchLaunch<R>& L, int sys, int dir, int nblocks, bool speeds,
                              hipStream_t s);
hipError_t launch_batch_ctrl(Ctrl* const* ctrls, int count, int op, int q, double dt, int mode,
                             int result_off, long long nsteps, bool fp32, hipStream_t s);

// Element-wise set-up kernels.
template <typename R>
hipError_t launch_derive_zc(const R* aux, R* zc, int64_t ncell, hipStream_t s);
template <typename R>
hipError_t launch_sync_state(Ctrl* c, int q, R* b0, R* b1, R* b2, int64_t n, hipStream_t s);

}  // namespace claw
