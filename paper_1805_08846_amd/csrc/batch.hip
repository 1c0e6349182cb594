// batch.hip -- ensemble kernels: one launch sweeps every instance of a batch
// of independent grids of different sizes.  A device table maps each
// workgroup of the launch to (instance, logical block); the workgroup then
// runs the same sweep body as the single-grid kernels with that instance's
// arguments, so every instance's result is bitwise the single-grid result.
// The order of the table (largest instances first, or round-robin) is the
// schedule the autotuner picks.
#include "claw_launch.h"
#include "sweep_body.h"

namespace claw {

template <typename R, int SYS, int MEQN, int CPL, bool SPEEDS, int LIMK, int RPW>
__global__ __launch_bounds__(256) void k_batch_row(BatchLaunch<R> L) {
    const BatchBlock bb = L.blocks[blockIdx.x];
    SweepArgs<R> a = L.args[bb.inst * 2 + 0];
    if (SPEEDS) a.src_off = 0;  // a speed pass reads the current state in every direction
    a.parity = L.parity;
    a.first = L.first;
    a.last = L.last;
    row_body<R, SYS, MEQN, CPL, SPEEDS, LIMK, RPW>(a, bb.x, bb.y, bb.x == 0 && bb.y == 0);
}

template <typename R, int SYS, int MEQN, int NRM, int PF, bool SPEEDS, int LIMK>
__global__ __launch_bounds__(256) void k_batch_col(BatchLaunch<R> L) {
    const BatchBlock bb = L.blocks[blockIdx.x];
    SweepArgs<R> a = L.args[bb.inst * 2 + 1];
    if (SPEEDS) a.src_off = 0;
    a.parity = L.parity;
    a.first = L.first;
    a.last = L.last;
    col_body<R, SYS, MEQN, NRM, PF, SPEEDS, LIMK>(a, bb.x, bb.y, bb.z, bb.x == 0 && bb.y == 0 && bb.z == 0);
}

// One thread per instance: step-state operations on copy q of every control block.
__global__ void k_batch_ctrl(Ctrl* const* ctrls, int count, int op, int q, double dt, int mode,
                             int result_off, long long nsteps, int fp32) {
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= count) return;
    Ctrl* c = ctrls[i];
    StepState& s = c->st[q];
    switch (op) {
        case BOP_COMMIT: {
            StepState N;
            decide(c, q, fp32 != 0, N);
            c->st[q] = N;
            const int o = q ^ 1;
            clear_speeds(c, o);
            c->nonphys[o] = 0;
            break;
        }
        case BOP_ZERO_SPEEDS:
            clear_speeds(c, q);
            c->nonphys[q] = 0;
            break;
        case BOP_OPEN: {  // a fused trial of parity q opens: decide copy q ^ 1 into copy q
            StepState N;
            decide(c, q ^ 1, fp32 != 0, N);
            N.pending = N.done ? 0 : 1;
            if (N.mode == MODE_ADAPT && !N.done) N.result_off = planned_result_off(N.cur, N.target - N.accepted);
            c->st[q] = N;
            clear_speeds(c, q);
            c->nonphys[q] = 0;
            break;
        }
        case BOP_BEGIN_FIXED:  // trial step dt in mode `mode`
            set_trial_dt(c, s, dt);
            s.mode = mode;
            s.result_off = result_off;
            s.done = 0;
            s.err = 0;
            s.pending = 0;
            break;
        case BOP_BEGIN_ADAPT: {  // dt_next of a previous run, else from the speed pass in slot q
            s.mode = MODE_ADAPT;
            s.result_off = result_off;
            s.done = 0;
            s.err = 0;
            s.pending = 0;
            double d = s.dt_next;
            if (!(d > 0)) {
                if (c->nonphys[q]) {
                    s.err = 5;
                    s.done = 1;
                    break;
                }
                if (!next_dt(c, sigma_of(c, q, fp32 != 0), &d)) {
                    s.err = 6;
                    s.done = 1;
                    break;
                }
            }
            set_trial_dt(c, s, d);
            s.target = s.accepted + nsteps;
            s.consecutive = 0;
            s.done = nsteps <= 0 ? 1 : 0;
            break;
        }
    }
}

template <typename R, int SYS, int MEQN, bool SPEEDS, int LIMK>
static hipError_t launch_batch_kind(const BatchLaunch<R>& L, int dir, int nblocks, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    if (dir == 0) {
        constexpr int CPL = sizeof(R) == 4 ? 4 : 2;
        if (L.rpw == 2)
            hipLaunchKernelGGL((k_batch_row<R, SYS, MEQN, CPL, SPEEDS, LIMK, 2>), dim3(nblocks), dim3(256), 0, s, L);
        else if (L.rpw == 4)
            hipLaunchKernelGGL((k_batch_row<R, SYS, MEQN, CPL, SPEEDS, LIMK, 4>), dim3(nblocks), dim3(256), 0, s, L);
        else if (L.rpw == 8)
            hipLaunchKernelGGL((k_batch_row<R, SYS, MEQN, CPL, SPEEDS, LIMK, 8>), dim3(nblocks), dim3(256), 0, s, L);
        else
            return hipErrorInvalidValue;
    } else {
        hipLaunchKernelGGL((k_batch_col<R, SYS, MEQN, 2, 4, SPEEDS, LIMK>), dim3(nblocks), dim3(256), 0, s, L);
    }
    return hipGetLastError();
}

// MC across the whole batch runs the kernels specialised for it.
template <typename R>
hipError_t launch_batch_sweep(const BatchLaunch<R>& L, int sys, int dir, int nblocks, bool speeds,
                              hipStream_t s) {
    if (sys != SYS_SW) return hipErrorInvalidValue;
    if (speeds) return launch_batch_kind<R, SYS_SW, 3, true, LIM_RUNTIME>(L, dir, nblocks, s);
    if (L.limiter == LIM_MC) return launch_batch_kind<R, SYS_SW, 3, false, LIM_MC>(L, dir, nblocks, s);
    return launch_batch_kind<R, SYS_SW, 3, false, LIM_RUNTIME>(L, dir, nblocks, s);
}

hipError_t launch_batch_ctrl(Ctrl* const* ctrls, int count, int op, int q, double dt, int mode,
                             int result_off, long long nsteps, bool fp32, hipStream_t s) {
    hipLaunchKernelGGL(k_batch_ctrl, dim3((count + 63) / 64), dim3(64), 0, s, ctrls, count, op, q, dt, mode,
                       result_off, nsteps, fp32 ? 1 : 0);
    return hipGetLastError();
}

template hipError_t launch_batch_sweep<float>(const BatchLaunch<float>&, int, int, int, bool, hipStream_t);
template hipError_t launch_batch_sweep<double>(const BatchLaunch<double>&, int, int, int, bool, hipStream_t);

}  // namespace claw
