// claw_launch.h -- host-side launch entry points of the device kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "claw_device.h"

namespace claw {

// Rows each row-sweep wavefront takes in turn: single grids (FP64 lanes hold
// two cells, so a wavefront's fixed work is spread over two rows); batched
// launches take 2, 4 or 8 (a batched workgroup first loads its table entry and
// its instance's arguments, so it pays for more rows), chosen by the tuner.
template <typename R>
constexpr int row_rpw_single() { return sizeof(R) == 4 ? 1 : 2; }
constexpr int ROW_RPW_BATCH_DEFAULT = 8;
inline bool batch_rpw_ok(int rpw) { return rpw == 2 || rpw == 4 || rpw == 8; }

// One directional sweep (or, with speeds, its speed-only pass) of system sys
// with meqn fields; a.dir selects the row (0) or column (1, 2) kernel.
template <typename R>
hipError_t launch_sweep(const SweepArgs<R>& a, int sys, int meqn, bool speeds, hipStream_t s);

// Fused 2D shallow-water step (fused.hip): each workgroup marches a strip of
// columns down a chunk of rows, x-sweeping rows into LDS and y-sweeping them
// out.  a: the x-sweep arguments (grid, buffers, control, x boundaries,
// parity, limiter); ny and the y boundaries complete the grid; chunk: rows
// per workgroup.
template <typename R>
struct FusedArgs {
    SweepArgs<R> a;
    int32_t ny, bcy_lo, bcy_hi, chunk;
};
template <typename R>
hipError_t launch_step2d(const FusedArgs<R>& F, hipStream_t s);
// The x and y sweeps of a 3D acoustics step fused (fused.hip), for rows of
// exactly 64 CPL cells (256 FP32, 128 FP64) with extrapolation at both x ends;
// the z sweep follows as a column sweep.  a: the x-sweep arguments; ny, nz
// and the y boundaries complete the grid; chunk: rows of one z plane per
// workgroup.  The result goes to buffer cur + 1, as the 2D step's does.  The
// kernel opens the trial (it decides the previous one, as a first sweep does).
template <typename R>
struct Fused3Args {
    SweepArgs<R> a;
    int32_t ny, nz, bcy_lo, bcy_hi, chunk;
};
template <typename R>
hipError_t launch_step_xy3(const Fused3Args<R>& F, int sys, hipStream_t s);
// Result buffer of a trial that one kernel runs (the fused 2D step), chosen
// when the trial opens: with r accepted steps to go in an adaptive run (r
// counts this trial), the last one writes buffer 0, the caller's array, so
// the run ends with no copy.  Two steps before the end the result goes to the
// buffer that is neither the current one nor 0; earlier ones rotate.  A
// result is never written over the trial's own input (a rejected trial keeps
// it).  Returns the offset from the current buffer (1 or 2).
__device__ __forceinline__ int planned_result_off(int cur, long long r) {
    int dst;
    if (r == 1) dst = cur != 0 ? 0 : 1;  // one step from buffer 0 cannot end in it
    else if (r == 2) dst = cur != 0 ? 3 - cur : 1;
    else dst = (cur + 1) % 3;
    return (dst - cur + 3) % 3;
}
// Decides the previous trial into step-state copy p and clears p's speed slots.
hipError_t launch_open(Ctrl* c, int p, bool fp32, hipStream_t s);
int fused_rows_per_iteration();

// One-thread step-control kernels on step-state copy q (see control.hip).
hipError_t launch_ctrl_init(Ctrl* c, const double* dx, int ndim, double cfl_desired,
                            double cfl_max, double dt_max, bool strang, int result_off, hipStream_t s);
hipError_t launch_commit(Ctrl* c, int q, bool fp32, hipStream_t s);
hipError_t launch_begin(Ctrl* c, int q, double dt, int mode, int result_off, hipStream_t s);
hipError_t launch_zero_speeds(Ctrl* c, int q, hipStream_t s);
hipError_t launch_init_dt(Ctrl* c, int q, bool fp32, int mode, int result_off, bool use_next, hipStream_t s);
hipError_t launch_set_target(Ctrl* c, int q, long long nsteps, hipStream_t s);
hipError_t launch_set_control(Ctrl* c, int q, double t, double dt_next, hipStream_t s);
// *out = max |s| of direction dir in copy q (NaN if the copy met a non-physical state).
hipError_t launch_report_smax(const Ctrl* c, int q, int dir, bool fp32, double* out, hipStream_t s);

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
    int parity, first, last;
    int limiter;  // the limiter every instance uses, or -1 if they differ
    int rpw;      // rows per row-sweep wavefront (2, 4 or 8; the row table is built for it)
};
// Batched fused 2D steps (fused.hip): blocks[i] maps workgroup i to an
// instance, a strip of columns (x) and a chunk of rows (y); args holds each
// instance's fused-step arguments.
template <typename R>
struct BatchFusedLaunch {
    const BatchBlock* blocks;
    const FusedArgs<R>* args;
    int parity;
    int limiter;  // the limiter every instance uses, or -1 if they differ
};
template <typename R>
hipError_t launch_batch_step2d(const BatchFusedLaunch<R>& L, int nblocks, hipStream_t s);
// BOP_OPEN: decide the previous trial into copy q and clear copy q's speed
// slots (what the single-grid fused step's opening kernel does).
enum { BOP_COMMIT = 0, BOP_ZERO_SPEEDS = 1, BOP_BEGIN_FIXED = 2, BOP_BEGIN_ADAPT = 3, BOP_OPEN = 4 };
template <typename R>
hipError_t launch_batch_sweep(const BatchLaunch<R>& L, int sys, int dir, int nblocks, bool speeds,
                              hipStream_t s);
hipError_t launch_batch_ctrl(Ctrl* const* ctrls, int count, int op, int q, double dt, int mode,
                             int result_off, long long nsteps, bool fp32, hipStream_t s);

// Learned coarse correction (learned.hip).  Two 12-64-64-3 networks, one
// per sweep direction (x faces, then y faces), each flat: W1 (64, 12), b1,
// W2 (64, 64), b2, W3 (3, 64), b3.  BF16 copies per network, each in the
// order its matrix-core operand takes (learned.hip: w1_slot, w2_slot,
// w3_slot): W1 with its 12 features padded to 16, W2, W3 with its 3 outputs
// padded to 16 rows.
enum {
    LC_NET = 5187,
    LC_NPARAM = 2 * LC_NET,
    LC_W1B = 64 * 16,
    LC_W2B = 64 * 64,
    LC_W3B = 16 * 64,
    LC_OFF_W1 = 0,
    LC_OFF_B1 = 768,
    LC_OFF_W2 = 832,
    LC_OFF_B2 = 4928,
    LC_OFF_W3 = 4992,
    LC_OFF_B3 = 5184
};
struct LcNorm {
    float mu_h;
    float sl[3], sd1[3], sd2[3], sd3[3], s_out[3];
};
// Network pass over the interior faces of a (ny, nx) grid (launch
// dimension y = sweep direction of the faces and of the network).  With ctrl set,
// the state is rotation buffer (cur + qsel) % 3 of step-state copy cq (the
// copy of a trial that ran and is not decided yet), and the pass does nothing
// if that trial failed, was skipped or flagged a non-physical state.
struct LcNet {
    const float* q;
    const Ctrl* ctrl;
    int cq, qsel;
    float *buf0, *buf1, *buf2;
    int nx, ny, ncell;
    int ntiles_x, tpr_x, tpr_y, ntiles;
    LcNorm nm;
    const float* theta;                     // both networks' FP32 masters
    const unsigned short *w1b, *w2b, *w3b;  // BF16 copies, two networks each
    float *dF, *dG;
    const float* g;  // training: cell gradients (3, ny, nx)
    float nux, nuy;
    float* partial;  // training: [direction][wave][LC_NET]
    // mask != 0: the forward pass writes zero on faces that fail the
    // fallback's indicator test (tau, kappa as in LcApply), for an
    // application that then skips that test (LcApply::premasked)
    int mask;
    float tau, kappa;
};
struct LcCell {
    const float *dF, *dG, *target, *plain;
    float* g;
    double* loss_part;
    int nx, ny, ncell;
    float nux, nuy;
    float w[3], gscale[3];
};
// Fallback and application; with ctrl set, qn / plain / out are resolved
// from the rotation buffers of trial copy cq as above: Q^n at (cur + qsel) % 3,
// plain and out (in place) at (cur + rsel) % 3.
struct LcApply {
    const float* qn;
    const float* plain;
    float* out;
    const Ctrl* ctrl;
    int cq, qsel, rsel;
    float *buf0, *buf1, *buf2;
    const float *dF, *dG;
    unsigned char *bad, *keep_x, *keep_y;
    int nx, ny, ncell;
    float nux, nuy, tau, kappa;
    float s_out[3];  // output scales per frame channel (magnitude test)
    int premasked;   // dF / dG already zero where the indicator test fails
};
struct LcParams {
    float *theta, *m, *v;
    unsigned short *w1b, *w2b, *w3b;
};
int lc_net_waves(const LcNet& a, int cap);  // wavefronts per direction
int lc_cell_blocks(int64_t ncell);
hipError_t launch_lc_forward(const LcNet& a, hipStream_t s);
hipError_t launch_lc_backward(const LcNet& a, hipStream_t s);
hipError_t launch_lc_cellgrad(const LcCell& a, hipStream_t s);
hipError_t launch_lc_reduce(const float* partial, int nparts, float* grad, const double* loss_part, int nloss,
                            double inv3n, double* loss, hipStream_t s);
hipError_t launch_lc_init(const LcParams& a, hipStream_t s);
hipError_t launch_lc_adam(const LcParams& a, const float* grad, float lr, float beta1, float beta2, float eps,
                          float c1, float c2, hipStream_t s);
hipError_t launch_lc_apply(const LcApply& a, hipStream_t s);
hipError_t launch_lc_coarsen(const float* fine, float* coarse, int nx, int ny, hipStream_t s);
hipError_t launch_lc_perturb(const float* q, float* out, int ncell, const float* sigma, unsigned seed,
                             unsigned call, hipStream_t s);

// Element-wise set-up kernels.
template <typename R>
hipError_t launch_derive_zc(const R* aux, R* zc, int64_t ncell, hipStream_t s);
template <typename R>
hipError_t launch_sync_state(Ctrl* c, int q, R* b0, R* b1, R* b2, int64_t n, hipStream_t s);

}  // namespace claw
