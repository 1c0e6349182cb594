/*
 * claw.h -- C ABI of the MI355X (gfx950) dimension-split wave-propagation
 * solver (the CUDACLAW method: Clawpack's second-order wave-propagation
 * scheme with dimensional splitting, run on the GPU).
 *
 * The method (section 3 of the paper): each time step applies, direction by
 * direction (x, then y, then z; equation LW-update), a sweep that solves a
 * Riemann problem at every cell interface (waves W^p, speeds s^p and
 * fluctuations A-dQ, A+dQ), limits the waves, forms the second-order
 * correction flux F~ and updates every cell once (single-stage update,
 * section 5.3).  The largest wave speed is reduced during the sweeps and a
 * control step checks the CFL condition (equation CFL-condition), accepts the
 * step or reverts it and picks the next time step (section 4.1).
 *
 * The user supplies the equations (Riemann solver kind), the grid, the
 * boundary conditions and the limiter (section 4.1); set-up and evolution are
 * driven from Python (section 6).
 *
 * Memory ownership: the library never allocates or frees device memory.  The
 * caller allocates the state q, the optional aux array and a workspace of
 * claw_workspace_bytes() bytes, keeps them alive until claw_destroy(), and
 * passes a HIP stream on which every call enqueues its work.
 *
 * Layouts (device memory, dtype per the descriptor):
 *   q   [meqn][nz][ny][nx], x fastest, no ghost cells.  Acoustics fields
 *       (p, u, v[, w]); shallow water (h, hu, hv); Burgers (q).
 *   aux [2][nz][ny][nx]: density rho and bulk modulus K per cell (acoustics
 *       with variable coefficients, maux = 2); NULL when maux = 0.
 * q is rotation buffer 0.  Between calls the current state may live in a
 * workspace buffer; claw_advance() ends with it copied back into q, and
 * claw_sync_state() does the same on demand.
 *
 * Errors: every call returns a claw_status; nothing throws across the ABI.
 * claw_last_error() gives a message for the last failing call of the thread.
 * Calls on one solver must not overlap (one host thread at a time).
 */
#ifndef CLAW_H
#define CLAW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct claw_solver claw_solver; /* opaque */

/* claw_desc.flags: CLAW_FLAG_FUSED_STEP runs each 2D shallow-water step as one
 * kernel (rows x-swept into LDS, then y-swept out of it) instead of an x and a
 * y sweep kernel; the same results, one read and one write of the state per
 * step.  CLAW_FLAG_SPLIT_STEP asks for the x and y sweep kernels.  With
 * neither flag an FP32 2D shallow-water grid (Godunov splitting) takes the
 * fused step when its state holds at least CLAW_FUSED_AUTO_BYTES (measured on
 * MI355X: fused faster from 3072^2 (108 MiB) up, the sweeps faster at 2048^2,
 * whose source and destination stay in the 256 MB Infinity Cache), else the x
 * and y sweeps; FP64 grids take the sweeps (measured faster at every size).
 * 3D acoustics grids whose rows hold 256 FP32 (128 FP64) cells with
 * extrapolation at both x ends follow the same rule with one kernel for the x
 * and y sweeps of every z plane, then the z sweep kernel (same results; at
 * 256^3 FP32 about 1.5x the three sweep kernels).  Other problems ignore both
 * flags. */
#define CLAW_FLAG_FUSED_STEP 1
#define CLAW_FLAG_SPLIT_STEP 4
#define CLAW_FUSED_AUTO_BYTES (96ull << 20)
/* claw_desc.flags: CLAW_FLAG_STRANG replaces Godunov splitting (x, y (, z)
 * sweeps of dt) by Strang splitting: sweeps of dt/2 around a full-dt sweep of
 * the last direction (x/2 y x/2 in 2D, x/2 y/2 z y/2 x/2 in 3D), second order
 * in time; the Courant number is still dt times the largest max|s|/dx. */
#define CLAW_FLAG_STRANG 2

typedef enum {
    CLAW_OK = 0,
    CLAW_E_INVALID = 1,     /* bad descriptor, pointer or argument */
    CLAW_E_UNSUPPORTED = 2, /* valid but not implemented combination */
    CLAW_E_HIP = 3,         /* HIP runtime failure */
    CLAW_E_CFL = 4,         /* step rejected by the CFL check; state is Q^n bitwise */
    CLAW_E_NONPHYSICAL = 5, /* depth <= 0 or not finite met in a sweep; state is Q^n */
    CLAW_E_STATE = 6        /* step control failed (no usable dt, too many rejections) */
} claw_status;

typedef enum { CLAW_FP32 = 0, CLAW_FP64 = 1 } claw_dtype;
/* Riemann solvers: linear acoustics (eq:acoustics, generalised to density
 * rho and bulk modulus K) and shallow water (eq:SW) with the Roe solver and
 * the Harten-Hyman entropy fix, both with specialised sweeps; and point-wise
 * solvers compiled in through the plug-in interface (section 4.2: the user
 * supplies the Riemann solver of one interface, the library runs it inside
 * its generic sweeps), ids from CLAW_RP_PLUGIN_BASE on:
 *   CLAW_RP_BURGERS              scalar q_t + sum_d (c_d q^2 / 2)_{x_d} = 0,
 *                                meqn = mwaves = 1, 2D or 3D, c_d = param[d],
 *                                transonic entropy fix;
 *   CLAW_RP_SHALLOW_WATER_GENERIC  the shallow-water solver written as a
 *                                plug-in (param[0] = g, param[1] != 0: entropy
 *                                fix), same results to rounding as the
 *                                specialised sweep.
 * claw_plugin_info() describes a plug-in id. */
typedef enum {
    CLAW_RP_ACOUSTICS = 0,
    CLAW_RP_SHALLOW_WATER = 1,
    CLAW_RP_PLUGIN_BASE = 16,
    CLAW_RP_BURGERS = 16,
    CLAW_RP_SHALLOW_WATER_GENERIC = 17
} claw_riemann;
/* Ghost-cell rules (2 ghost cells per side): zero-order extrapolation,
 * reflecting wall (normal velocity / momentum negated), periodic. */
typedef enum { CLAW_BC_EXTRAP = 0, CLAW_BC_WALL = 1, CLAW_BC_PERIODIC = 2 } claw_bc;
/* Wave limiters phi(theta) of the high-resolution method (section 3): MC,
 * none (phi = 1, Lax-Wendroff), first order (no correction), minmod, superbee,
 * van Leer. */
typedef enum {
    CLAW_LIM_MC = 0,
    CLAW_LIM_NONE = 1,
    CLAW_FIRST_ORDER = 2,
    CLAW_LIM_MINMOD = 3,
    CLAW_LIM_SUPERBEE = 4,
    CLAW_LIM_VANLEER = 5
} claw_limiter;

typedef struct {
    int32_t ndim;        /* 2 or 3 */
    int32_t meqn;        /* acoustics 1 + ndim; shallow water 3 (2D only) */
    int32_t mwaves;      /* acoustics 2; shallow water 3 */
    int32_t maux;        /* 0, or 2 for acoustics with per-cell rho, K */
    int64_t n[3];        /* cells per direction, x fastest; n[2] = 1 in 2D */
    double lower[3];     /* domain corner */
    double upper[3];
    int32_t riemann;     /* claw_riemann */
    int32_t limiter;     /* claw_limiter */
    int32_t dtype;       /* claw_dtype */
    int32_t efix;        /* shallow water: 1 = entropy fix (default) */
    int32_t bc_lo[3];    /* claw_bc per direction */
    int32_t bc_hi[3];
    int32_t num_ghost;   /* must be 2 */
    int32_t flags;       /* CLAW_FLAG_* bits, 0 for the default path */
    double rho, bulk;    /* acoustics coefficients when maux = 0 */
    double grav;         /* shallow water gravity */
    double cfl_desired;  /* target Courant number for the next step (0.9) */
    double cfl_max;      /* largest accepted Courant number (1.0) */
    double dt_max;       /* upper bound on dt (+inf for none) */
    double param[4];     /* plug-in solvers: their parameters (see claw_riemann) */
} claw_desc;

/* Fills *d with defaults (MC limiter, entropy fix on, 2 ghosts, CFL 0.9 / 1.0,
 * dt_max = +inf); the caller then sets grid, system and boundary conditions.
 * Defined by: section 4.1 (the user states the equations, grid, boundary conditions
 * and limiter) and equation CFL-condition (the Courant limits). */
void claw_desc_init(claw_desc* d);

/* Plug-in solver id (claw_desc.riemann >= CLAW_RP_PLUGIN_BASE): its field
 * and wave counts, the largest ndim it runs in, the first field of the vector
 * that rotates with the sweep direction (-1 if none; a wall negates its normal
 * component) and a static name.  Any output pointer may be NULL.
 * CLAW_E_INVALID if id names no compiled plug-in.
 * Defined by: section 4.2 (point-wise Riemann solver supplied by the user). */
claw_status claw_plugin_info(int32_t id, int32_t* meqn, int32_t* mwaves, int32_t* ndim_max,
                             int32_t* vec_field, const char** name);

/* Workspace size in bytes for descriptor d (two scratch state buffers, the
 * derived acoustic coefficients and the control block).  CLAW_E_INVALID for a
 * bad descriptor.
 * Defined by: section 4.3 (one global array per field; waves never stored) and
 * section 4.1 (a revert needs Q^n kept). */
claw_status claw_workspace_bytes(const claw_desc* d, size_t* bytes);

/* Validates d and binds the caller's device buffers.  q, aux, workspace are
 * device pointers (aux NULL iff maux = 0); stream is a hipStream_t (NULL =
 * the null stream).  Enqueues the set-up kernels (derived coefficients,
 * control block) on the stream.  *out receives the handle.  The rows per
 * column-sweep workgroup are chosen from the grid and the device's CU count;
 * the environment variables CLAW_COL_WAVES (target wavefronts per column
 * sweep) and CLAW_COL_CHUNK (rows per chunk) override that choice for tuning,
 * read once per process; values <= 0 are ignored.
 * Defined by: section 4.1 (problem set-up: Riemann solver, grid, boundary conditions)
 * and section 6 (set-up driven from Python). */
claw_status claw_create(const claw_desc* d, void* q, const void* aux, void* workspace,
                        size_t workspace_bytes, void* stream, claw_solver** out);

/* Speed-only pass (Riemann speeds of every direction on the current state,
 * nothing updated) and host sync: *sigma = max_d max|s| / dx_d.  smax (may be
 * NULL) receives max|s| per direction.
 * Defined by: equation CFL-condition and the speed reduction of section 4.1. */
claw_status claw_cfl(claw_solver* h, double* sigma, double* smax);

/* One trial step x, y (, z) with time step dt (section 4.1 pipeline).  If the
 * Courant number dt * sigma exceeds cfl_max the step is reverted (state stays
 * Q^n bitwise).  If cfl != NULL the call synchronises, stores the Courant
 * number and returns CLAW_E_CFL for a rejected step, CLAW_E_NONPHYSICAL for a
 * non-physical state; with cfl == NULL nothing is synchronised and the
 * outcome is only recorded in the control block.
 * Defined by: equation LW-update (the split step) and section 4.1 (pipeline; revert
 * when the CFL condition fails). */
claw_status claw_step(claw_solver* h, double dt, double* cfl);

/* One directional sweep dir (0, 1, 2) with time step dt, always accepted
 * (a building block for tests; the result becomes the current state).
 * smax (may be NULL) receives the largest |s| of the sweep (synchronises).
 * Defined by: equation LW-update (one directional sweep of the splitting) and
 * section 5.3 (single-stage update). */
claw_status claw_sweep(claw_solver* h, int32_t dir, double dt, double* smax);

/* Adaptive stepping with revert (the production path): advances by nsteps
 * accepted steps.  The first trial step is dt0 if dt0 > 0, else the dt_next
 * left by a previous call, else cfl_desired / sigma of a speed pass.  Each
 * trial's dt is min(dt_max, cfl_desired / sigma) of the previous trial.  The
 * step sequence runs from a captured HIP graph with dt kept on the device;
 * the call synchronises once at the end and leaves the state in q.
 * *t receives the simulation time, *nreject the rejected trials of this call
 * (either may be NULL).
 * Defined by: section 4.1 (time step from the previous step's speeds; revert and redo
 * on a CFL violation) and equation CFL-condition. */
claw_status claw_advance(claw_solver* h, int64_t nsteps, double dt0, double* t,
                         int64_t* nreject);

/* Prescribed time steps: one step per entry of dts (host array), each always
 * accepted; cfl_log (host, may be NULL) receives each step's Courant number.
 * Synchronises; the state is left in q.
 * Defined by: equation LW-update applied with given time steps. */
claw_status claw_advance_fixed(claw_solver* h, int64_t nsteps, const double* dts,
                               double* cfl_log);

/* Like claw_advance but launched eagerly with a HIP event pair around every
 * kernel, for per-kernel timing: kernel_ms[k] receives the summed duration of
 * the sweeps in direction k (0: x, 1: y, 2: z; the step control runs inside
 * the last sweep of a step; slot 3 is unused) and launches[k] their count
 * (either array may be NULL; both have 4 entries).
 * Defined by: section 7.1 (per-kernel measurement behind the roofline). */
claw_status claw_advance_timed(claw_solver* h, int64_t nsteps, double* kernel_ms,
                               int64_t* launches);

/* One directional sweep like claw_sweep, without a solver handle or a
 * workspace, for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).  The
 * grid is described by d (claw_create's rules; flags must not ask for
 * Strang splitting); src and dst are device states in q's layout (16-byte
 * aligned, not aliasing); dst receives the sweep of src in direction dir
 * (0, 1, 2) with time step dt, always accepted; aux as for claw_create.
 * smax_dev (device double, may be NULL) receives the largest |s| of the
 * sweep, or a NaN if the sweep met a non-physical state (depth <= 0 or not
 * finite).  Enqueued on stream, which must belong to the current device; no
 * synchronisation.
 * Scratch: the step state, the speed maxima and (maux = 2) the derived
 * coefficients Z, c live in one static device array per GPU, held until
 * the process ends: a 32 KiB control block plus CLAW_NOALLOC_ZC_BYTES for
 * the coefficients; a grid whose coefficients (2 ncell sizeof(real) bytes)
 * exceed that limit gets CLAW_E_UNSUPPORTED.  Every call clears what it
 * uses first.  Calls on one GPU share the array: calls that overlap in time
 * (other streams or host threads on the same GPU) race and must be
 * serialised by the caller.  The call allocates nothing (no hipMalloc, no
 * stream or event creation). */
#define CLAW_NOALLOC_ZC_BYTES (16u << 20)
claw_status claw_sweep_noalloc(const claw_desc* d, const void* src, void* dst, const void* aux, int32_t dir,
                               double dt, double* smax_dev, void* stream);

/* Enqueues a copy of the current state into q if it lives in a workspace
 * buffer; no synchronisation.
 * Defined by: section 6 (the caller's array holds the solution it evolves). */
claw_status claw_sync_state(claw_solver* h);

/* Step-control scalars (synchronises).  Any output pointer may be NULL.
 * Defined by: section 4.1 (time, next time step, accepted and reverted steps). */
claw_status claw_get_control(claw_solver* h, double* t, double* dt_next, int64_t* accepted,
                             int64_t* rejected);
/* Restores t and dt_next (checkpoint / resume); enqueued, no sync.
 * Defined by: section 4.1 (the next step's dt comes from the previous step). */
claw_status claw_set_control(claw_solver* h, double t, double dt_next);

/* Releases the handle (waits for its stream first).  Device buffers stay the
 * caller's.
 * Defined by: section 6 (the caller owns the arrays it passed in). */
claw_status claw_destroy(claw_solver* h);


/* ---------------------------------------------------------------------------
 * Batched ensembles: many independent 2D shallow-water grids of different
 * sizes advanced together (each with its own adaptive dt, accept / revert and
 * step count).  Every sweep of every instance runs in one launch per sweep
 * direction; a table maps each workgroup to (instance, block), and the
 * whole multi-step run replays a captured HIP graph.  Each instance's result is
 * bitwise the single-grid result on the same step.  A batch runs the fused 2D
 * step (per trial one opening launch, one thread per instance, and one fused
 * launch for all instances) under the single grid's rule applied to the
 * batch's whole state: with CLAW_FLAG_FUSED_STEP, or FP32 with at least
 * CLAW_FUSED_AUTO_BYTES of state and no CLAW_FLAG_SPLIT_STEP; else the x and
 * y sweeps.  Descriptors carry no other flag, and all carry the same ones
 * (CLAW_E_INVALID otherwise).
 * ------------------------------------------------------------------------- */
typedef struct claw_batch claw_batch; /* opaque */

/* Workspace bytes for count descriptors (all 2D shallow water, one dtype).
 * Defined by: section 8 (independent subproblems on one device) and section 4.3
 * (one array per field). */
claw_status claw_batch_workspace_bytes(const claw_desc* descs, int32_t count, size_t* bytes);
/* q[i]: device state of instance i (layout as for claw_create, 256-byte
 * aligned); workspace: device buffer of claw_batch_workspace_bytes() bytes.
 * Defined by: section 8 (independent subproblems) and section 4.1 (set-up). */
claw_status claw_batch_create(const claw_desc* descs, int32_t count, void* const* q, void* workspace,
                              size_t workspace_bytes, void* stream, claw_batch** out);
/* Autotuner: times state-preserving trial steps (dt = 0) for each candidate
 * column chunk {16, 32, 64, 128} x block schedule (0 largest instances
 * first, 1 round-robin) x rows each row-sweep wavefront takes in turn
 * {2, 4, 8} (fused batches: rows per fused workgroup {16, 24, 32, 48, 64} x
 * schedule), keeps the fastest, and records it in the JSON cache file
 * cache_path (may be NULL) keyed by arch, dtype, system, instance count and
 * total-cell bucket; a cached key is used without timing.  Outputs may be
 * NULL.  Synchronises.
 * Defined by: section 5.2 (block shapes chosen for the hardware). */
claw_status claw_batch_tune(claw_batch* b, const char* cache_path, int32_t* chunk, int32_t* schedule,
                            int32_t* rows_per_wave, double* us_per_step);
/* Fixes the tile choice by hand (chunk >= 8, fused batches >= 16: their rows
 * per fused workgroup; schedule 0 or 1; rows_per_wave
 * 2, 4 or 8; the default after claw_batch_create is 32, 0, 8).
 * Defined by: section 5.2 (block shapes). */
claw_status claw_batch_set_tiles(claw_batch* b, int32_t chunk, int32_t schedule, int32_t rows_per_wave);
/* Advances every instance by nsteps accepted steps (adaptive dt per
 * instance, first dt from a speed pass); t[i], nreject[i] (host arrays of
 * count entries, may be NULL) receive each instance's time and rejected
 * trials of this call.  Synchronises; states end in q[i].
 * Defined by: section 4.1 (adaptive step with revert, per instance) and section 8
 * (independent subproblems). */
claw_status claw_batch_advance(claw_batch* b, int64_t nsteps, double* t, int64_t* nreject);
/* Defined by: section 6 (the caller owns the arrays it passed in). */
claw_status claw_batch_destroy(claw_batch* b);

/* ------------------------------------------------------------------------
 * Learned coarse-grid flux correction.
 *
 * On a shallow-water grid twice as coarse as a reference run, a small network
 * maps the four-cell stencil around every interior face to a correction of
 * that face's flux, and the corrected step is the plain split step followed
 * by the difference of the corrections (the flux-difference form of the
 * conservative update, section 3, equation LW-update):
 *   Q^{n+1} = S(Q^n) - nu_x (dF_{i+1/2} - dF_{i-1/2}) - nu_y (dG_{j+1/2} - dG_{j-1/2}),
 * nu = dt/dx.  Wall faces carry no correction, so every field's sum changes
 * by rounding only.  Two networks (12 -> 64 -> 64 -> 3, ReLU), one for the
 * faces of each sweep direction (the split step sweeps x then y, so the two
 * directions carry different errors), run on BF16 matrix cores with FP32
 * accumulation; their parameters are FP32 masters with BF16 copies of the
 * weights.  Grids are FP32 (3, ny, nx) states (h, hu, hv)
 * with reflecting walls on all four sides.
 *
 * Face frame: faces along x see (h, hu, hv), faces along y (h, hv, hu) =
 * (depth, normal momentum, tangential momentum); stencil cells k-2 .. k+1
 * of face k-1/2, mirrored across a wall with the normal momentum negated.
 * Inputs per channel c with stencil values a, b, e, f (level, slope,
 * curvature, third difference):
 *   ((b + e)/2 - mu_c)/sl[c], (e - b)/sd1[c], ((a + f) - (b + e))/sd2[c],
 *   ((f - a) - 3 (e - b))/sd3[c]
 * with mu = (mu_h, 0, 0); the outputs are scaled by s_out[c].
 * ------------------------------------------------------------------------ */
#define CLAW_LC_NET 5187 /* per network: W1 (64,12), b1 (64), W2 (64,64), b2 (64), W3 (3,64), b3 (3) */
#define CLAW_LC_NPARAM (2 * CLAW_LC_NET) /* x-face network, then y-face network */

typedef struct {
    int64_t nx, ny; /* coarse grid, both >= 2, 3 nx ny < 2^31 */
    float mu_h;     /* input normalisation */
    float sl[3], sd1[3], sd2[3], sd3[3];
    float s_out[3]; /* output scale per frame channel */
} claw_lc_desc;

/* Device bytes of the parameter block (masters, Adam moments, BF16 copies;
 * layout private except that the first CLAW_LC_NPARAM floats are the FP32
 * masters in the order above) and of the scratch workspace a grid needs.
 * Defined by: equation LW-update (the correction enters as a flux difference). */
claw_status claw_lc_sizes(const claw_lc_desc* d, size_t* param_bytes, size_t* work_bytes);

/* After the caller has written the masters: zeroes the Adam moments and
 * emits the BF16 copies.  Enqueued on `stream`.
 * Defined by: equation LW-update (parameters of the flux-difference correction). */
claw_status claw_lc_init(void* params, void* stream);

/* Corrections of every face of state q: dF (3, ny, nx+1) and dG (3, ny+1, nx)
 * in state component order, zero on wall faces.  Enqueued.
 * Defined by: equation LW-update (per-face fluxes F~, G~ of the update). */
claw_status claw_lc_forward(const claw_lc_desc* d, const void* params, const float* q, float* dF, float* dG,
                            void* stream);

/* Training pass on one sample: state q = Q^n, plain = S(Q^n), target =
 * reference state at t^{n+1}.  Loss
 *   L = sum_{cells, f} w[f] (p - r)^2 / (3 nx ny),  r = target - plain,
 *   p = -nu_x (dF_{i+1/2} - dF_{i-1/2}) - nu_y (dG_{j+1/2} - dG_{j-1/2}).
 * Writes the parameter gradient to grad (device, CLAW_LC_NPARAM floats) and,
 * if loss != NULL, loss[0] = L and loss[1..3] = sum r_f^2 (device doubles).
 * BF16 rounding points: inputs, weights, activations, and the output and
 * pre-activation gradients entering products; bias gradients sum unrounded
 * values.  Enqueued; workspace from claw_lc_sizes.
 * Defined by: equation LW-update (the corrected update whose error is fitted). */
claw_status claw_lc_loss_grad(const claw_lc_desc* d, const void* params, const float* q, const float* target,
                              const float* plain, double nux, double nuy, const double* w, void* work,
                              float* grad, double* loss, void* stream);

/* One Adam step (step counts from 1) on the masters with gradient grad, then
 * new BF16 copies.  Enqueued.
 * Defined by: equation LW-update (training of the flux-difference correction). */
claw_status claw_lc_adam(void* params, const float* grad, int64_t step, double lr, double beta1, double beta2,
                         double eps, void* stream);

/* Fallback and application: out = plain - flux difference of the kept
 * corrections.  A face keeps its correction when |h_R - h_L| <= tau min(h_L,
 * h_R) (no shock across it, h from qn) and |d_c| <= kappa s_out[c] for the
 * three components in the face frame (the output within kappa of its scale);
 * then faces next to a bad cell are dropped: a cell whose depth from only
 * those kept faces that lower it is below half its plain depth, or not
 * positive (that worst case bounds its depth whatever faces are dropped, so
 * every cell ends at half its plain depth or more).  FP32 decisions.  out may alias plain.  keep_x (ny, nx+1) and keep_y (ny+1, nx),
 * optional, receive 1 where a face kept its correction.  Enqueued.
 * Defined by: equation LW-update (conservative flux-difference form) and eq:SW (depth
 * positivity). */
claw_status claw_lc_apply(const claw_lc_desc* d, const float* qn, const float* plain, const float* dF,
                          const float* dG, double nux, double nuy, double tau, double kappa, float* out,
                          uint8_t* keep_x, uint8_t* keep_y, void* work, void* stream);

/* 2 x 2 cell averages of a fine FP32 state (3, 2ny, 2nx) into coarse (3, ny, nx).
 * Enqueued.
 * Defined by: section 3 (cell averages Q_ij of the finite-volume method). */
claw_status claw_lc_coarsen(int64_t nx, int64_t ny, const float* fine, float* coarse, void* stream);

/* Training input noise: out = q + sigma_f z for every value of an FP32 state
 * (3, ny, nx) (f the field), z standard normal from Philox4x32-10 (a
 * counter-based generator: counter (i / 2, call, 0, 0), key (seed, 0)) and
 * the Box-Muller transform of its first two words (values 2k and 2k + 1 share
 * one draw).  q, out: device buffers (may alias); sigma: host array of 3.
 * Enqueued.
 * Defined by: equation LW-update (training of the flux-difference correction
 * on perturbed coarse states). */
claw_status claw_lc_perturb(int64_t nx, int64_t ny, const float* q, float* out, const float* sigma, uint32_t seed,
                            uint32_t call, void* stream);

/* Output scales and loss weights from the residual energy of the first
 * samples: r2[f] = sum over ncell cells of the squared residual of field f
 * (host array of 3).  With ms_f = max(r2[f] / ncell, 1e-30): w[f] = 1 / ms_f,
 * s_out = (sqrt(ms_h) / nu or 0 when correct_depth is 0, m / nu, m / nu) with
 * m the mean of the momenta's sqrt(ms).  Host arithmetic only.
 * Defined by: equation LW-update (scales of the flux-difference correction). */
claw_status claw_lc_scales(const double* r2, int64_t ncell, double nu, int32_t correct_depth, float* s_out,
                           double* w);

/* nsteps learned coarse steps of fixed dt on solver h (FP32 2D shallow water,
 * walls, grid d->nx x d->ny): each is the plain split step followed by the
 * corrections computed from Q^n and applied as above, with no host round trip
 * between steps.  The state is left in the solver's q.  Synchronises at the end;
 * CLAW_E_NONPHYSICAL as for claw_advance_fixed.
 * Defined by: equation LW-update (plain split step plus the flux difference). */
claw_status claw_lc_advance(claw_solver* h, const claw_lc_desc* d, const void* params, int64_t nsteps, double dt,
                            double tau, double kappa, void* work);

/* Achievable-bandwidth microbenchmark (the paper's achievable roof, section
 * 7.1): streams over device buffers a (read, must be zero-filled) and b
 * (written), each of `bytes` bytes, reps times per kernel, on `stream`, and
 * stores GB/s in gbps[5]: copy, copy with non-temporal stores, read only,
 * write only, write only non-temporal.  Synchronises.
 * Defined by: section 7.1 (achievable bandwidth roof). */
claw_status claw_stream_bench(void* a, void* b, size_t bytes, int32_t reps, void* stream,
                              double* gbps);

/* Range checks of a debug build (libclaw_debug.so, compiled with CLAW_DEBUG),
 * for callers hunting an indexing error: every buffer load and store of the
 * kernels checks its byte range against the field it addresses, and the
 * boundary index map checks the cell it resolves (the boundary-condition
 * stage of section 4.1).
 * A failed check is counted on the device and the kernel carries on as a
 * release build would.  Returns in *count the number of failed checks since
 * the last call (over every kernel file) and in *first_line the source line
 * of the first one (0 if none), then clears the counts; synchronises the
 * current device.  Either pointer may be NULL.  A release build returns
 * CLAW_E_UNSUPPORTED. */
claw_status claw_debug_take(uint64_t* count, uint32_t* first_line);

/* Defined by: section 4.1 (the CFL revert and failure outcomes of a step). */
const char* claw_status_string(claw_status s);
/* Defined by: section 4.1 (why the last call failed). */
const char* claw_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
