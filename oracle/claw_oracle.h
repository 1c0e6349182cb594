/*
 * claw_oracle.h -- CPU oracle for the dimension-split wave-propagation step.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, deliberately unoptimised
 * FP64 implementation of the finite-volume scheme of the CUDACLAW paper
 * (section 3: the Godunov-split update, equation LW-update; the Riemann solve
 * and the wave limiter described right after it; the CFL condition, equation
 * CFL-condition; the acoustics and shallow-water systems, equations
 * eq:acoustics and eq:SW; the revert-and-redo rule of section 4.1), plus a
 * scalar Burgers-type law as the example of a user-supplied point-wise
 * Riemann solver (section 4.2).  Where the
 * paper leaves a formula unstated the textbook definition it cites for the
 * method (LeVeque, Finite Volume Methods for Hyperbolic Problems, 2002) is
 * written out instead; each such reading is named in the source.
 *
 * Only the test suite, the smoke check and the CPU baseline of the benchmark
 * may load this library.  It shares no code, header or constant with the GPU
 * library; the two are compared on the same seeded inputs.
 *
 * Layout: a state q is structure-of-arrays, q[m][nz][ny][nx] contiguous with x
 * fastest, no ghost cells.  aux (acoustics only) is aux[2][nz][ny][nx] holding
 * density rho and bulk modulus K per cell.  All pointers are host pointers owned
 * by the caller.  Functions return 0 on success and a nonzero code on error:
 *   1 invalid description, 5 non-physical state (depth <= 0 or not finite),
 *   6 step control failed (no acceptable time step / too many rejections).
 */
#ifndef CLAW_ORACLE_H
#define CLAW_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_ACOUSTICS = 0, ORC_SHALLOW_WATER = 1, ORC_BURGERS = 2 };
enum { ORC_BC_EXTRAP = 0, ORC_BC_WALL = 1, ORC_BC_PERIODIC = 2 };
enum { ORC_LIM_MC = 0, ORC_LIM_NONE = 1 /* phi = 1: Lax-Wendroff */, ORC_FIRST_ORDER = 2,
       ORC_LIM_MINMOD = 3, ORC_LIM_SUPERBEE = 4, ORC_LIM_VANLEER = 5 };

typedef struct {
    int ndim;            /* 2 or 3 */
    long n[3];           /* cells per direction, n[2] = 1 in 2D */
    double lower[3];
    double upper[3];
    int meqn;            /* acoustics: 1 + ndim; shallow water: 3; Burgers: 1 */
    int system;          /* ORC_ACOUSTICS, ORC_SHALLOW_WATER or ORC_BURGERS */
    int limiter;         /* ORC_LIM_* */
    int efix;            /* shallow water: 1 = Harten-Hyman entropy fix */
    int bc_lo[3];
    int bc_hi[3];
    int has_aux;         /* acoustics: 1 = per-cell rho, K in aux */
    double rho, bulk;    /* acoustics coefficients when has_aux == 0 */
    double grav;         /* shallow water gravity */
    int splitting;       /* ORC_GODUNOV: x, y (, z) sweeps of dt; ORC_STRANG: half-step
                            sweeps around a full step of the last direction */
    double coef[3];      /* Burgers: flux coef[d] q^2 / 2 along direction d */
} oracle_desc;

enum { ORC_GODUNOV = 0, ORC_STRANG = 1 };

/* Single-interface Riemann solvers (section 3; section 4.2 point-wise form).
 * ql, qr: the meqn-vectors of the left and right cell.  normal: index of the
 * normal velocity / momentum component.  Outputs: W[p*meqn + i] (waves),
 * s[p] (speeds), amdq, apdq (fluctuations A-dQ, A+dQ). */
int oracle_riemann_acoustics(const double* ql, const double* qr, double Zl, double cl,
                             double Zr, double cr, int meqn, int normal, double* W,
                             double* s, double* amdq, double* apdq);
int oracle_riemann_sw(const double* ql, const double* qr, double grav, int normal,
                      int efix, double* W, double* s, double* amdq, double* apdq);

/* Scalar Burgers-type law q_t + sum_d (coef_d q^2 / 2)_{x_d} = 0 along one
 * direction with coefficient c: one wave qr - ql at the Rankine-Hugoniot speed
 * c (ql + qr) / 2; a transonic rarefaction (c ql < 0 < c qr) splits its flux
 * difference at q = 0.  Returns 5 for a non-finite state. */
int oracle_riemann_burgers(double ql, double qr, double c, double* W, double* s, double* amdq,
                           double* apdq);

/* MC limiter function phi(theta). */
double oracle_mc_phi(double theta);
/* phi(theta) of a limiter (ORC_LIM_*); 1 for ORC_LIM_NONE, 0 for ORC_FIRST_ORDER. */
double oracle_phi(int limiter, double theta);

/* One directional sweep d (0 = x, 1 = y, 2 = z) with time step dt:
 * qout = sweep_d(q); *smax = largest |s| over the sweep's interfaces. */
int oracle_sweep(const oracle_desc* d, const double* q, const double* aux, int dir, double dt,
                 double* qout, double* smax);

/* One full split step x, y (, z).  smax[dir] as above per direction,
 * *cfl = dt * max_dir smax[dir] / dx[dir]. */
int oracle_step(const oracle_desc* d, const double* q, const double* aux, double dt,
                double* qout, double* smax, double* cfl);

/* Speed-only pass: Riemann speeds of every direction on q, nothing updated. */
int oracle_speeds(const oracle_desc* d, const double* q, const double* aux, double* smax);

/* Adaptive time stepping with revert: advances q in place by nsteps accepted
 * steps.  dt0 > 0 is the first trial step, else cfl_desired / sigma(q0).
 * dt_log (optional, length max_log) receives every trial dt in order and
 * acc_log (optional) whether it was accepted.  */
int oracle_advance(const oracle_desc* d, double* q, const double* aux, long nsteps, double dt0,
                   double cfl_desired, double cfl_max, double dt_max, double* t_out,
                   long* nreject, double* dt_log, int* acc_log, long max_log);

/* Fixed time steps: applies oracle_step with dts[0..nsteps-1] in place. */
int oracle_advance_fixed(const oracle_desc* d, double* q, const double* aux, long nsteps,
                         const double* dts, double* cfl_log);

/* Number of threads the library's parallel loops use (1 if built without OpenMP). */
int oracle_num_threads(void);
void oracle_set_num_threads(int n);

#ifdef __cplusplus
}
#endif
#endif
