/*
 * claw_oracle.c -- plain CPU oracle of the dimension-split wave-propagation
 * step (CUDACLAW paper, section 3 and section 4.1).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  It is written
 * for a reader to check against the paper by eye: explicit ghost cells, one
 * padded line at a time, every stage (boundary conditions, Riemann solve,
 * limiter, correction flux, update, speed maximum) as its own loop, in the
 * order the paper lists the pipeline stages (section 4.1).  Floating point is
 * FP64 (built with -ffp-contract=off, no fast-math).  The same source built with
 * -DORACLE_REAL=float gives an FP32 instantiation used only to measure the
 * rounding floor of single precision; the time-step scalars stay FP64 there.
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *  - wave limiter: MC limiter with the wave-projection ratio theta formed from
 *    the upwind neighbour chosen by the sign of the wave speed (LeVeque 2002,
 *    section 9.13); a wave of zero length has no correction;
 *  - correction flux F~ = 1/2 sum_p |s^p| (1 - dt/dx |s^p|) W~^p (LeVeque,
 *    section 6.13), the F~ / G~ terms of equation LW-update;
 *  - shallow water: Roe solver with arithmetic-mean depth and sqrt(h)-weighted
 *    velocities (LeVeque, section 15.3.3) and the Harten-Hyman entropy fix
 *    (LeVeque, section 15.3.5) applied to the 1- and 3-waves with strict
 *    inequalities; the fix is skipped for a middle state of depth <= 0;
 *  - acoustics: variable-coefficient solver with impedance Z = sqrt(rho K) and
 *    sound speed c = sqrt(K / rho) per cell (LeVeque, section 9.9); with rho =
 *    K = 1 it is the paper's system eq:acoustics;
 *  - boundary conditions are applied along the sweep direction before every
 *    sweep, from that sweep's input (2 ghost cells: extrapolation, reflecting
 *    wall, periodic); aux ghost cells use the same index map without sign flip;
 *    a wall on a line of a single cell mirrors that cell into both ghosts;
 *  - the speed maximum runs over the m+1 interfaces bounding interior cells.
 */
#include "claw_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#ifndef ORACLE_REAL
#define ORACLE_REAL double
#endif
typedef ORACLE_REAL real;

#define MAXEQ 4
#define MAXW 3
#define NG 2 /* ghost cells per side */

static int g_threads = 0;

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_num_threads(int n) { g_threads = n; }

static real rabs(real a) { return a < 0 ? -a : a; }
static real rmin(real a, real b) { return a < b ? a : b; }
static real rmax(real a, real b) { return a > b ? a : b; }

/* ------------------------------------------------------------------------ */
/* Riemann solvers (section 3: waves W^p, speeds s^p, fluctuations A-+dQ).   */
/* ------------------------------------------------------------------------ */

/* Linear acoustics p_t + K div u = 0, u_t + grad p / rho = 0 (eq:acoustics is
 * the case rho = K = 1).  Eigenvectors (-Z_l, 1) and (Z_r, 1) in the (p, u_n)
 * plane with speeds -c_l, +c_r; tangential velocities carry no wave. */
static void rp_acoustics(const real* ql, const real* qr, real Zl, real cl, real Zr, real cr,
                         int meqn, int nrm, real W[MAXW][MAXEQ], real s[MAXW],
                         real amdq[MAXEQ], real apdq[MAXEQ])
{
    int p, i;
    real dp = qr[0] - ql[0];
    real du = qr[nrm] - ql[nrm];
    real a1 = (-dp + Zr * du) / (Zl + Zr);
    real a2 = (dp + Zl * du) / (Zl + Zr);
    for (p = 0; p < 2; p++)
        for (i = 0; i < meqn; i++) W[p][i] = 0;
    W[0][0] = -a1 * Zl;
    W[0][nrm] = a1;
    W[1][0] = a2 * Zr;
    W[1][nrm] = a2;
    s[0] = -cl;
    s[1] = cr;
    for (i = 0; i < meqn; i++) {
        amdq[i] = s[0] * W[0][i];
        apdq[i] = s[1] * W[1][i];
    }
}

/* Shallow water (eq:SW), Roe linearisation plus Harten-Hyman entropy fix.
 * Components (h, m_n, m_t) with m_n the normal momentum.  Returns 5 if a
 * depth is not positive. */
static int rp_shallow_water(const real* ql, const real* qr, real g, int nrm, int efix,
                            real W[MAXW][MAXEQ], real s[MAXW], real amdq[MAXEQ],
                            real apdq[MAXEQ])
{
    int tng = 3 - nrm;
    int p, i;
    real hl = ql[0], hr = qr[0];
    real ul, vl, ur, vr, shl, shr, hbar, uhat, vhat, chat;
    real dh, dn, dtg, a1, a2, a3;
    real aminus[MAXW];

    if (!(hl > 0) || !(hr > 0) || !isfinite((double)hl) || !isfinite((double)hr)) return 5;

    ul = ql[nrm] / hl;
    vl = ql[tng] / hl;
    ur = qr[nrm] / hr;
    vr = qr[tng] / hr;

    /* Roe averages */
    shl = sqrt(hl);
    shr = sqrt(hr);
    hbar = (real)0.5 * (hl + hr);
    uhat = (shl * ul + shr * ur) / (shl + shr);
    vhat = (shl * vl + shr * vr) / (shl + shr);
    chat = sqrt(g * hbar);

    /* wave strengths: dQ projected on the Roe eigenvectors */
    dh = hr - hl;
    dn = qr[nrm] - ql[nrm];
    dtg = qr[tng] - ql[tng];
    a1 = ((uhat + chat) * dh - dn) / (2 * chat);
    a2 = dtg - vhat * dh;
    a3 = (dn - (uhat - chat) * dh) / (2 * chat);

    s[0] = uhat - chat;
    s[1] = uhat;
    s[2] = uhat + chat;

    W[0][0] = a1;
    W[0][nrm] = a1 * s[0];
    W[0][tng] = a1 * vhat;
    W[1][0] = 0;
    W[1][nrm] = 0;
    W[1][tng] = a2;
    W[2][0] = a3;
    W[2][nrm] = a3 * s[2];
    W[2][tng] = a3 * vhat;

    /* left-going share a_p of each wave: min(s, 0) unless transonic */
    for (p = 0; p < 3; p++) aminus[p] = rmin(s[p], 0);
    if (efix) {
        /* 1-wave: characteristic speed left of it and in the middle state q_l + W^1 */
        real lam_l = ul - sqrt(g * hl);
        real hm = hl + W[0][0];
        real mm = ql[nrm] + W[0][nrm];
        if (hm > 0) {
            real lam_r = mm / hm - sqrt(g * hm);
            if (lam_l < 0 && lam_r > 0) aminus[0] = lam_l * (lam_r - s[0]) / (lam_r - lam_l);
        }
        /* 3-wave: middle state q_r - W^3 and the right state */
        {
            real lam_r3 = ur + sqrt(g * hr);
            real hm3 = hr - W[2][0];
            real mm3 = qr[nrm] - W[2][nrm];
            if (hm3 > 0) {
                real lam_l3 = mm3 / hm3 + sqrt(g * hm3);
                if (lam_l3 < 0 && lam_r3 > 0)
                    aminus[2] = lam_l3 * (lam_r3 - s[2]) / (lam_r3 - lam_l3);
            }
        }
    }
    for (i = 0; i < 3; i++) {
        amdq[i] = aminus[0] * W[0][i] + aminus[1] * W[1][i] + aminus[2] * W[2][i];
        apdq[i] = s[0] * W[0][i] + s[1] * W[1][i] + s[2] * W[2][i] - amdq[i];
    }
    return 0;
}

/* Scalar Burgers-type law with flux f(q) = c q^2 / 2 along the sweep: the
 * wave is the jump qr - ql and its speed the Rankine-Hugoniot shock speed
 * (f(qr) - f(ql)) / (qr - ql) = c (ql + qr) / 2 (LeVeque 2002, section 11.8
 * and the Burgers solver of section 12.2).  Entropy fix: when the
 * characteristic speeds c ql < 0 < c qr the exact solution is a transonic
 * rarefaction whose flux at the interface is f(0) = 0, so A-dQ = f(0) - f(ql)
 * and A+dQ = f(qr) - f(0); otherwise the whole jump moves to one side. */
static int rp_burgers(real ql, real qr, real c, real W[MAXW][MAXEQ], real s[MAXW],
                      real amdq[MAXEQ], real apdq[MAXEQ])
{
    if (!isfinite((double)ql) || !isfinite((double)qr)) return 5;
    W[0][0] = qr - ql;
    s[0] = c * (ql + qr) / 2;
    if (c * ql < 0 && c * qr > 0) {
        amdq[0] = -(c * ql * ql / 2);
        apdq[0] = c * qr * qr / 2;
    } else {
        amdq[0] = rmin(s[0], 0) * W[0][0];
        apdq[0] = rmax(s[0], 0) * W[0][0];
    }
    return 0;
}

/* MC limiter: phi(theta) = max(0, min((1 + theta) / 2, 2, 2 theta)). */
static real phi_mc(real theta)
{
    real a = (1 + theta) / 2;
    real b = 2 * theta;
    return rmax(0, rmin(a, rmin((real)2, b)));
}

double oracle_mc_phi(double theta) { return (double)phi_mc((real)theta); }

/* The other classical wave limiters of the high-resolution method (LeVeque
 * 2002, section 6.12): minmod max(0, min(1, theta)); superbee
 * max(0, min(1, 2 theta), min(2, theta)); van Leer (theta + |theta|) / (1 + |theta|). */
static real phi_of(int limiter, real theta)
{
    switch (limiter) {
    case ORC_LIM_MC: return phi_mc(theta);
    case ORC_LIM_MINMOD: return rmax(0, rmin(1, theta));
    case ORC_LIM_SUPERBEE: return rmax(0, rmax(rmin(1, 2 * theta), rmin(2, theta)));
    case ORC_LIM_VANLEER: return (theta + rabs(theta)) / (1 + rabs(theta));
    case ORC_LIM_NONE: return 1;
    default: return 0;
    }
}

double oracle_phi(int limiter, double theta) { return (double)phi_of(limiter, (real)theta); }

int oracle_riemann_acoustics(const double* ql, const double* qr, double Zl, double cl,
                             double Zr, double cr, int meqn, int normal, double* W,
                             double* s, double* amdq, double* apdq)
{
    real l[MAXEQ], r[MAXEQ], w[MAXW][MAXEQ], sp[MAXW], am[MAXEQ], ap[MAXEQ];
    int i, p;
    if (meqn < 2 || meqn > MAXEQ || normal < 1 || normal >= meqn) return 1;
    for (i = 0; i < meqn; i++) {
        l[i] = (real)ql[i];
        r[i] = (real)qr[i];
    }
    rp_acoustics(l, r, (real)Zl, (real)cl, (real)Zr, (real)cr, meqn, normal, w, sp, am, ap);
    for (p = 0; p < 2; p++) {
        s[p] = sp[p];
        for (i = 0; i < meqn; i++) W[p * meqn + i] = w[p][i];
    }
    for (i = 0; i < meqn; i++) {
        amdq[i] = am[i];
        apdq[i] = ap[i];
    }
    return 0;
}

int oracle_riemann_sw(const double* ql, const double* qr, double grav, int normal, int efix,
                      double* W, double* s, double* amdq, double* apdq)
{
    real l[MAXEQ], r[MAXEQ], w[MAXW][MAXEQ], sp[MAXW], am[MAXEQ], ap[MAXEQ];
    int i, p, rc;
    if (normal != 1 && normal != 2) return 1;
    for (i = 0; i < 3; i++) {
        l[i] = (real)ql[i];
        r[i] = (real)qr[i];
    }
    rc = rp_shallow_water(l, r, (real)grav, normal, efix, w, sp, am, ap);
    if (rc) return rc;
    for (p = 0; p < 3; p++) {
        s[p] = sp[p];
        for (i = 0; i < 3; i++) W[p * 3 + i] = w[p][i];
    }
    for (i = 0; i < 3; i++) {
        amdq[i] = am[i];
        apdq[i] = ap[i];
    }
    return 0;
}

int oracle_riemann_burgers(double ql, double qr, double c, double* W, double* s, double* amdq,
                           double* apdq)
{
    real w[MAXW][MAXEQ], sp[MAXW], am[MAXEQ], ap[MAXEQ];
    int rc = rp_burgers((real)ql, (real)qr, (real)c, w, sp, am, ap);
    if (rc) return rc;
    W[0] = w[0][0];
    s[0] = sp[0];
    amdq[0] = am[0];
    apdq[0] = ap[0];
    return 0;
}

/* ------------------------------------------------------------------------ */
/* One line of one sweep.                                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int system, meqn, mwaves, nrm, limiter, efix, has_aux;
    real g, dtdx, Z0, c0, coef;
} line_cfg;

typedef struct {
    long cap;
    real* P;    /* padded states, cell-major [(m+4)][meqn] */
    real* Zp;   /* padded impedance */
    real* cp;   /* padded sound speed */
    real* W;    /* [(m+4)][MAXW][MAXEQ] waves at interface j (between padded j-1 and j) */
    real* s;    /* [(m+4)][MAXW] */
    real* amdq; /* [(m+4)][MAXEQ] */
    real* apdq;
    real* F;    /* correction flux */
    real* Q;    /* updated interior cells [m][meqn] */
} line_work;

static int work_init(line_work* w, long m)
{
    long c = m + 2 * NG;
    memset(w, 0, sizeof(*w));
    w->cap = m;
    w->P = (real*)calloc((size_t)c * MAXEQ, sizeof(real));
    w->Zp = (real*)calloc((size_t)c, sizeof(real));
    w->cp = (real*)calloc((size_t)c, sizeof(real));
    w->W = (real*)calloc((size_t)c * MAXW * MAXEQ, sizeof(real));
    w->s = (real*)calloc((size_t)c * MAXW, sizeof(real));
    w->amdq = (real*)calloc((size_t)c * MAXEQ, sizeof(real));
    w->apdq = (real*)calloc((size_t)c * MAXEQ, sizeof(real));
    w->F = (real*)calloc((size_t)c * MAXEQ, sizeof(real));
    w->Q = (real*)calloc((size_t)m * MAXEQ, sizeof(real));
    return w->P && w->Zp && w->cp && w->W && w->s && w->amdq && w->apdq && w->F && w->Q;
}

static void work_free(line_work* w)
{
    free(w->P);
    free(w->Zp);
    free(w->cp);
    free(w->W);
    free(w->s);
    free(w->amdq);
    free(w->apdq);
    free(w->F);
    free(w->Q);
}

#define WV(w, j, p, i) ((w)->W[(((j) * MAXW) + (p)) * MAXEQ + (i)])
#define SV(w, j, p) ((w)->s[(j) * MAXW + (p)])

/* Solves every interface of the padded line, limits the waves, forms the
 * correction flux and updates the m interior cells.  Padded cell j holds cell
 * j - 2; interface j lies between padded cells j-1 and j.  Returns 0 or 5. */
static int sweep_line(const line_cfg* c, long m, line_work* w, real* smax, int speeds_only)
{
    const int meqn = c->meqn, mw = c->mwaves;
    long j;
    int p, i;
    real sm = 0;

    /* Riemann problems at interfaces 1 .. m+3 (1-based cells k-1/2, k = 0..m+2) */
    for (j = 1; j <= m + 3; j++) {
        const real* ql = w->P + (j - 1) * MAXEQ;
        const real* qr = w->P + j * MAXEQ;
        real Wl[MAXW][MAXEQ], sl[MAXW];
        if (c->system == ORC_ACOUSTICS) {
            real Zl = c->has_aux ? w->Zp[j - 1] : c->Z0;
            real cl = c->has_aux ? w->cp[j - 1] : c->c0;
            real Zr = c->has_aux ? w->Zp[j] : c->Z0;
            real cr = c->has_aux ? w->cp[j] : c->c0;
            rp_acoustics(ql, qr, Zl, cl, Zr, cr, meqn, c->nrm, Wl, sl, w->amdq + j * MAXEQ,
                         w->apdq + j * MAXEQ);
        } else if (c->system == ORC_SHALLOW_WATER) {
            int rc = rp_shallow_water(ql, qr, c->g, c->nrm, c->efix, Wl, sl,
                                      w->amdq + j * MAXEQ, w->apdq + j * MAXEQ);
            if (rc) return rc;
        } else {
            int rc = rp_burgers(ql[0], qr[0], c->coef, Wl, sl, w->amdq + j * MAXEQ,
                                w->apdq + j * MAXEQ);
            if (rc) return rc;
        }
        for (p = 0; p < mw; p++) {
            SV(w, j, p) = sl[p];
            for (i = 0; i < meqn; i++) WV(w, j, p, i) = Wl[p][i];
        }
    }

    /* largest speed over the interfaces bounding interior cells (j = 2 .. m+2) */
    for (j = 2; j <= m + 2; j++)
        for (p = 0; p < mw; p++) sm = rmax(sm, rabs(SV(w, j, p)));
    *smax = sm;
    if (speeds_only) return 0;

    /* limited waves and correction flux at j = 2 .. m+2 */
    for (j = 2; j <= m + 2; j++) {
        real* F = w->F + j * MAXEQ;
        for (i = 0; i < meqn; i++) F[i] = 0;
        if (c->limiter == ORC_FIRST_ORDER) continue;
        for (p = 0; p < mw; p++) {
            real sp = SV(w, j, p);
            real wnorm2 = 0, phi, coef;
            for (i = 0; i < meqn; i++) wnorm2 += WV(w, j, p, i) * WV(w, j, p, i);
            if (wnorm2 == 0) continue; /* no wave: no correction */
            if (c->limiter != ORC_LIM_NONE) {
                long J = sp > 0 ? j - 1 : j + 1; /* upwind interface */
                real dotup = 0;
                for (i = 0; i < meqn; i++) dotup += WV(w, J, p, i) * WV(w, j, p, i);
                phi = phi_of(c->limiter, dotup / wnorm2);
            } else {
                phi = 1;
            }
            coef = (real)0.5 * rabs(sp) * (1 - c->dtdx * rabs(sp));
            for (i = 0; i < meqn; i++) F[i] += coef * (phi * WV(w, j, p, i));
        }
    }

    /* conservative update of interior padded cells 2 .. m+1 (equation LW-update) */
    for (j = 2; j <= m + 1; j++) {
        const real* q = w->P + j * MAXEQ;
        real* out = w->Q + (j - 2) * MAXEQ;
        for (i = 0; i < meqn; i++)
            out[i] = q[i] - c->dtdx * (w->apdq[j * MAXEQ + i] + w->amdq[(j + 1) * MAXEQ + i]) -
                     c->dtdx * (w->F[(j + 1) * MAXEQ + i] - w->F[j * MAXEQ + i]);
    }
    return 0;
}

/* Ghost-cell source index along a line of m cells; *flip = 1 when the normal
 * component changes sign (reflecting wall). */
static long ghost_source(long i, long m, int bc_lo, int bc_hi, int* flip)
{
    long r;
    *flip = 0;
    if (i < 0) {
        if (bc_lo == ORC_BC_EXTRAP) return 0;
        if (bc_lo == ORC_BC_WALL) {
            *flip = 1;
            r = -1 - i;
            return r > m - 1 ? m - 1 : r;
        }
        return ((i % m) + m) % m;
    }
    if (i >= m) {
        if (bc_hi == ORC_BC_EXTRAP) return m - 1;
        if (bc_hi == ORC_BC_WALL) {
            *flip = 1;
            r = 2 * m - 1 - i;
            return r < 0 ? 0 : r;
        }
        return i % m;
    }
    return i;
}

/* ------------------------------------------------------------------------ */
/* Whole-grid sweeps.                                                       */
/* ------------------------------------------------------------------------ */

static int check_desc(const oracle_desc* d)
{
    int k;
    if (!d) return 1;
    if (d->ndim != 2 && d->ndim != 3) return 1;
    for (k = 0; k < 3; k++) {
        if (d->n[k] < 1) return 1;
        if (k < d->ndim && !(d->upper[k] > d->lower[k])) return 1;
        if (d->bc_lo[k] < 0 || d->bc_lo[k] > 2 || d->bc_hi[k] < 0 || d->bc_hi[k] > 2) return 1;
    }
    if (d->ndim == 2 && d->n[2] != 1) return 1;
    if (d->limiter < 0 || d->limiter > 5) return 1;
    if (d->splitting != ORC_GODUNOV && d->splitting != ORC_STRANG) return 1;
    if (d->system == ORC_ACOUSTICS) {
        if (d->meqn != 1 + d->ndim) return 1;
        if (!d->has_aux && !(d->rho > 0 && d->bulk > 0)) return 1;
    } else if (d->system == ORC_SHALLOW_WATER) {
        if (d->ndim != 2 || d->meqn != 3 || !(d->grav > 0)) return 1;
    } else if (d->system == ORC_BURGERS) {
        if (d->meqn != 1) return 1;
        for (k = 0; k < d->ndim; k++)
            if (!isfinite(d->coef[k])) return 1;
    } else {
        return 1;
    }
    return 0;
}

static double cell_width(const oracle_desc* d, int dir)
{
    return (d->upper[dir] - d->lower[dir]) / (double)d->n[dir];
}

/* q, qout: SoA arrays of real, size meqn * ncell. */
static int sweep_grid(const oracle_desc* d, const real* q, const real* aux, int dir, double dt,
                      real* qout, real* smax_out, int speeds_only)
{
    const long nx = d->n[0], ny = d->n[1], nz = d->n[2];
    const long ncell = nx * ny * nz;
    const long m = d->n[dir];
    const long stride = dir == 0 ? 1 : (dir == 1 ? nx : nx * ny);
    const long nlines = ncell / m;
    const int meqn = d->meqn;
    line_cfg cfg;
    real smax = 0;
    int status = 0;

    cfg.system = d->system;
    cfg.meqn = meqn;
    cfg.mwaves = d->system == ORC_ACOUSTICS ? 2 : (d->system == ORC_SHALLOW_WATER ? 3 : 1);
    /* the field that changes sign at a wall: the normal velocity / momentum;
     * a scalar law has none (a wall mirrors it) */
    cfg.nrm = d->system == ORC_BURGERS ? -1 : 1 + dir;
    cfg.coef = d->system == ORC_BURGERS ? (real)d->coef[dir] : 0;
    cfg.limiter = d->limiter;
    cfg.efix = d->efix;
    cfg.has_aux = d->system == ORC_ACOUSTICS && d->has_aux;
    cfg.g = (real)d->grav;
    cfg.dtdx = (real)(dt / cell_width(d, dir));
    cfg.Z0 = d->system == ORC_ACOUSTICS ? (real)sqrt(d->rho * d->bulk) : 0;
    cfg.c0 = d->system == ORC_ACOUSTICS ? (real)sqrt(d->bulk / d->rho) : 0;

#ifdef _OPENMP
#pragma omp parallel num_threads(oracle_num_threads())
#endif
    {
        line_work w;
        real my_max = 0;
        int my_status = 0;
        long L;
        int ok = work_init(&w, m);
        if (!ok) my_status = 1;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (L = 0; L < nlines; L++) {
            long base, j;
            int e;
            real sm = 0;
            if (my_status) continue;
            /* first cell of line L */
            if (dir == 0) base = L * nx;
            else if (dir == 1) base = (L / nx) * nx * ny + (L % nx);
            else base = L;
            /* gather the padded line with its ghost cells */
            for (j = -NG; j < m + NG; j++) {
                int flip;
                long src = ghost_source(j, m, d->bc_lo[dir], d->bc_hi[dir], &flip);
                long idx = base + src * stride;
                real* P = w.P + (j + NG) * MAXEQ;
                for (e = 0; e < meqn; e++) P[e] = q[e * ncell + idx];
                if (flip && cfg.nrm >= 0) P[cfg.nrm] = -P[cfg.nrm];
                if (cfg.has_aux) {
                    real rho = aux[idx], K = aux[ncell + idx];
                    w.Zp[j + NG] = sqrt(rho * K);
                    w.cp[j + NG] = sqrt(K / rho);
                }
            }
            e = sweep_line(&cfg, m, &w, &sm, speeds_only);
            if (e) {
                my_status = e;
                continue;
            }
            if (sm > my_max) my_max = sm;
            if (!speeds_only)
                for (j = 0; j < m; j++)
                    for (e = 0; e < meqn; e++)
                        qout[e * ncell + base + j * stride] = w.Q[j * MAXEQ + e];
        }
        if (ok) work_free(&w);
#ifdef _OPENMP
#pragma omp critical
#endif
        {
            if (my_max > smax) smax = my_max;
            if (my_status && !status) status = my_status;
        }
    }
    *smax_out = smax;
    return status;
}

/* ------------------------------------------------------------------------ */
/* Public entry points (double in, double out).                             */
/* ------------------------------------------------------------------------ */

static real* to_real(const double* a, long n)
{
    long i;
    real* r = (real*)malloc((size_t)(n > 0 ? n : 1) * sizeof(real));
    if (!r) return NULL;
    for (i = 0; i < n; i++) r[i] = (real)a[i];
    return r;
}

static void to_double(const real* a, double* out, long n)
{
    long i;
    for (i = 0; i < n; i++) out[i] = (double)a[i];
}

static long ncells(const oracle_desc* d) { return d->n[0] * d->n[1] * d->n[2]; }

int oracle_sweep(const oracle_desc* d, const double* q, const double* aux, int dir, double dt,
                 double* qout, double* smax)
{
    long nc, nq;
    real *rq, *ra = NULL, *ro, sm = 0;
    int rc;
    if (check_desc(d) || dir < 0 || dir >= d->ndim) return 1;
    nc = ncells(d);
    nq = nc * d->meqn;
    rq = to_real(q, nq);
    ro = (real*)malloc((size_t)nq * sizeof(real));
    if (d->system == ORC_ACOUSTICS && d->has_aux) ra = to_real(aux, 2 * nc);
    rc = sweep_grid(d, rq, ra, dir, dt, ro, &sm, 0);
    if (!rc) to_double(ro, qout, nq);
    if (smax) *smax = (double)sm;
    free(rq);
    free(ro);
    free(ra);
    return rc;
}

/* One split step on real arrays.  The input q0 is left untouched (a rejected
 * step must keep Q^n); the sweeps alternate between the scratch arrays s1 and
 * s2 and *res points at the one holding the result. */
/* One split step (section 3): Godunov splitting sweeps x, y (, z) with dt;
 * Strang splitting sweeps x, y (, z) with dt/2 except the last direction,
 * which takes dt, and then the half steps again in reverse order
 * (x/2 y x/2 in 2D, x/2 y/2 z y/2 x/2 in 3D).  The Courant number is dt times
 * the largest max|s|/dx over the directions. */
static int step_real(const oracle_desc* d, const real* q0, real* s1, real* s2, const real* aux,
                     double dt, real** res, double* smax, double* cfl)
{
    int k, rc, nsw, seq[5];
    double frac[5];
    const real* src = q0;
    real* dst = s1;
    double sm_dir[3] = {0, 0, 0}, sigma = 0;
    if (d->splitting == ORC_STRANG) {
        nsw = 2 * d->ndim - 1;
        for (k = 0; k < nsw; k++) {
            seq[k] = k < d->ndim ? k : nsw - 1 - k;
            frac[k] = seq[k] == d->ndim - 1 ? 1.0 : 0.5;
        }
    } else {
        nsw = d->ndim;
        for (k = 0; k < nsw; k++) {
            seq[k] = k;
            frac[k] = 1.0;
        }
    }
    for (k = 0; k < nsw; k++) {
        real sm = 0;
        rc = sweep_grid(d, src, aux, seq[k], frac[k] * dt, dst, &sm, 0);
        if (rc) return rc;
        if ((double)sm > sm_dir[seq[k]]) sm_dir[seq[k]] = (double)sm;
        src = dst;
        dst = dst == s1 ? s2 : s1;
    }
    for (k = 0; k < d->ndim; k++) {
        if (smax) smax[k] = sm_dir[k];
        if (sm_dir[k] / cell_width(d, k) > sigma) sigma = sm_dir[k] / cell_width(d, k);
    }
    *res = (real*)src;
    if (cfl) *cfl = dt * sigma;
    return 0;
}

int oracle_step(const oracle_desc* d, const double* q, const double* aux, double dt,
                double* qout, double* smax, double* cfl)
{
    long nc, nq;
    real *a, *b, *c, *ra = NULL, *res = NULL;
    int rc;
    if (check_desc(d)) return 1;
    nc = ncells(d);
    nq = nc * d->meqn;
    a = to_real(q, nq);
    b = (real*)malloc((size_t)nq * sizeof(real));
    c = (real*)malloc((size_t)nq * sizeof(real));
    if (d->system == ORC_ACOUSTICS && d->has_aux) ra = to_real(aux, 2 * nc);
    rc = step_real(d, a, b, c, ra, dt, &res, smax, cfl);
    if (!rc) to_double(res, qout, nq);
    free(a);
    free(b);
    free(c);
    free(ra);
    return rc;
}

static int speeds_real(const oracle_desc* d, const real* q, const real* aux, double* smax,
                       double* sigma)
{
    int dir, rc;
    double sg = 0;
    for (dir = 0; dir < d->ndim; dir++) {
        real sm = 0;
        rc = sweep_grid(d, q, aux, dir, 0.0, NULL, &sm, 1);
        if (rc) return rc;
        if (smax) smax[dir] = (double)sm;
        if ((double)sm / cell_width(d, dir) > sg) sg = (double)sm / cell_width(d, dir);
    }
    if (sigma) *sigma = sg;
    return 0;
}

int oracle_speeds(const oracle_desc* d, const double* q, const double* aux, double* smax)
{
    long nc;
    real *rq, *ra = NULL;
    int rc;
    if (check_desc(d)) return 1;
    nc = ncells(d);
    rq = to_real(q, nc * d->meqn);
    if (d->system == ORC_ACOUSTICS && d->has_aux) ra = to_real(aux, 2 * nc);
    rc = speeds_real(d, rq, ra, smax, NULL);
    free(rq);
    free(ra);
    return rc;
}

/* Next trial step from the largest speed sigma = max_d smax_d / dx_d. */
static int next_dt(double sigma, double cfl_desired, double dt_max, double* dt)
{
    if (sigma > 0) {
        double c = cfl_desired / sigma;
        *dt = c < dt_max ? c : dt_max;
        return 0;
    }
    if (isfinite(dt_max)) {
        *dt = dt_max;
        return 0;
    }
    return 6;
}

int oracle_advance(const oracle_desc* d, double* q, const double* aux, long nsteps, double dt0,
                   double cfl_desired, double cfl_max, double dt_max, double* t_out,
                   long* nreject, double* dt_log, int* acc_log, long max_log)
{
    long nc, nq, accepted = 0, rejected = 0, trials = 0, consecutive = 0;
    real *a, *b, *c, *ra = NULL;
    double dt, sigma, t = 0;
    int rc;
    if (check_desc(d) || nsteps < 0) return 1;
    nc = ncells(d);
    nq = nc * d->meqn;
    a = to_real(q, nq);
    b = (real*)malloc((size_t)nq * sizeof(real));
    c = (real*)malloc((size_t)nq * sizeof(real));
    if (d->system == ORC_ACOUSTICS && d->has_aux) ra = to_real(aux, 2 * nc);

    /* first trial step: given, or from the speeds of the initial state */
    rc = 0;
    if (dt0 > 0) {
        dt = dt0;
    } else {
        rc = speeds_real(d, a, ra, NULL, &sigma);
        if (!rc) rc = next_dt(sigma, cfl_desired, dt_max, &dt);
    }
    while (!rc && accepted < nsteps) {
        real* res = NULL;
        double smax[3] = {0, 0, 0};
        double cfl;
        int dir;
        rc = step_real(d, a, b, c, ra, dt, &res, smax, &cfl);
        if (rc) break;
        sigma = 0;
        for (dir = 0; dir < d->ndim; dir++)
            if (smax[dir] / cell_width(d, dir) > sigma) sigma = smax[dir] / cell_width(d, dir);
        if (dt_log && trials < max_log) dt_log[trials] = dt;
        if (cfl <= cfl_max) {
            /* accept: the result becomes the current state */
            real* old = a;
            a = res;
            if (res == b) b = old;
            else c = old;
            t += dt;
            accepted++;
            consecutive = 0;
            if (acc_log && trials < max_log) acc_log[trials] = 1;
        } else {
            /* revert: keep the state, redo with a smaller step */
            rejected++;
            consecutive++;
            if (acc_log && trials < max_log) acc_log[trials] = 0;
            if (consecutive > 64) rc = 6;
        }
        trials++;
        if (!rc) rc = next_dt(sigma, cfl_desired, dt_max, &dt);
    }
    if (!rc) to_double(a, q, nq);
    if (t_out) *t_out = t;
    if (nreject) *nreject = rejected;
    free(a);
    free(b);
    free(c);
    free(ra);
    return rc;
}

int oracle_advance_fixed(const oracle_desc* d, double* q, const double* aux, long nsteps,
                         const double* dts, double* cfl_log)
{
    long nc, nq, k;
    real *a, *b, *c, *ra = NULL;
    int rc = 0;
    if (check_desc(d) || nsteps < 0) return 1;
    nc = ncells(d);
    nq = nc * d->meqn;
    a = to_real(q, nq);
    b = (real*)malloc((size_t)nq * sizeof(real));
    c = (real*)malloc((size_t)nq * sizeof(real));
    if (d->system == ORC_ACOUSTICS && d->has_aux) ra = to_real(aux, 2 * nc);
    for (k = 0; k < nsteps && !rc; k++) {
        real* res = NULL;
        double cfl;
        rc = step_real(d, a, b, c, ra, dts[k], &res, NULL, &cfl);
        if (rc) break;
        if (cfl_log) cfl_log[k] = cfl;
        {
            real* old = a;
            a = res;
            if (res == b) b = old;
            else c = old;
        }
    }
    if (!rc) to_double(a, q, nq);
    free(a);
    free(b);
    free(c);
    free(ra);
    return rc;
}
