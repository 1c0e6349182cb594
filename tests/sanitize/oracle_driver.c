/* Drives the CPU oracle through every system, boundary rule, limiter and
 * splitting on small ragged grids, for a build under AddressSanitizer and
 * UndefinedBehaviorSanitizer (test infrastructure; see
 * tests/test_sanitizers.py).  Exits nonzero on an oracle error code. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/claw_oracle.h"

static double urand(unsigned* s) {
    *s = *s * 1664525u + 1013904223u;
    return (double)(*s >> 8) / 16777216.0;
}

static int run(oracle_desc* d, int nsteps, unsigned seed) {
    const long ncell = d->n[0] * d->n[1] * d->n[2];
    double* q = malloc(sizeof(double) * d->meqn * ncell);
    double* aux = d->has_aux ? malloc(sizeof(double) * 2 * ncell) : NULL;
    double* dts = malloc(sizeof(double) * (2 * nsteps + 64));
    int* acc = malloc(sizeof(int) * (2 * nsteps + 64));
    for (long i = 0; i < ncell; ++i) {
        if (d->system == ORC_SHALLOW_WATER) {
            q[i] = 0.5 + urand(&seed);
            q[ncell + i] = 0.4 * (urand(&seed) - 0.5);
            q[2 * ncell + i] = 0.4 * (urand(&seed) - 0.5);
        } else {
            for (int m = 0; m < d->meqn; ++m) q[m * ncell + i] = urand(&seed) - 0.5;
        }
        if (aux) {
            aux[i] = 0.5 + urand(&seed);
            aux[ncell + i] = 0.5 + urand(&seed);
        }
    }
    double t = 0, smax[3];
    long nrej = 0;
    int rc = oracle_speeds(d, q, aux, smax);
    if (!rc) rc = oracle_advance(d, q, aux, nsteps, 0.0, 0.9, 1.0, INFINITY, &t, &nrej, dts, acc, 2 * nsteps + 64);
    for (int dir = 0; dir < d->ndim && !rc; ++dir) {
        double* out = malloc(sizeof(double) * d->meqn * ncell);
        double sm = 0;
        rc = oracle_sweep(d, q, aux, dir, 1e-3, out, &sm);
        free(out);
    }
    free(q);
    free(aux);
    free(dts);
    free(acc);
    return rc;
}

int main(void) {
    const int lims[] = {ORC_LIM_MC, ORC_LIM_NONE, ORC_FIRST_ORDER, ORC_LIM_MINMOD, ORC_LIM_SUPERBEE,
                        ORC_LIM_VANLEER};
    int failures = 0, runs = 0;
    for (int sys = 0; sys < 3; ++sys)
        for (int ndim = 2; ndim <= 3; ++ndim) {
            if (sys == ORC_SHALLOW_WATER && ndim == 3) continue;
            for (int bc = 0; bc < 3; ++bc)
                for (int li = 0; li < 6; ++li)
                    for (int split = 0; split < 2; ++split) {
                        oracle_desc d;
                        memset(&d, 0, sizeof d);
                        d.ndim = ndim;
                        d.n[0] = 13 + bc;
                        d.n[1] = 7 + li;
                        d.n[2] = ndim == 3 ? 5 : 1;
                        for (int k = 0; k < 3; ++k) {
                            d.lower[k] = 0;
                            d.upper[k] = 1.0 + 0.1 * k;
                            d.bc_lo[k] = (bc + k) % 3;
                            d.bc_hi[k] = (bc + 2 * k + 1) % 3;
                        }
                        d.system = sys;
                        d.meqn = sys == ORC_ACOUSTICS ? 1 + ndim : (sys == ORC_SHALLOW_WATER ? 3 : 1);
                        d.limiter = lims[li];
                        d.efix = 1;
                        d.has_aux = sys == ORC_ACOUSTICS && bc == 1;
                        d.rho = 1.3;
                        d.bulk = 2.1;
                        d.grav = 1.0;
                        d.splitting = split;
                        d.coef[0] = 1.0;
                        d.coef[1] = -0.5;
                        d.coef[2] = 0.75;
                        const int rc = run(&d, 6, 1234u + (unsigned)(runs * 7919));
                        ++runs;
                        if (rc) {
                            fprintf(stderr, "oracle error %d: system %d ndim %d bc %d limiter %d split %d\n", rc,
                                    sys, ndim, bc, li, split);
                            ++failures;
                        }
                    }
        }
    /* single interfaces, including a zero-depth middle state input */
    double W[9], s[3], am[3], ap[3];
    const double ql[3] = {1.0, -6.0, 2.0}, qr[3] = {49.0, -294.0, 49.0};
    failures += oracle_riemann_sw(ql, qr, 1.0, 1, 1, W, s, am, ap) != 0;
    const double bad[3] = {0.0, 1.0, 0.0};
    failures += oracle_riemann_sw(bad, qr, 1.0, 1, 1, W, s, am, ap) != 5;
    printf("%d oracle runs, %d failures\n", runs, failures);
    return failures ? 1 : 0;
}
