/*
 * Test infrastructure: a driver of the oracle's direct sum (direct.c) for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer.  It runs the
 * sum over the argument shapes the tests use -- free space and image blocks
 * K = 1..2, with and without leaf coordinates, coincident particles (r = 0),
 * empty target or source sets -- and checks what holds for any input: the
 * results are finite, a lone particle induces no velocity on itself, and the
 * velocity of two particles is antisymmetric in their exchange.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_direct(int64_t nt, const double *xt, int64_t ns, const double *xs, const double *as, double sigma,
                  double box_len, int K, const int32_t *ct, const int32_t *cs, int level, double *u, double *J);

static double urand(unsigned *s) {
    *s = *s * 1664525u + 1013904223u;
    return (double)(*s >> 8) / 16777216.0;
}

static int finite_all(const double *v, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

int main(void) {
    unsigned seed = 12345u;
    const double L = 6.283185307179586;
    int failures = 0;
    for (int K = 0; K <= 2; ++K)
        for (int with_cells = 0; with_cells <= 1; ++with_cells)
            for (int nt = 0; nt <= 9; nt += 3)
                for (int ns = 0; ns <= 17; ns += 17) {
                    double *xt = malloc(sizeof(double) * 3 * (nt + 1)), *xs = malloc(sizeof(double) * 3 * (ns + 1));
                    double *as = malloc(sizeof(double) * 3 * (ns + 1));
                    double *u = malloc(sizeof(double) * 3 * (nt + 1)), *J = malloc(sizeof(double) * 9 * (nt + 1));
                    int32_t *ct = malloc(sizeof(int32_t) * 3 * (nt + 1)), *cs = malloc(sizeof(int32_t) * 3 * (ns + 1));
                    for (int i = 0; i < 3 * ns; ++i) {
                        xs[i] = L * urand(&seed);
                        as[i] = urand(&seed) - 0.5;
                        cs[i] = (int32_t)(xs[i] / L * 4.0);
                    }
                    for (int i = 0; i < 3 * nt; ++i) {
                        /* every third target sits on a source: r = 0 */
                        xt[i] = (ns > 0 && (i / 3) % 3 == 0) ? xs[i % (3 * ns)] : L * urand(&seed);
                        ct[i] = (int32_t)(xt[i] / L * 4.0);
                    }
                    const int rc = oracle_direct(nt, xt, ns, xs, as, 0.3, L, K, with_cells ? ct : NULL,
                                                 with_cells ? cs : NULL, 2, u, J);
                    if (rc != 0 || !finite_all(u, 3 * (int64_t)nt) || !finite_all(J, 9 * (int64_t)nt)) {
                        printf("FAIL K=%d cells=%d nt=%d ns=%d rc=%d\n", K, with_cells, nt, ns, rc);
                        ++failures;
                    }
                    free(xt); free(xs); free(as); free(u); free(J); free(ct); free(cs);
                }
    /* a lone particle: no velocity on itself */
    {
        const double x[3] = {1.0, 2.0, 3.0}, a[3] = {0.3, -0.2, 0.5};
        double u[3], J[9];
        oracle_direct(1, x, 1, x, a, 0.2, L, 0, NULL, NULL, 0, u, J);
        if (u[0] != 0.0 || u[1] != 0.0 || u[2] != 0.0) {
            printf("FAIL self velocity\n");
            ++failures;
        }
    }
    /* exchange antisymmetry: with equal strengths the velocity of a on b is minus that of b on a */
    {
        const double xa[3] = {1.0, 2.0, 3.0}, xb[3] = {1.4, 1.7, 3.2}, al[3] = {0.3, -0.2, 0.5};
        double ua[3], ub[3], J[9];
        oracle_direct(1, xa, 1, xb, al, 0.2, L, 0, NULL, NULL, 0, ua, J);
        oracle_direct(1, xb, 1, xa, al, 0.2, L, 0, NULL, NULL, 0, ub, J);
        for (int d = 0; d < 3; ++d)
            if (fabs(ua[d] + ub[d]) > 1e-15 * (fabs(ua[d]) + 1e-300)) {
                printf("FAIL antisymmetry %d\n", d);
                ++failures;
            }
    }
    /* invalid arguments are rejected */
    if (oracle_direct(1, NULL, 1, NULL, NULL, -1.0, L, 0, NULL, NULL, 0, NULL, NULL) == 0) {
        printf("FAIL negative sigma accepted\n");
        ++failures;
    }
    printf(failures ? "FAILED %d\n" : "OK\n", failures);
    return failures ? 1 : 0;
}
