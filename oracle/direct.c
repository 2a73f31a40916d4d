/*
 * Test infrastructure: plain CPU oracle, not part of the product path.
 *
 * Direct O(N_t * N_s * N_img) sum of the Gaussian-regularised Biot-Savart
 * velocity and its gradient, in double precision, written from the paper's
 * definitions:
 *   - blob vorticity omega = sum_j gamma_j zeta_sigma (eqs. 3-4),
 *   - velocity u_i = sum_j gamma_j x grad(G g_sigma) with G = 1/(4 pi r) and
 *     the cutoff g_sigma = erf(s) - (2/sqrt(pi)) s exp(-s^2), s = r/(sqrt(2) sigma)
 *     (eqs. 5-6); with the right-hand rule this reads
 *         u_i = 1/(4 pi) sum_j q(r) alpha_j x r,   r = x_i - x_j,  q = g/r^3,
 *   - gradient J[a][b] = d u_b / d x_a (the tensor the stretching term of
 *     eq. 8 contracts):
 *         J[a][b] = 1/(4 pi) sum_j [ q eps_{bca} alpha_c + (q'/r) r_a (alpha_j x r)_b ],
 *     q'/r = (sqrt(2/pi) sigma^-3 exp(-rho^2/2) - 3 q) / r^2,  rho = r/sigma.
 * Periodic sums run over the cubic image block S_K = {-R..R}^3,
 * R = (3^K - 1)/2 (K = 3 gives the paper's 27^3 images, Sec. 4.1).
 *
 * With leaf coordinates supplied, pairs whose leaves are not adjacent (with
 * the image shift applied) use g = 1: the far field of the FMM drops the
 * cutoff (Sec. 3.1, below eqs. 12-13), so this is the value the FMM
 * converges to as p grows.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define INV4PI 0.079577471545947667884441881686257181
#define SQRT_2_OVER_PI 0.79788456080286535587989211986876373

/* q(r) and (dq/dr)/r for r > 0, both exact in double precision.  For small
 * rho the closed form cancels, so the Taylor series of g (integral of the
 * Gaussian mass, g'(rho) = sqrt(2/pi) rho^2 exp(-rho^2/2)) is summed. */
static void cutoff_q(double r2, double sigma, double *q, double *dq_r)
{
    const double s2 = sigma * sigma;
    const double rho2 = r2 / s2;
    const double is3 = 1.0 / (s2 * sigma);
    if (rho2 < 0.0625) {
        /* g/rho^3 = sqrt(2/pi) sum_n (-1)^n rho^{2n} / (2^n n! (2n+3))
         * (g/rho^3)' / rho = sqrt(2/pi) sum_{n>=1} (-1)^n 2n rho^{2n-2} / (2^n n! (2n+3)) */
        double h0 = 0.0, h1 = 0.0, term = 1.0;   /* term = (-rho^2/2)^n / n! */
        for (int n = 0; n < 14; ++n) {
            h0 += term / (2.0 * n + 3.0);
            term *= -0.5 * rho2 / (n + 1.0);
        }
        term = -0.5;                              /* n = 1: (-1/2)^1/1! times 2n/rho^2 factor below */
        for (int n = 1; n < 14; ++n) {
            h1 += term * 2.0 * n / (2.0 * n + 3.0);
            term *= -0.5 * rho2 / (n + 1.0);
        }
        *q = SQRT_2_OVER_PI * h0 * is3;
        *dq_r = SQRT_2_OVER_PI * h1 * is3 / s2;
        return;
    }
    const double r = sqrt(r2);
    const double rho = r / sigma;
    const double e = exp(-0.5 * rho2);
    const double g = erf(rho / sqrt(2.0)) - SQRT_2_OVER_PI * rho * e;
    *q = g / (r2 * r);
    *dq_r = (SQRT_2_OVER_PI * is3 * e - 3.0 * (*q)) / r2;
}

/*
 * xt: targets (nt, 3); xs, as: sources (ns, 3); all row-major.
 * K: 0 free space, K >= 1 periodic image block 3^K per side of period box_len.
 * ct, cs: leaf coordinates (n, 3) at leaf level `level` (2^level leaves per
 *   side), or NULL for the exact kernel everywhere.
 * u: (nt, 3) out; J: (nt, 9) out (J[3a+b] = d u_b / d x_a), may be NULL.
 * Returns 0, or -1 on bad arguments.
 */
int oracle_direct(int64_t nt, const double *xt, int64_t ns, const double *xs,
                  const double *as, double sigma, double box_len, int K,
                  const int32_t *ct, const int32_t *cs, int level,
                  double *u, double *J)
{
    if (nt < 0 || ns < 0 || sigma <= 0.0 || K < 0 || K > 4) return -1;
    int R = 0;
    for (int k = 0; k < K; ++k) R = 3 * R + 1;
    const int64_t side = (int64_t)1 << (level < 0 ? 0 : level);

#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nt; ++i) {
        double ui[3] = {0, 0, 0};
        double Ji[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int nx = -R; nx <= R; ++nx)
        for (int ny = -R; ny <= R; ++ny)
        for (int nz = -R; nz <= R; ++nz) {
            const double sh[3] = {nx * box_len, ny * box_len, nz * box_len};
            const int nimg[3] = {nx, ny, nz};
            for (int64_t j = 0; j < ns; ++j) {
                double r[3];
                for (int d = 0; d < 3; ++d) r[d] = xt[3 * i + d] - xs[3 * j + d] - sh[d];
                const double r2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
                const double *a = as + 3 * j;
                int exact = 1;
                if (ct && cs) {
                    int64_t cheb = 0;
                    for (int d = 0; d < 3; ++d) {
                        int64_t dd = (int64_t)ct[3 * i + d] - ((int64_t)cs[3 * j + d] + nimg[d] * side);
                        if (dd < 0) dd = -dd;
                        if (dd > cheb) cheb = dd;
                    }
                    exact = cheb <= 1;
                }
                double q, dq_r;
                if (!exact) {
                    const double ir2 = 1.0 / r2;
                    q = ir2 / sqrt(r2);
                    dq_r = -3.0 * q * ir2;
                } else if (r2 == 0.0) {
                    /* r -> 0 limit: q(0) = sqrt(2/pi) / (3 sigma^3); the rank-one term vanishes */
                    q = SQRT_2_OVER_PI / (3.0 * sigma * sigma * sigma);
                    dq_r = 0.0;
                } else {
                    cutoff_q(r2, sigma, &q, &dq_r);
                }
                const double c[3] = {a[1] * r[2] - a[2] * r[1],
                                     a[2] * r[0] - a[0] * r[2],
                                     a[0] * r[1] - a[1] * r[0]};
                for (int b = 0; b < 3; ++b) ui[b] += q * c[b];
                /* antisymmetric part: J[a][b] += q eps_{abc} alpha_c */
                Ji[0 * 3 + 1] += q * a[2];
                Ji[1 * 3 + 0] -= q * a[2];
                Ji[1 * 3 + 2] += q * a[0];
                Ji[2 * 3 + 1] -= q * a[0];
                Ji[2 * 3 + 0] += q * a[1];
                Ji[0 * 3 + 2] -= q * a[1];
                for (int aa = 0; aa < 3; ++aa)
                    for (int b = 0; b < 3; ++b) Ji[3 * aa + b] += dq_r * r[aa] * c[b];
            }
        }
        for (int b = 0; b < 3; ++b) u[3 * i + b] = INV4PI * ui[b];
        if (J)
            for (int k = 0; k < 9; ++k) J[9 * i + k] = INV4PI * Ji[k];
    }
    return 0;
}
