// Device helpers shared by the expansion kernels: precision-dispatched table
// access and the balanced regular solid harmonics by recurrence.
#pragma once

#include "kernels.h"

namespace vmfmm {
namespace dev {

template <typename T> struct Tab;
template <> struct Tab<double> {
    static __device__ const double *c1(const DevTables &t) { return t.c1_64; }
    static __device__ const double *c2(const DevTables &t) { return t.c2_64; }
    static __device__ const double *dg(const DevTables &t) { return t.diag_64; }
    static __device__ const double *w(const DevTables &t) { return t.l2p_w64; }
};
template <> struct Tab<float> {
    static __device__ const float *c1(const DevTables &t) { return t.c1_32; }
    static __device__ const float *c2(const DevTables &t) { return t.c2_32; }
    static __device__ const float *dg(const DevTables &t) { return t.diag_32; }
    static __device__ const float *w(const DevTables &t) { return t.l2p_w32; }
};

template <typename T> struct PartOf;
template <> struct PartOf<double> { using type = Part64; };
template <> struct PartOf<float> { using type = Part32; };

// Visits c(X) = [Rb_n^0, Re Rb_n^m, -Im Rb_n^m] for all n <= deg, m <= n, in
// the order m outer, n inner: f(n, m, re, negim).
template <typename T, typename F>
__device__ __forceinline__ void for_each_harmonic(T X, T Y, T Z, int deg, const T *__restrict__ c1,
                                                  const T *__restrict__ c2, const T *__restrict__ dg, F &&f) {
    const T r2 = X * X + Y * Y + Z * Z;
    T dre = T(1), dim = T(0);
    for (int m = 0; m <= deg; ++m) {
        if (m > 0) {
            // Rb_m^m = -(X + iY) diag[m] Rb_{m-1}^{m-1}
            const T s = -dg[m];
            const T nre = s * (X * dre - Y * dim);
            const T nim = s * (X * dim + Y * dre);
            dre = nre;
            dim = nim;
        }
        T are = dre, aim = dim, bre = T(0), bim = T(0);
        f(m, m, are, -aim);
        for (int n = m + 1; n <= deg; ++n) {
            const int e = n * (n + 1) / 2 + m;
            const T k1 = c1[e] * Z, k2 = c2[e] * r2;
            const T cre = k1 * are - k2 * bre;
            const T cim = k1 * aim - k2 * bim;
            bre = are; bim = aim;
            are = cre; aim = cim;
            f(n, m, are, -aim);
        }
    }
}

// Balanced irregular solid harmonics Ib_n^m(X) for n <= deg, m <= n, by the
// recurrence the regular ones use, divided by r^2 at each step:
//   Ib_0^0 = 1/r,  Ib_m^m = -(X + iY) diag[m] Ib_{m-1}^{m-1} / r^2,
//   Ib_n^m = (c1 Z Ib_{n-1}^m - c2 Ib_{n-2}^m) / r^2   (n > m),
// with the regular harmonics' constants (c1, c2, diag of a table of degree
// >= deg).  Written packed, [Ib_n^0, Re Ib_n^m, sgn Im Ib_n^m] at
// n^2, n^2 + 2m - 1, n^2 + 2m, with sgn = +1 or -1 (the conjugate).
template <typename T>
__device__ __forceinline__ void irregular_packed(T X, T Y, T Z, int deg, const T *__restrict__ c1,
                                                 const T *__restrict__ c2, const T *__restrict__ dg, T sgn,
                                                 T *__restrict__ out, int stride) {
    const T r2 = X * X + Y * Y + Z * Z;
    const T ir2 = T(1) / r2;
    T dre = sqrt(ir2), dim = T(0);
    for (int m = 0; m <= deg; ++m) {
        if (m > 0) {
            const T s = -dg[m] * ir2;
            const T nre = s * (X * dre - Y * dim);
            const T nim = s * (X * dim + Y * dre);
            dre = nre;
            dim = nim;
        }
        T are = dre, aim = dim, bre = T(0), bim = T(0);
        for (int n = m; n <= deg; ++n) {
            if (n > m) {
                const int e = n * (n + 1) / 2 + m;
                const T k1 = c1[e] * Z, k2 = c2[e];
                const T cre = (k1 * are - k2 * bre) * ir2;
                const T cim = (k1 * aim - k2 * bim) * ir2;
                bre = are; bim = aim;
                are = cre; aim = cim;
            }
            if (m == 0) {
                out[(n * n) * stride] = are;
            } else {
                out[(n * n + 2 * m - 1) * stride] = are;
                out[(n * n + 2 * m) * stride] = sgn * aim;
            }
        }
    }
}

// The orders m = m0, m0 + mstep, ... of irregular_packed only (the diagonal
// chain runs through every order; the n-chains of the other orders are skipped):
// lanes that share a point can split its harmonics between them.
template <typename T>
__device__ __forceinline__ void irregular_packed_orders(T X, T Y, T Z, int deg, const T *__restrict__ c1,
                                                        const T *__restrict__ c2, const T *__restrict__ dg, T sgn,
                                                        int m0, int mstep, T *__restrict__ out, int stride) {
    const T r2 = X * X + Y * Y + Z * Z;
    const T ir2 = T(1) / r2;
    T dre = sqrt(ir2), dim = T(0);
    for (int m = 0; m <= deg; ++m) {
        if (m > 0) {
            const T s = -dg[m] * ir2;
            const T nre = s * (X * dre - Y * dim);
            const T nim = s * (X * dim + Y * dre);
            dre = nre;
            dim = nim;
        }
        if (m < m0 || (m - m0) % mstep != 0) continue;
        T are = dre, aim = dim, bre = T(0), bim = T(0);
        for (int n = m; n <= deg; ++n) {
            if (n > m) {
                const int e = n * (n + 1) / 2 + m;
                const T k1 = c1[e] * Z, k2 = c2[e];
                const T cre = (k1 * are - k2 * bre) * ir2;
                const T cim = (k1 * aim - k2 * bim) * ir2;
                bre = are; bim = aim;
                are = cre; aim = cim;
            }
            if (m == 0) {
                out[(n * n) * stride] = are;
            } else {
                out[(n * n + 2 * m - 1) * stride] = are;
                out[(n * n + 2 * m) * stride] = sgn * aim;
            }
        }
    }
}

}  // namespace dev
}  // namespace vmfmm
