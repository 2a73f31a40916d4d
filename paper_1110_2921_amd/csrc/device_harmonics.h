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

}  // namespace dev
}  // namespace vmfmm
