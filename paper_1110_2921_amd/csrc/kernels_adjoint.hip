// Discrete adjoint of the FMM evaluation (transposed pipeline).
//
// For a cotangent ubar of the velocity, the strength gradient is
//   alpha_bar = P2P^T ubar + P2M^T M2M^T (lattice^T) M2L^T L2L^T L2P^T ubar
// and the position gradient collects the derivatives of every place a
// position enters: the target of L2P and P2P (J ubar), the source of P2P
// (the near gradient of the field of strengths ubar, contracted with alpha)
// and the source of P2M (the gradient of the multipole basis, weighted by the
// multipole adjoint).  P2P^T is the P2P kernel itself with ubar as strengths
// (the pair kernel K(r) satisfies K(r)^T = K(-r)); M2L^T, L2L^T and M2M^T reuse
// the MFMA translation kernel with transposed operators.  This file holds the
// per-leaf L2P^T and P2M^T kernels and the final combination.
#include "device_harmonics.h"

namespace vmfmm {

namespace {

using dev::for_each_harmonic;
using dev::PartOf;
using dev::Tab;

// L2P^T: V[b][s] = sum_i ubar_{i,b} c_s(X_i) (degree < p), lam_bar = su * T V.
// PT > 0 fixes the degree at compile time (the harmonic recurrence may then
// unroll with its table offsets folded); PT = 0 takes it from p_arg.
template <typename T, int PT>
__global__ void __launch_bounds__(64) k_l2p_adj(const typename PartOf<T>::type *__restrict__ parts,
                                                const int32_t *__restrict__ start, const int32_t *__restrict__ perm,
                                                int n, const double *__restrict__ ubar, int p_arg, int kp, T inv_w,
                                                T su, DevTables tab, const int32_t *__restrict__ t_idx,
                                                const T *__restrict__ t_w, int width, int chunk,
                                                T *__restrict__ lbar) {
    extern __shared__ unsigned char smem_raw[];
    const int p = PT > 0 ? PT : p_arg;
    const int nu = p * p, C = (p + 1) * (p + 1);
    T *cv = reinterpret_cast<T *>(smem_raw);   // [chunk][nu]
    T *ub = cv + size_t(chunk) * nu;           // [chunk][3]
    T *V = ub + size_t(chunk) * 3;             // [3][nu]
    const int leaf = blockIdx.x, lane = threadIdx.x;
    const int s0 = start[leaf], cnt = start[leaf + 1] - s0;
    constexpr int MAXS = 7;   // ceil(400 / 64)
    T acc[3][MAXS];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int t = 0; t < MAXS; ++t) acc[c][t] = T(0);
    const T *c1 = Tab<T>::c1(tab), *c2 = Tab<T>::c2(tab), *dg = Tab<T>::dg(tab);
    for (int base = 0; base < cnt; base += chunk) {
        const int nj = min(chunk, cnt - base);
        if (lane < nj) {
            const int gi = s0 + base + lane;
            const auto q = parts[gi];
            T *row = cv + size_t(lane) * nu;
            for_each_harmonic<T>(T(q.dx) * inv_w, T(q.dy) * inv_w, T(q.dz) * inv_w, p - 1, c1, c2, dg,
                                 [&](int nn, int m, T re, T nim) {
                                     if (m == 0) {
                                         row[nn * nn] = re;
                                     } else {
                                         row[nn * nn + 2 * m - 1] = re;
                                         row[nn * nn + 2 * m] = nim;
                                     }
                                 });
            const int oi = perm[gi];
            for (int b = 0; b < 3; ++b) ub[lane * 3 + b] = T(ubar[size_t(b) * n + oi]);
        }
        __syncthreads();
        for (int j = 0; j < nj; ++j) {
            const T u0 = ub[j * 3 + 0], u1 = ub[j * 3 + 1], u2 = ub[j * 3 + 2];
            const T *row = cv + size_t(j) * nu;
#pragma unroll
            for (int t = 0; t < MAXS; ++t) {
                const int s = lane + 64 * t;
                if (s < nu) {
                    const T v = row[s];
                    acc[0][t] += u0 * v;
                    acc[1][t] += u1 * v;
                    acc[2][t] += u2 * v;
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int t = 0; t < MAXS; ++t) {
            const int s = lane + 64 * t;
            if (s < nu) V[b * nu + s] = acc[b][t];
        }
    __syncthreads();
    T *dst = lbar + size_t(leaf) * 3 * kp;
    for (int j = lane; j < 3 * kp; j += 64) {
        const int c = j / kp, t = j - c * kp;
        T v = T(0);
        if (t < C) {
            const int r = c * C + t;
            for (int e = 0; e < width; ++e) v += t_w[size_t(r) * width + e] * V[t_idx[size_t(r) * width + e]];
            v *= su;
        }
        dst[j] = v;
    }
}

// P2M^T and the source-position term of P2M: per particle
//   alpha_far[c] = F_c(Y),  x_P2M[a] = (1/w) sum_c alpha_c dF_c/dY_a,  F_c = sum_s Mbar[c][s] c_s(Y).
// Output in sorted order: adj[0..2][n] alpha_far, adj[3..5][n] x_P2M.
template <typename T>
__global__ void __launch_bounds__(64) k_p2m_adj(const typename PartOf<T>::type *__restrict__ parts,
                                                const int32_t *__restrict__ start, int n, int p, int kp, T inv_w,
                                                DevTables tab, const int32_t *__restrict__ g_idx,
                                                const T *__restrict__ g_w, int width, const T *__restrict__ mbar,
                                                double *__restrict__ adj) {
    extern __shared__ unsigned char smem_raw[];
    const int nu = p * p, C = (p + 1) * (p + 1);
    T *mb = reinterpret_cast<T *>(smem_raw);   // [3][C]
    T *g3 = mb + 3 * C;                         // [nu][9]: (c, a)
    const int leaf = blockIdx.x, lane = threadIdx.x;
    const int s0 = start[leaf], cnt = start[leaf + 1] - s0;
    if (cnt == 0) return;
    const T *src = mbar + size_t(leaf) * 3 * kp;
    for (int i = lane; i < 3 * C; i += 64) mb[i] = src[(i / C) * kp + (i % C)];
    __syncthreads();
    for (int r = lane; r < 3 * nu; r += 64) {     // r = a * nu + s
        const int a = r / nu, s = r - a * nu;
        for (int c = 0; c < 3; ++c) {
            T v = T(0);
            for (int e = 0; e < width; ++e) v += g_w[size_t(r) * width + e] * mb[c * C + g_idx[size_t(r) * width + e]];
            g3[s * 9 + c * 3 + a] = v;
        }
    }
    __syncthreads();
    const T *c1 = Tab<T>::c1(tab), *c2 = Tab<T>::c2(tab), *dg = Tab<T>::dg(tab);
    for (int base = 0; base < cnt; base += 64) {
        const int i = base + lane;
        if (i >= cnt) break;
        const auto q = parts[s0 + i];
        T ab[3] = {T(0), T(0), T(0)};
        T gF[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) gF[k] = T(0);
        for_each_harmonic<T>(T(q.dx) * inv_w, T(q.dy) * inv_w, T(q.dz) * inv_w, p, c1, c2, dg,
                             [&](int nn, int m, T re, T nim) {
                                 const int sr = m == 0 ? nn * nn : nn * nn + 2 * m - 1;
#pragma unroll
                                 for (int c = 0; c < 3; ++c) {
                                     ab[c] += mb[c * C + sr] * re;
                                     if (m > 0) ab[c] += mb[c * C + sr + 1] * nim;
                                 }
                                 if (nn < p) {
                                     const T *gr = g3 + sr * 9;
#pragma unroll
                                     for (int k = 0; k < 9; ++k) gF[k] += gr[k] * re;
                                     if (m > 0) {
#pragma unroll
                                         for (int k = 0; k < 9; ++k) gF[k] += gr[9 + k] * nim;
                                     }
                                 }
                             });
        const size_t gi = size_t(s0) + i;
        const double al[3] = {double(q.ax), double(q.ay), double(q.az)};
        for (int c = 0; c < 3; ++c) adj[size_t(c) * n + gi] = double(ab[c]);
        for (int a = 0; a < 3; ++a) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += al[c] * double(gF[c * 3 + a]);
            adj[size_t(3 + a) * n + gi] = s * double(inv_w);
        }
    }
}

// Sorted particle records with the strengths replaced by ubar.
template <typename P>
__global__ void __launch_bounds__(256) k_parts_with(int n, const P *__restrict__ in, const int32_t *__restrict__ perm,
                                                    const double *__restrict__ ubar, P *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    P r = in[i];
    const int oi = perm[i];
    r.ax = decltype(r.ax)(ubar[oi]);
    r.ay = decltype(r.ay)(ubar[size_t(n) + oi]);
    r.az = decltype(r.az)(ubar[2 * size_t(n) + oi]);
    out[i] = r;
}

// alpha_bar = v + alpha_far; x_bar = J ubar + Jv alpha + x_P2M (caller order).
__global__ void __launch_bounds__(256) k_adj_combine(int n, const int32_t *__restrict__ perm,
                                                     const double *__restrict__ ubar, const double *__restrict__ alpha,
                                                     const double *__restrict__ J, const double *__restrict__ v,
                                                     const double *__restrict__ Jv, const double *__restrict__ adj,
                                                     double *__restrict__ xbar, double *__restrict__ abar) {
    const int gi = blockIdx.x * blockDim.x + threadIdx.x;
    if (gi >= n) return;
    const int oi = perm[gi];
    if (abar)
        for (int c = 0; c < 3; ++c)
            abar[size_t(c) * n + oi] = v[size_t(c) * n + oi] + (adj ? adj[size_t(c) * n + gi] : 0.0);
    if (xbar) {
        double ub[3], al[3];
        for (int b = 0; b < 3; ++b) {
            ub[b] = ubar[size_t(b) * n + oi];
            al[b] = alpha[size_t(b) * n + oi];
        }
        for (int a = 0; a < 3; ++a) {
            double s = adj ? adj[size_t(3 + a) * n + gi] : 0.0;
            for (int b = 0; b < 3; ++b)
                s += J[size_t(3 * a + b) * n + oi] * ub[b] + Jv[size_t(3 * a + b) * n + oi] * al[b];
            xbar[size_t(a) * n + oi] = s;
        }
    }
}

inline int blocks(int n, int t) { return (n + t - 1) / t; }

}  // namespace

template <typename T>
hipError_t launch_l2p_adj(hipStream_t s, int nleaf, int n, const void *parts, const int32_t *start,
                          const int32_t *perm, const double *ubar, int p, int kp, double inv_w, double w,
                          const DevTables &tab, const int32_t *t_idx, const T *t_w, int width, T *lbar) {
    const int nu = p * p;
    int chunk = int(40960 / (sizeof(T) * (nu + 3)));
    if (chunk > 64) chunk = 64;
    if (chunk < 1) chunk = 1;
    const size_t smem = sizeof(T) * (size_t(chunk) * (nu + 3) + 3 * size_t(nu));
    const double su = 1.0 / (12.566370614359172953850573533118 * w * w);
    const auto *pp = (const typename PartOf<T>::type *)parts;
    switch (p) {   // the workloads' degrees at compile time, any other at run time
    case 6: hipLaunchKernelGGL((k_l2p_adj<T, 6>), dim3(nleaf), dim3(64), smem, s, pp, start, perm, n, ubar, p, kp, T(inv_w), T(su), tab, t_idx, t_w, width, chunk, lbar); break;
    case 8: hipLaunchKernelGGL((k_l2p_adj<T, 8>), dim3(nleaf), dim3(64), smem, s, pp, start, perm, n, ubar, p, kp, T(inv_w), T(su), tab, t_idx, t_w, width, chunk, lbar); break;
    case 10: hipLaunchKernelGGL((k_l2p_adj<T, 10>), dim3(nleaf), dim3(64), smem, s, pp, start, perm, n, ubar, p, kp, T(inv_w), T(su), tab, t_idx, t_w, width, chunk, lbar); break;
    default: hipLaunchKernelGGL((k_l2p_adj<T, 0>), dim3(nleaf), dim3(64), smem, s, pp, start, perm, n, ubar, p, kp, T(inv_w), T(su), tab, t_idx, t_w, width, chunk, lbar);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_p2m_adj(hipStream_t s, int nleaf, int n, const void *parts, const int32_t *start, int p, int kp,
                          double inv_w, const DevTables &tab, const int32_t *g_idx, const T *g_w, int width,
                          const T *mbar, double *adj) {
    const int nu = p * p, C = (p + 1) * (p + 1);
    const size_t smem = sizeof(T) * (3 * size_t(C) + 9 * size_t(nu) + 9);
    hipLaunchKernelGGL(k_p2m_adj<T>, dim3(nleaf), dim3(64), smem, s, (const typename PartOf<T>::type *)parts,
                       start, n, p, kp, T(inv_w), tab, g_idx, g_w, width, mbar, adj);
    return hipGetLastError();
}

hipError_t launch_parts_with64(hipStream_t s, int n, const Part64 *in, const int32_t *perm, const double *ubar,
                               Part64 *out) {
    hipLaunchKernelGGL(k_parts_with<Part64>, dim3(blocks(n, 256)), dim3(256), 0, s, n, in, perm, ubar, out);
    return hipGetLastError();
}

hipError_t launch_parts_with32(hipStream_t s, int n, const Part32 *in, const int32_t *perm, const double *ubar,
                               Part32 *out) {
    hipLaunchKernelGGL(k_parts_with<Part32>, dim3(blocks(n, 256)), dim3(256), 0, s, n, in, perm, ubar, out);
    return hipGetLastError();
}

hipError_t launch_adj_combine(hipStream_t s, int n, const int32_t *perm, const double *ubar, const double *alpha,
                              const double *J, const double *v, const double *Jv, const double *adj, double *xbar,
                              double *abar) {
    hipLaunchKernelGGL(k_adj_combine, dim3(blocks(n, 256)), dim3(256), 0, s, n, perm, ubar, alpha, J, v, Jv, adj,
                       xbar, abar);
    return hipGetLastError();
}

#define VM_INST(T)                                                                                              \
    template hipError_t launch_l2p_adj<T>(hipStream_t, int, int, const void *, const int32_t *, const int32_t *, \
                                          const double *, int, int, double, double, const DevTables &,           \
                                          const int32_t *, const T *, int, T *);                                 \
    template hipError_t launch_p2m_adj<T>(hipStream_t, int, int, const void *, const int32_t *, int, int,        \
                                          double, const DevTables &, const int32_t *, const T *, int, const T *, \
                                          double *);
VM_INST(double)
VM_INST(float)
#undef VM_INST

}  // namespace vmfmm
