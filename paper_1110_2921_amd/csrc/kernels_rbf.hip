// RBF interpolation (Sec. 2): the Gaussian smoothing sums that form the
// matrix-vector product of the interpolation system, and the vector kernels
// of its GMRES iteration.
//
// Gaussian sums over the neighbour list of the tree: for a target in leaf c,
// every source in the 27 leaves c + d (periodic: wrapped, with the image
// shift), omega_i = (2 pi sigma^2)^(-3/2) sum_j gamma_j exp(-r_ij^2 / (2 sigma^2)).
// One wave per target leaf, one target per lane; the source records (position
// relative to the leaf centre, strength gamma in the a-fields) are read at
// wave-uniform addresses (scalar loads).  Vectors are in the sorted particle
// order, [3][n] FP64.
#include "kernels.h"

namespace vmfmm {

namespace {

__device__ __forceinline__ int leaf_coord(int k, int d, int level) {
    int c = 0;
    for (int b = 0; b < level; ++b) c |= ((k >> (3 * b + d)) & 1) << b;
    return c;
}

__device__ __forceinline__ int leaf_key(int cx, int cy, int cz, int level) {
    int k = 0;
    for (int b = 0; b < level; ++b)
        k |= (((cx >> b) & 1) << (3 * b)) | (((cy >> b) & 1) << (3 * b + 1)) | (((cz >> b) & 1) << (3 * b + 2));
    return k;
}

// Workgroup b runs leaf (b mod 8) nleaf/8 + b/8: workgroups go to the 8 XCDs
// round-robin, so each XCD takes one contiguous Morton range whose neighbour
// leaves its L2 shares.
__device__ __forceinline__ int gauss_leaf(int nleaf) {
    const int b = blockIdx.x;
    if (nleaf % 8 != 0) return b;
    return (b & 7) * (nleaf >> 3) + (b >> 3);
}

// One source against the lane's target: scaled coordinates, c = sqrt(log2(e)
// / (2 sigma^2)), so that exp(-r^2 / (2 sigma^2)) = 2^-(|c r|^2) and c r =
// c t - c s takes one FMA per axis.
template <typename T, typename P>
__device__ __forceinline__ void gauss_pair(const P &src, T ctx_, T cty, T ctz, T mc, T part[3]) {
    const T rx = fma(T(src.dx), mc, ctx_), ry = fma(T(src.dy), mc, cty), rz = fma(T(src.dz), mc, ctz);
    const T q = rx * rx + ry * ry + rz * rz;
    T e;
    if constexpr (sizeof(T) == 4) e = __builtin_amdgcn_exp2f(-q);
    else e = exp2(-q);
    part[0] = fma(T(src.ax), e, part[0]);
    part[1] = fma(T(src.ay), e, part[1]);
    part[2] = fma(T(src.az), e, part[2]);
}

// T: arithmetic of the pair (double: FP64 form; float: mixed form, FP32
// differences, exponential and per-source-leaf sums, added into FP64 sums).
template <typename T, typename P>
__global__ void __launch_bounds__(64) k_gauss(GaussArgs a, const P *__restrict__ parts) {
    const int leaf = gauss_leaf(a.nleaf), lane = threadIdx.x;
    const int s0 = a.tstart[leaf], cnt = a.tstart[leaf + 1] - s0;
    if (cnt == 0) return;
    const P *__restrict__ targets = static_cast<const P *>(a.tparts);
    const int side = 1 << a.level;
    const int cx = leaf_coord(leaf, 0, a.level), cy = leaf_coord(leaf, 1, a.level), cz = leaf_coord(leaf, 2, a.level);
    const size_t n = size_t(a.n);
    const double c64 = sqrt(0.5 * 1.4426950408889634074) / a.sigma;
    const T c = T(c64), mc = -c, cw = T(c64 * a.w);
    const double s2pi = 2.0 * 3.14159265358979323846 * a.sigma * a.sigma;
    const double norm = 1.0 / (s2pi * sqrt(s2pi));
    for (int base = 0; base < cnt; base += 64) {
        const int i = base + lane;
        const bool valid = i < cnt;
        const P me = targets[s0 + (valid ? i : 0)];
        const T mx = T(me.dx) * c, my = T(me.dy) * c, mz = T(me.dz) * c;
        double acc[3] = {0.0, 0.0, 0.0};
        for (int nb = 0; nb < 27; ++nb) {
            const int dx = nb % 3 - 1, dy = (nb / 3) % 3 - 1, dz = nb / 9 - 1;
            int nx = cx + dx, ny = cy + dy, nz = cz + dz;
            if (a.periodic) {
                nx = (nx + side) % side;
                ny = (ny + side) % side;
                nz = (nz + side) % side;
            } else if (nx < 0 || ny < 0 || nz < 0 || nx >= side || ny >= side || nz >= side) {
                continue;
            }
            const int nk = leaf_key(nx, ny, nz, a.level);
            const int js = a.start[nk], m = a.start[nk + 1] - js;
            if (m <= 0) continue;
            // c (x_i - x_j) = c (delta_i - d w) - c delta_j, d = source - target cell offset
            const T tx = mx - T(dx) * cw, ty = my - T(dy) * cw, tz = mz - T(dz) * cw;
            T part[3] = {T(0), T(0), T(0)};
            const P *src = parts + js;
            const P *const end4 = src + (m & ~3), *const end = src + m;
            for (; src != end4; src += 4) {
                const P s0_ = src[0], s1_ = src[1], s2_ = src[2], s3_ = src[3];
                gauss_pair(s0_, tx, ty, tz, mc, part);
                gauss_pair(s1_, tx, ty, tz, mc, part);
                gauss_pair(s2_, tx, ty, tz, mc, part);
                gauss_pair(s3_, tx, ty, tz, mc, part);
            }
            for (; src != end; ++src) gauss_pair(src[0], tx, ty, tz, mc, part);
            for (int q = 0; q < 3; ++q) acc[q] += double(part[q]);
        }
        if (valid)
            for (int q = 0; q < 3; ++q) a.out[q * n + s0 + i] = norm * acc[q];
    }
}

// parts[i].a = gamma[:][i] (sorted order): the strengths of the next product
template <typename P, typename S>
__global__ void __launch_bounds__(256) k_pack(int n, const double *__restrict__ gamma, P *__restrict__ parts) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const size_t m = size_t(n);
    parts[i].ax = S(gamma[i]);
    parts[i].ay = S(gamma[m + i]);
    parts[i].az = S(gamma[2 * m + i]);
}

// dst[c][i] = src[c][perm[i]] (caller order -> sorted order)
__global__ void __launch_bounds__(256) k_gather3(int n, const int32_t *__restrict__ perm,
                                                 const double *__restrict__ src, double *__restrict__ dst) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int j = perm[i];
    if (j < 0 || j >= n) return;   // never for a valid permutation
    for (int c = 0; c < 3; ++c) dst[size_t(c) * n + i] = src[size_t(c) * n + j];
}

// dst[c][perm[i]] = scale * src[c][i] (sorted order -> caller order)
__global__ void __launch_bounds__(256) k_scatter3(int n, const int32_t *__restrict__ perm,
                                                  const double *__restrict__ src, double scale,
                                                  double *__restrict__ dst) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int j = perm[i];
    if (j < 0 || j >= n) return;
    for (int c = 0; c < 3; ++c) dst[size_t(c) * n + j] = scale * src[size_t(c) * n + i];
}

// partial[(3 j + c) kRbfDotBlocks + block] = sum over the block's share of i
// of w[c][i] v_j[c][i], j < k, v_j = V + j ldv: grid-stride order, then a
// fixed tree over the workgroup.  Four Krylov vectors per pass over w.
__global__ void __launch_bounds__(256) k_multidot(int n, const double *__restrict__ w,
                                                  const double *__restrict__ V, int64_t ldv, int k,
                                                  double *__restrict__ partial) {
    __shared__ double red[4][4];
    const int tid = threadIdx.x;
    const size_t m = size_t(n);
    for (int c = 0; c < 3; ++c) {
        const double *wc = w + c * m;
        for (int j0 = 0; j0 < k; j0 += 4) {
            const int kk = k - j0 < 4 ? k - j0 : 4;
            double s[4] = {0.0, 0.0, 0.0, 0.0};
            for (int64_t i = int64_t(blockIdx.x) * 256 + tid; i < n; i += int64_t(kRbfDotBlocks) * 256) {
                const double wi = wc[i];
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (q < kk) s[q] = fma(wi, V[(j0 + q) * ldv + c * m + i], s[q]);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                for (int off = 32; off > 0; off >>= 1) s[q] += __shfl_xor(s[q], off);
                if ((tid & 63) == 0) red[q][tid >> 6] = s[q];
            }
            __syncthreads();
            if (tid < kk)
                partial[size_t(3 * (j0 + tid) + c) * kRbfDotBlocks + blockIdx.x] =
                    (red[tid][0] + red[tid][1]) + (red[tid][2] + red[tid][3]);
            __syncthreads();
        }
    }
}

// out[r] = sum_b partial[r kRbfDotBlocks + b] in a fixed order: one workgroup per r
__global__ void __launch_bounds__(256) k_dot_finish(const double *__restrict__ partial, double *__restrict__ out) {
    __shared__ double red[4];
    const int tid = threadIdx.x, r = blockIdx.x;
    double s = 0.0;
    for (int b = tid; b < kRbfDotBlocks; b += 256) s += partial[size_t(r) * kRbfDotBlocks + b];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
    if ((tid & 63) == 0) red[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) out[r] = (red[0] + red[1]) + (red[2] + red[3]);
}

// w[c][i] = alpha_c w[c][i] + sum_{j < k} c_{j,c} v_j[c][i]
__global__ void __launch_bounds__(256) k_multiaxpy(int n, double *__restrict__ w, const double *__restrict__ V,
                                                   int64_t ldv, int k, RbfCoefs cf) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const size_t m = size_t(n);
    for (int c = 0; c < 3; ++c) {
        double s = cf.alpha[c] * w[c * m + i];
        for (int j = 0; j < k; ++j) s = fma(cf.c[3 * j + c], V[j * ldv + c * m + i], s);
        w[c * m + i] = s;
    }
}

// Cell centres of the ng^3 lattice on the box: site k = (ix ng + iy) ng + iz
// at lo + (i + 1/2) h, written as [3][ng^3].
__global__ void __launch_bounds__(256) k_lattice_sites(int ng, double lo0, double lo1, double lo2, double h,
                                                       double *__restrict__ out) {
    const int n = ng * ng * ng;
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const int ix = k / (ng * ng), iy = (k / ng) % ng, iz = k % ng;
    const size_t m = size_t(n);
    out[k] = lo0 + (double(ix) + 0.5) * h;
    out[m + k] = lo1 + (double(iy) + 0.5) * h;
    out[2 * m + k] = lo2 + (double(iz) + 0.5) * h;
}

unsigned blocks256(int n) { return unsigned((n + 255) / 256); }

}  // namespace

hipError_t launch_gauss(hipStream_t s, const GaussArgs &a, const void *parts, int mixed) {
    if (mixed)
        hipLaunchKernelGGL((k_gauss<float, Part32>), dim3(a.nleaf), dim3(64), 0, s, a, (const Part32 *)parts);
    else
        hipLaunchKernelGGL((k_gauss<double, Part64>), dim3(a.nleaf), dim3(64), 0, s, a, (const Part64 *)parts);
    return hipGetLastError();
}

hipError_t launch_pack(hipStream_t s, int n, const double *gamma, void *parts, int mixed) {
    if (mixed)
        hipLaunchKernelGGL((k_pack<Part32, float>), dim3(blocks256(n)), dim3(256), 0, s, n, gamma, (Part32 *)parts);
    else
        hipLaunchKernelGGL((k_pack<Part64, double>), dim3(blocks256(n)), dim3(256), 0, s, n, gamma, (Part64 *)parts);
    return hipGetLastError();
}

hipError_t launch_lattice_sites(hipStream_t s, int ng, const double lo[3], double h, double *out) {
    const int n = ng * ng * ng;
    hipLaunchKernelGGL(k_lattice_sites, dim3(blocks256(n)), dim3(256), 0, s, ng, lo[0], lo[1], lo[2], h, out);
    return hipGetLastError();
}

hipError_t launch_gather3(hipStream_t s, int n, const int32_t *perm, const double *src, double *dst) {
    hipLaunchKernelGGL(k_gather3, dim3(blocks256(n)), dim3(256), 0, s, n, perm, src, dst);
    return hipGetLastError();
}

hipError_t launch_scatter3(hipStream_t s, int n, const int32_t *perm, const double *src, double scale, double *dst) {
    hipLaunchKernelGGL(k_scatter3, dim3(blocks256(n)), dim3(256), 0, s, n, perm, src, scale, dst);
    return hipGetLastError();
}

hipError_t launch_multidot(hipStream_t s, int n, const double *w, const double *V, int64_t ldv, int k,
                           double *partial, double *out) {
    hipLaunchKernelGGL(k_multidot, dim3(kRbfDotBlocks), dim3(256), 0, s, n, w, V, ldv, k, partial);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_dot_finish, dim3(unsigned(3 * k)), dim3(256), 0, s, partial, out);
    return hipGetLastError();
}

hipError_t launch_multiaxpy(hipStream_t s, int n, double *w, const double *V, int64_t ldv, int k,
                            const RbfCoefs &c) {
    hipLaunchKernelGGL(k_multiaxpy, dim3(blocks256(n)), dim3(256), 0, s, n, w, V, ldv, k, c);
    return hipGetLastError();
}

}  // namespace vmfmm
