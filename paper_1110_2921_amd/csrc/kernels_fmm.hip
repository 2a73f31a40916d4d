// Expansion kernels: P2M and L2P (one workgroup per leaf), the translation
// GEMMs (M2M, M2L, L2L) on the MFMA units, and the periodic lattice operator.
//
// Coefficient layout: cell-major, [cell][component][kp] with kp = (p+1)^2
// rounded up to a multiple of 32 (whole k blocks); entries C..kp-1 are zero.
#include <algorithm>

#include "device_harmonics.h"
#include "kernels.h"

namespace vmfmm {

namespace {

using dev::for_each_harmonic;
using dev::PartOf;
using dev::Tab;

template <typename T>
struct Quad {                               // four consecutive T from 16-byte aligned memory
    T v[4];
    __device__ __forceinline__ void load(const T *p) {
        if constexpr (sizeof(T) == 4) {
            typedef float f4 __attribute__((ext_vector_type(4)));
            const f4 q = *reinterpret_cast<const f4 *>(p);
            v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else {
            typedef double d2 __attribute__((ext_vector_type(2)));
            const d2 q0 = *reinterpret_cast<const d2 *>(p);
            const d2 q1 = *reinterpret_cast<const d2 *>(p + 2);
            v[0] = q0.x; v[1] = q0.y; v[2] = q1.x; v[3] = q1.y;
        }
    }
};

// ---------------------------------------------------------------- P2M ----
// Mb[leaf][c][s] = sum_j alpha_j[c] c_s((x_j - centre) / w).
// The orders m = 0..p are split into G >= 4 contiguous ranges of about equal
// coefficient count, at most 64 each; one wave takes one (leaf, m range): lane j
// evaluates the harmonics of particle j for its m range into LDS (row j),
// then lane t sums coefficient t of the range over the particles for the
// three strength components.  A wave needs only 64 rows of a quarter of the
// coefficients, so four to five waves fit per SIMD.  The G waves of a leaf
// are consecutive on one XCD (which serves a contiguous range of leaves).
constexpr int kP2mMaxGroups = 16;

struct MGroups {
    int ng;                       // number of ranges G
    int lo[kP2mMaxGroups + 1];    // range g takes orders lo[g] .. lo[g+1]-1
    int maxn;                     // largest coefficient count of a range (<= 64)
};

__device__ __forceinline__ int group_count(int p, int mlo, int mhi) {
    int c = 0;
    for (int m = mlo; m < mhi; ++m) c += (p + 1 - m) * (m > 0 ? 2 : 1);
    return c;
}

// Contiguous m ranges of about C / G coefficients each, the smallest G >= 4
// with at most 64 per range (ng = 0 if there is none).
constexpr MGroups p2m_groups(int p) {
    MGroups grp{};
    const int C = (p + 1) * (p + 1);
    for (int G = 4; G <= kP2mMaxGroups; ++G) {
        grp.ng = G;
        int m = 0, done = 0;
        for (int g = 0; g < G; ++g) {
            grp.lo[g] = m;
            const int target = (C * (g + 1) + G - 1) / G;
            while (m <= p && (g == G - 1 || done + (p + 1 - m) * (m > 0 ? 2 : 1) / 2 < target)) {
                done += (p + 1 - m) * (m > 0 ? 2 : 1);
                ++m;
            }
        }
        grp.lo[G] = p + 1;
        grp.maxn = 0;
        for (int g = 0; g < G; ++g) {
            int c = 0;
            for (int mm = grp.lo[g]; mm < grp.lo[g + 1]; ++mm) c += (p + 1 - mm) * (mm > 0 ? 2 : 1);
            grp.maxn = c > grp.maxn ? c : grp.maxn;
        }
        if (grp.maxn <= 64) return grp;
    }
    grp.ng = 0;
    return grp;
}

// Regular harmonics of one particle, orders mlo .. mhi-1 and degrees m .. p, into
// row (order m, then n, (re, -im) pairs for m > 0).  With PT > 0 the degree and
// the range are the compile-time PT, MLO, MHI: the recurrence then unrolls and
// its table reads become scalar loads at fixed offsets, issued together.
// (the unroll requests cannot be met where the bounds are run-time values)
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wpass-failed"
template <typename T, int PT, int MLO, int MHI>
__device__ __forceinline__ void p2m_row(T X, T Y, T Z, int p_rt, int mlo_rt, int mhi_rt, const T *__restrict__ c1,
                                        const T *__restrict__ c2, const T *__restrict__ dg, T *row) {
    const int p = PT > 0 ? PT : p_rt, mlo = PT > 0 ? MLO : mlo_rt, mhi = PT > 0 ? MHI : mhi_rt;
    const T r2 = X * X + Y * Y + Z * Z;
    // diagonal Rb_m^m = -(X + iY) diag[m] Rb_{m-1}^{m-1} up to the range start
    T dre = T(1), dim = T(0);
#pragma unroll
    for (int m = 1; m <= mlo; ++m) {
        const T sc = -dg[m];
        const T nre = sc * (X * dre - Y * dim);
        const T nim = sc * (X * dim + Y * dre);
        dre = nre;
        dim = nim;
    }
    int o = 0;
#pragma unroll
    for (int m = mlo; m < mhi; ++m) {
        if (m > mlo) {
            const T sc = -dg[m];
            const T nre = sc * (X * dre - Y * dim);
            const T nim = sc * (X * dim + Y * dre);
            dre = nre;
            dim = nim;
        }
        T are = dre, aim = dim, bre = T(0), bim = T(0);
        row[o++] = are;
        if (m > 0) row[o++] = -aim;
#pragma unroll
        for (int n = m + 1; n <= p; ++n) {
            const int e = n * (n + 1) / 2 + m;
            const T k1 = c1[e] * Z, k2 = c2[e] * r2;
            const T cre = k1 * are - k2 * bre;
            const T cim = k1 * aim - k2 * bim;
            bre = are;
            bim = aim;
            are = cre;
            aim = cim;
            row[o++] = are;
            if (m > 0) row[o++] = -aim;
        }
    }
}

#pragma clang diagnostic pop

// p2m_row for range g of the compile-time partition of degree PT.
template <typename T, int PT, int GI>
__device__ __forceinline__ void p2m_row_fixed(int g, T X, T Y, T Z, const T *__restrict__ c1,
                                              const T *__restrict__ c2, const T *__restrict__ dg, T *row) {
    constexpr MGroups GP = p2m_groups(PT);
    if constexpr (GI < GP.ng) {
        if (g == GI) {
            p2m_row<T, PT, GP.lo[GI], GP.lo[GI + 1]>(X, Y, Z, 0, 0, 0, c1, c2, dg, row);
            return;
        }
        p2m_row_fixed<T, PT, GI + 1>(g, X, Y, Z, c1, c2, dg, row);
    }
}

// PT > 0: the degree p is PT (the partition grp is p2m_groups(PT)).
template <typename T, int PT>
__global__ void __launch_bounds__(64) k_p2m(const typename PartOf<T>::type *__restrict__ parts,
                                            const int32_t *__restrict__ start, int nleaf, int p, int kp,
                                            T inv_w, DevTables tab, MGroups grp, T *__restrict__ mout,
                                            LeafMap lm, T *__restrict__ mcout, const int16_t *__restrict__ mc_pos,
                                            int kc) {
    static_assert(PT == 0 || p2m_groups(PT).ng > 0, "no partition of the orders for this degree");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int lane = threadIdx.x;
    // XCD-aware: blockIdx mod 8 selects the XCD's leaf range; the 4 groups of a leaf follow
    const int b = blockIdx.x, G = grp.ng;
    int leaf, g;
    if (nleaf % 8 == 0) {
        const int k = b >> 3;
        g = k % G;
        leaf = (b & 7) * (nleaf >> 3) + k / G;
    } else {
        g = b % G;
        leaf = b / G;
    }
    size_t mcell = size_t(leaf);
    if (lm.cell) {               // adaptive tree: the leaf's own width and cell slot
        inv_w = T(ldexp(lm.inv_len, lm.lev[leaf]));
        mcell = size_t(lm.cell[leaf]);
    }
    const int mlo = grp.lo[g], mhi = grp.lo[g + 1];
    const int ng = group_count(p, mlo, mhi);
    const int stride = grp.maxn + 1;                     // odd row stride: conflict-free column reads
    T *rows = reinterpret_cast<T *>(smem_raw);           // [64][stride]
    T *al = rows + 64 * stride;                          // [64][3]
    const int s0 = start[leaf], cnt = start[leaf + 1] - s0;
    const T *c1 = Tab<T>::c1(tab), *c2 = Tab<T>::c2(tab), *dg = Tab<T>::dg(tab);
    T acc[3] = {T(0), T(0), T(0)};
    for (int base = 0; base < cnt; base += 64) {
        const int nj = min(64, cnt - base);
        if (lane < nj) {
            const auto q = parts[s0 + base + lane];
            T *row = rows + lane * stride;
            const T X = T(q.dx) * inv_w, Y = T(q.dy) * inv_w, Z = T(q.dz) * inv_w;
            if constexpr (PT > 0) p2m_row_fixed<T, PT, 0>(g, X, Y, Z, c1, c2, dg, row);
            else p2m_row<T, 0, 0, 0>(X, Y, Z, p, mlo, mhi, c1, c2, dg, row);
            al[lane * 3 + 0] = q.ax;
            al[lane * 3 + 1] = q.ay;
            al[lane * 3 + 2] = q.az;
        }
        __syncthreads();
        if (lane < ng)
            for (int j = 0; j < nj; ++j) {
                const T v = rows[j * stride + lane];
                acc[0] += al[j * 3 + 0] * v;
                acc[1] += al[j * 3 + 1] * v;
                acc[2] += al[j * 3 + 2] * v;
            }
        __syncthreads();
    }
    if (lane >= ng) return;
    // local index -> packed index: order m, then n, (re, -im) pairs for m > 0
    int m = mlo, n = mlo, part = 0;
    for (int o = 0; o < lane; ++o) {
        if (m > 0 && part == 0) {
            part = 1;
            continue;
        }
        part = 0;
        if (++n > p) {
            ++m;
            n = m;
        }
    }
    const int sidx = m == 0 ? n * n : n * n + 2 * m - 1 + part;
    T *dst = mout + mcell * 3 * kp;
    for (int c = 0; c < 3; ++c) dst[c * kp + sidx] = acc[c];
    if (mcout) {
        // the class-major copy the reflection-orbit M2L reads (padding stays zero)
        T *mc = mcout + mcell * 3 * kc + mc_pos[sidx];
        for (int c = 0; c < 3; ++c) mc[c * kc] = acc[c];
    }
}

// ---------------------------------------------------------------- L2P ----
// Per leaf: velocity / gradient expansions from the sparse table, then per
// particle u_b = sU sum U_b c(X), J_ab = sJ sum G_ab c(X), written in sorted
// order as far[0..2][n] (u) and far[3..11][n] (J, index 3a+b).
constexpr double kInv4PiL2P = 0.079577471545947667884441881686257181;

// u, grad, dalpha of sorted target gi from the near field of a P2P launch and
// the far field uf, Jf: the P2P epilogue's operations in its order.
__device__ __forceinline__ void combine_store(const NearCombine &c, size_t n, size_t gi, const double uf[3],
                                              const double Jf[9]) {
    const double *nr = c.near;
    const int oi = c.perm[gi];
    for (int b = 0; b < 3; ++b) c.u[b * n + oi] = nr[b * n + gi] * kInv4PiL2P + uf[b];
    if (!c.grad && !c.dalpha) return;
    double Sd[3];
    for (int k = 0; k < 3; ++k) Sd[k] = nr[(12 + k) * n + gi];
    double al[3] = {0.0, 0.0, 0.0};
    if (c.dalpha)
        for (int k = 0; k < 3; ++k) al[k] = c.alpha[k * n + oi];
    double da[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            // antisymmetric part eps_rkm S_m of the near gradient J[r][k]
            const int m = 3 - r - k;
            const double anti = r == k ? 0.0 : ((k == (r + 1) % 3) ? Sd[m] : -Sd[m]);
            const double J = (nr[(3 + 3 * r + k) * n + gi] + anti) * kInv4PiL2P + Jf[3 * r + k];
            if (c.grad) c.grad[(3 * r + k) * n + oi] = J;
            if (c.scheme == 0) da[k] += al[r] * J;      // classic: sum_a alpha_a J[a][b]
            else da[r] += J * al[k];                     // transpose: sum_c J[b][c] alpha_c
        }
    }
    if (c.dalpha)
        for (int b = 0; b < 3; ++b) c.dalpha[b * n + oi] = da[b];
}

template <typename T>
__global__ void __launch_bounds__(64) k_l2p(const typename PartOf<T>::type *__restrict__ parts,
                                            const int32_t *__restrict__ start, int n, int p, int kp,
                                            T inv_w, double su, double sj, DevTables tab,
                                            const T *__restrict__ lleaf, double *__restrict__ far, LeafMap lm,
                                            NearCombine nc) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int C = (p + 1) * (p + 1);
    const int nu = tab.nu, ng = tab.ng, width = tab.l2p_width;
    T *coef = reinterpret_cast<T *>(smem_raw);  // [nu][12]: U_x U_y U_z G_00 .. G_22 (16-byte rows)
    T *lam = coef + 12 * nu;                    // [3 C]
    const int leaf = blockIdx.x, lane = threadIdx.x;
    const int s0 = start[leaf], cnt = start[leaf + 1] - s0;
    if (cnt == 0) return;
    size_t lcell = size_t(leaf);
    if (lm.cell) {               // adaptive tree: the leaf's own width and cell slot
        const double w = ldexp(lm.box_len, -lm.lev[leaf]);
        inv_w = T(ldexp(lm.inv_len, lm.lev[leaf]));
        su = 1.0 / (12.566370614359172953850573533118 * w * w);
        sj = 1.0 / (12.566370614359172953850573533118 * w * w * w);
        lcell = size_t(lm.cell[leaf]);
    }
    const T *src = lleaf + lcell * 3 * kp;
    // the expansion in 64-element rounds of loads issued together (clamped
    // indices, unconditional loads), then stored
    for (int i0 = 0; i0 < 3 * C; i0 += 256) {
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + 64 * u + lane, ic = i < 3 * C ? i : 0;
            v[u] = src[(ic / C) * kp + (ic % C)];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + 64 * u + lane;
            if (i < 3 * C) lam[i] = v[u];
        }
    }
    for (int r = lane; r < 12 * nu; r += 64) coef[r] = T(0);
    __syncthreads();
    const T *tw = Tab<T>::w(tab);
    const int rows = 3 * nu + 9 * ng;
    auto put = [&](int r, T v) {
        int slot, comp;
        if (r < 3 * nu) {
            comp = r / nu;
            slot = r % nu;
        } else {
            comp = 3 + (r - 3 * nu) / ng;
            slot = (r - 3 * nu) % ng;
        }
        coef[slot * 12 + comp] = v;
    };
    // two rows per lane at a time (r, r + 64): twice the table loads in flight
    for (int r = lane; r < rows; r += 128) {
        const int r2 = r + 64;
        const int rc = r2 < rows ? r2 : r;
        T s = T(0), s2 = T(0);
        for (int e = 0; e < width; ++e) {
            const size_t e0 = size_t(e) * rows;
            s += tw[e0 + r] * lam[tab.l2p_idx[e0 + r]];
            s2 += tw[e0 + rc] * lam[tab.l2p_idx[e0 + rc]];
        }
        put(r, s);
        if (r2 < rows) put(r2, s2);
    }
    __syncthreads();
    const T *c1 = Tab<T>::c1(tab), *c2 = Tab<T>::c2(tab), *dg = Tab<T>::dg(tab);
    for (int base = 0; base < cnt; base += 64) {
        const int i = base + lane;
        if (i >= cnt) break;
        const auto q = parts[s0 + i];
        T u[3] = {T(0), T(0), T(0)};
        T J[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) J[k] = T(0);
        for_each_harmonic<T>(T(q.dx) * inv_w, T(q.dy) * inv_w, T(q.dz) * inv_w, p - 1, c1, c2, dg,
                             [&](int nn, int m, T re, T nim) {
                                 const int sr = m == 0 ? nn * nn : nn * nn + 2 * m - 1;
                                 Quad<T> cq[3];
#pragma unroll
                                 for (int q4 = 0; q4 < 3; ++q4) cq[q4].load(coef + sr * 12 + 4 * q4);
#pragma unroll
                                 for (int b = 0; b < 3; ++b) u[b] += cq[b / 4].v[b % 4] * re;
#pragma unroll
                                 for (int k = 0; k < 9; ++k) J[k] += cq[(3 + k) / 4].v[(3 + k) % 4] * re;
                                 if (m > 0) {
#pragma unroll
                                     for (int q4 = 0; q4 < 3; ++q4) cq[q4].load(coef + (sr + 1) * 12 + 4 * q4);
#pragma unroll
                                     for (int b = 0; b < 3; ++b) u[b] += cq[b / 4].v[b % 4] * nim;
#pragma unroll
                                     for (int k = 0; k < 9; ++k) J[k] += cq[(3 + k) / 4].v[(3 + k) % 4] * nim;
                                 }
                             });
        const size_t gi = size_t(s0) + i;
        double uf[3], Jf[9];
        for (int b = 0; b < 3; ++b) uf[b] = double(u[b]) * su;
        for (int kk = 0; kk < 9; ++kk) Jf[kk] = double(J[kk]) * sj;
        if (nc.near) {
            combine_store(nc, size_t(n), gi, uf, Jf);
        } else {
            for (int b = 0; b < 3; ++b) far[size_t(b) * n + gi] = uf[b];
            for (int kk = 0; kk < 9; ++kk) far[size_t(3 + kk) * n + gi] = Jf[kk];
        }
    }
}

// ----------------------------------------------------------- translate ----
// The translations are GEMMs over a tile of target cells that share one list
// of (operator, source) pairs (M2L: one octant and its 189 offsets; L2L: one
// child octant; M2M: the 8 children of each parent):
//   out[tile] (C x 3 tile) += sum over pairs Op (C x C) * Src (C x 3 tile),
// with the sums kept in MFMA accumulators across all pairs.
// MFMA 16x16x4: A lane l = (row l%16, k l/16), B lane l = (k l/16, col l%16);
// accumulator register r of lane l holds column l%16 and row (l/16) + 4r for
// FP64, 4(l/16) + r for FP32 (both checked on gfx950).
template <typename T> struct Mfma;
template <> struct Mfma<double> {
    typedef double v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(double a, double b, v4 c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
    typedef float v4 __attribute__((ext_vector_type(4)));
    static __device__ __forceinline__ v4 op(float a, float b, v4 c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

__device__ __forceinline__ uint32_t morton3(int cx, int cy, int cz, int level) {
    uint32_t k = 0;
    for (int b = 0; b < level; ++b) {
        k |= uint32_t((cx >> b) & 1) << (3 * b);
        k |= uint32_t((cy >> b) & 1) << (3 * b + 1);
        k |= uint32_t((cz >> b) & 1) << (3 * b + 2);
    }
    return k;
}

__device__ __forceinline__ int demorton1(uint32_t k, int d, int level) {
    int c = 0;
    for (int b = 0; b < level; ++b) c |= int((k >> (3 * b + d)) & 1u) << b;
    return c;
}

// Workgroup of 8 waves (two per SIMD); wave w owns the row blocks w, w+8, ...
// PF > 0: the sources of pair k+1 are loaded into registers (PF per thread)
// while pair k runs on the MFMA units, then written to the other LDS buffer,
// so each pair costs one barrier and the loads overlap the matrix work.
// PF = 0: single buffer, loads and compute in turn (large p).
//
// K order: within each block of 16 coefficients, MFMA k step 4b+s takes
// coefficient 16b + 4h + s in lane group h (the operator fragments are built
// on the host in the same order), so a lane reads the B values of four k
// steps as one 16-byte LDS load.  With the row stride S of the staging
// buffer chosen so that S/4 (FP32) or S/2 (FP64) is odd, the 16 lanes of a
// group hit 16 distinct 16-byte bank groups.
//
// Split form (M2L at coarse levels, where there are too few target tiles to
// fill the chip): blockIdx.y selects a contiguous range of the 189 offsets
// and the partial sums go to `part` ([split][cell][3][kp]), reduced in
// order by k_split_reduce.
constexpr int kTrThreads = 512;
constexpr int kTrWaves = kTrThreads / 64;
static_assert(kTrWaves == kTrWaveCount, "operator padding assumes one row-block group per wave");

template <typename T>
__host__ __device__ constexpr int tr_row_stride(int nks) { return 4 * nks + (sizeof(T) == 4 ? 4 : 2); }

template <typename T, int NRBW, int NT, int mode, int PF>
__global__ void __launch_bounds__(kTrThreads) k_translate(int level, int periodic, int C, int kp,
                                                          int nrb, int nks, const T *__restrict__ ops,
                                                          const int16_t *__restrict__ oct_lists,
                                                          const int8_t *__restrict__ offsets,
                                                          const T *__restrict__ src, T *__restrict__ dst,
                                                          int accumulate, int nsplit, T *__restrict__ part,
                                                          AdaptTr ad) {
    using V = typename Mfma<T>::v4;
    constexpr int TTN = 16 * NT;
    constexpr int NCB = 3 * NT;                          // column blocks: (group, component)
    constexpr int NBUF = PF > 0 ? 2 : 1;
    constexpr int APF = 8;                               // operator prefetch distance (k steps)
    static_assert(APF % 8 == 0, "the ring holds whole pairs of k blocks (k blocks per operator are even)");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int ks_stride = tr_row_stride<T>(nks);
    const int buf_elems = TTN * 3 * ks_stride;
    T *bs = reinterpret_cast<T *>(smem_raw);             // [NBUF][TTN * 3][ks_stride]
    __shared__ int32_t tkey[TTN];
    __shared__ int32_t skey[2][TTN];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int per_cell = 3 * kp;

    int octant = 0, tile = blockIdx.x, npair = 1, pr0 = 0;
    int64_t ncell_t;
    const bool adaptive = ad.tcell != nullptr;   // cells and sources from tables (adaptive tree)
    if (mode == 2) {                  // M2M: targets are the parents at `level`
        ncell_t = adaptive ? ad.ntarget : int64_t(1) << (3 * level);
        npair = 8;
    } else if (adaptive) {            // octant groups of one level, tile_start[o] .. workgroups each
        octant = 0;
        while (octant < 7 && int(blockIdx.x) >= ad.tile_start[octant + 1]) ++octant;
        tile = int(blockIdx.x) - ad.tile_start[octant];
        ncell_t = ad.oct_n[octant];
        if (mode == 0) {
            pr0 = int(blockIdx.y) * 189 / nsplit;
            npair = (int(blockIdx.y) + 1) * 189 / nsplit - pr0;
        }
    } else {                          // M2L / L2L: targets at `level`, grouped by octant
        octant = blockIdx.x & 7;
        tile = blockIdx.x >> 3;
        ncell_t = int64_t(1) << (3 * (level - 1));
        if (mode == 0) {
            pr0 = int(blockIdx.y) * 189 / nsplit;
            npair = (int(blockIdx.y) + 1) * 189 / nsplit - pr0;
        }
    }
    if (tid < TTN) {
        const int64_t slot = int64_t(tile) * TTN + tid;
        int32_t k = -1;
        if (adaptive) {
            if (slot < ncell_t) k = mode == 2 ? ad.tcell[slot] : ad.tcell[ad.oct_base[octant] + slot];
            if (mode == 2 && k >= 0) {
                bool any = false;
                for (int o = 0; o < 8; ++o) any = any || ad.child[8 * size_t(k) + o] >= 0;
                if (!any) k = -1;     // a leaf: its multipole is its own P2M
            }
        } else if (slot < ncell_t) {
            k = mode == 2 ? int32_t(slot) : int32_t((slot << 3) | octant);
        }
        tkey[tid] = k;
    }
    // the K padding of the staging buffers stays zero
    for (int e = tid; e < NBUF * buf_elems; e += kTrThreads) bs[e] = T(0);
    const int side = 1 << level;
    // operator of local pair i
    auto op_of = [&](int i) -> int {
        if (mode == 0) return oct_lists[octant * 189 + pr0 + i];
        if (mode == 1) return octant;
        return i;
    };
    // source cell of target slot `tid` for local pair i (or -1)
    auto source_key = [&](int i) -> int32_t {
        const int32_t t = tkey[tid];
        if (t < 0) return -1;
        if (adaptive) {
            if (mode == 0) return ad.stab[size_t(t - ad.cell0) * 189 + pr0 + i];
            if (mode == 1) return ad.parent[t];
            return ad.child[8 * size_t(t) + i];
        }
        if (mode == 0) {
            const int op = op_of(i);
            int c[3];
            for (int d = 0; d < 3; ++d) {
                c[d] = demorton1(uint32_t(t), d, level) + offsets[op * 3 + d];
                if (periodic) c[d] = (c[d] % side + side) % side;
                else if (c[d] < 0 || c[d] >= side) return -1;
            }
            return int32_t(morton3(c[0], c[1], c[2], level));
        }
        if (mode == 1) return t >> 3;
        return (t << 3) | i;
    };
    // staging map: thread tid serves target slot tid / TPT and walks that cell's
    // 3 kp coefficients with stride TPT (coalesced within the slot's threads)
    constexpr int TPT = kTrThreads / TTN;
    const int st_t = tid / TPT, st_r0 = tid % TPT;
    auto stage_direct = [&](int kb, T *buf) {
        const int32_t sk = skey[kb][st_t];
        int c = 0, k = st_r0;
        for (int r = st_r0; r < per_cell; r += TPT) {
            while (k >= kp) { k -= kp; ++c; }
            buf[(st_t * 3 + c) * ks_stride + k] = sk >= 0 ? src[size_t(sk) * per_cell + r] : T(0);
            k += TPT;
        }
    };

    V acc[NRBW][NCB];
#pragma unroll
    for (int i = 0; i < NRBW; ++i)
#pragma unroll
        for (int c = 0; c < NCB; ++c) acc[i][c] = V{T(0), T(0), T(0), T(0)};
    __syncthreads();

    // One pair: out += Op * Src.  Straight-line k blocks (four k steps): the A
    // quads stream from L2 through a ring of RQ blocks; the B values of a k
    // block arrive in one 16-byte LDS read per column block.
    constexpr int RQ = APF / 4;
    const int nkb = nks / 4;
    auto mfma_pair = [&](int i_pair, const T *buf) {
        const T *opb = ops + size_t(op_of(i_pair)) * nrb * nks * 64 + 4 * lane;
        Quad<T> ring[RQ][NRBW];
#pragma unroll
        for (int q = 0; q < RQ; ++q)
#pragma unroll
            for (int i = 0; i < NRBW; ++i) ring[q][i].load(opb + (size_t(wave + kTrWaves * i) * nkb + q) * 256);
        const T *bl = buf + (lane & 15) * 3 * ks_stride + 4 * (lane >> 4);
        for (int kb0 = 0; kb0 < nkb; kb0 += RQ) {
#pragma unroll
            for (int q = 0; q < RQ; ++q) {
                const int kb = kb0 + q;
                Quad<T> bq[NCB];
#pragma unroll
                for (int g = 0; g < NT; ++g)
#pragma unroll
                    for (int c = 0; c < 3; ++c) bq[g * 3 + c].load(bl + (g * 16 * 3 + c) * ks_stride + 16 * kb);
                const int kn = kb + RQ < nkb ? kb + RQ : nkb - 1;
                Quad<T> a_use[NRBW];
#pragma unroll
                for (int i = 0; i < NRBW; ++i) {
                    a_use[i] = ring[q][i];
                    ring[q][i].load(opb + (size_t(wave + kTrWaves * i) * nkb + kn) * 256);
                }
#pragma unroll
                for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                    for (int i = 0; i < NRBW; ++i)
#pragma unroll
                        for (int cb = 0; cb < NCB; ++cb)
                            acc[i][cb] = Mfma<T>::op(a_use[i].v[s4], bq[cb].v[s4], acc[i][cb]);
            }
        }
    };

    if constexpr (PF > 0) {
        if (tid < TTN) skey[0][tid] = source_key(0);
        __syncthreads();
        stage_direct(0, bs);
        if (tid < TTN && npair > 1) skey[1][tid] = source_key(1);
        __syncthreads();
        for (int pr = 0; pr < npair; ++pr) {
            const int cur = pr & 1, nxt = cur ^ 1;
            const bool more = pr + 1 < npair;
            T pf[PF];
            if (more) {
                const int32_t sk = skey[nxt][st_t];
                const T *sp = src + size_t(sk >= 0 ? sk : 0) * per_cell;
#pragma unroll
                for (int j = 0; j < PF; ++j) {
                    const int r = st_r0 + TPT * j;
                    pf[j] = (sk >= 0 && r < per_cell) ? sp[r] : T(0);
                }
            }
            mfma_pair(pr, bs + cur * buf_elems);
            if (more) {
                T *nb = bs + nxt * buf_elems + st_t * 3 * ks_stride;
                int c = 0, k = st_r0;
#pragma unroll
                for (int j = 0; j < PF; ++j) {
                    const int r = st_r0 + TPT * j;
                    if (r < per_cell) {
                        while (k >= kp) { k -= kp; ++c; }
                        nb[c * ks_stride + k] = pf[j];
                        k += TPT;
                    }
                }
            }
            if (tid < TTN && pr + 2 < npair) skey[cur][tid] = source_key(pr + 2);
            __syncthreads();
        }
    } else {
        for (int pr = 0; pr < npair; ++pr) {
            if (tid < TTN) skey[0][tid] = source_key(pr);
            __syncthreads();
            stage_direct(0, bs);
            __syncthreads();
            mfma_pair(pr, bs);
            __syncthreads();
        }
    }
    // write back: lane holds rows rb*16 + Mfma::row(lane, r) of target column lane%16 of each group
    const bool split = part != nullptr;
#pragma unroll
    for (int g = 0; g < NT; ++g) {
        const int32_t t = tkey[g * 16 + (lane & 15)];
        if (t < 0) continue;
        T *out = !split ? dst + size_t(t) * per_cell
                 : adaptive ? part + (size_t(blockIdx.y) * size_t(ad.part_cells) + size_t(t - ad.part_cell0)) * per_cell
                            : part + (size_t(blockIdx.y) * (size_t(1) << (3 * level)) + t) * per_cell;
#pragma unroll
        for (int i = 0; i < NRBW; ++i) {
            const int rb = wave + kTrWaves * i;
#pragma unroll
            for (int c = 0; c < 3; ++c)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = rb * 16 + Mfma<T>::row(lane, r);
                    if (row < C) {
                        const T v = acc[i][g * 3 + c][r];
                        T *o = out + c * kp + row;
                        *o = (accumulate && !split) ? *o + v : v;
                    }
                }
        }
    }
}

// dst[cell] (+)= sum over splits of part[split][cell], rows < C only, fixed order.
template <typename T>
__global__ void __launch_bounds__(256) k_split_reduce(int64_t nelem, int kp, int C, int nsplit,
                                                      const T *__restrict__ part, T *__restrict__ dst,
                                                      int accumulate) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= nelem) return;
    if (int(e % kp) >= C) return;
    T s = T(0);
    for (int k = 0; k < nsplit; ++k) s += part[size_t(k) * nelem + e];
    dst[e] = accumulate ? dst[e] + s : s;
}

// M2L in FP32, operator-stationary form.  A workgroup of 8 waves takes 64
// same-octant target cells; wave w serves targets 16 (w/2) .. +15 and row
// blocks NRBH (w%2) .. +NRBH-1.  Per interaction offset the operator (2 NRBH
// row blocks x NB k blocks of A quads) sits in LDS, double-buffered and
// shared by all waves, while each lane holds its own target's source
// coefficients as B quads in registers (NB x 3 quads).  The next offset's
// operator is copied into the other LDS buffer in 8 KB chunks held two k blocks
// in registers, and the next offset's sources are loaded into a B quad right
// after its last use, so the loads overlap the MFMAs and each offset costs one
// barrier.
//
// Source loads are unconditional: a missing source (no target in the slot,
// or a free-space offset leaving the domain) reads `zero_cell`, and the last
// k block may read up to 4 nks - kp values past a component, which meet zero
// operator columns (the expansion buffers carry that much slack at their end).
// Scheduling barriers keep each k block in the order chunk store, chunk load,
// A reads, MFMAs, source loads, so the wait for a chunk never covers the
// newer source loads.
//
// TRI: operators truncated to n + n' <= p (target degree n, source degree
// n'), whose row block rb is zero beyond its first kb(rb) k blocks.  Slot i of
// wave half rh then serves row block (rbmap >> 4 (rh NRBH + i)) & 15 and runs
// its MFMAs and A reads for the first (kbmap >> 4 (rh NRBH + i)) & 15 k blocks
// only; the host balances the two halves' k blocks.
template <int NRBH, int NB, bool TRI>
__global__ void __launch_bounds__(kTrThreads) k_m2l_os(int level, int periodic, int C, int kp, int nrb_pad,
                                                       int nks, const float *__restrict__ ops,
                                                       const int16_t *__restrict__ oct_lists,
                                                       const int8_t *__restrict__ offsets,
                                                       const float *__restrict__ src, float *__restrict__ dst,
                                                       int accumulate, int nsplit, float *__restrict__ part,
                                                       const float *__restrict__ zero_cell, uint32_t rbmap,
                                                       uint32_t kbmap) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    using V = Mfma<float>::v4;
    constexpr int TT = 64;                               // target cells per workgroup
    constexpr int OPF = 2 * NRBH * NB * 256;             // floats of one operator in LDS
    constexpr int CHUNK = 4 * kTrThreads;                // floats copied per k block
    constexpr int NCHUNK = (OPF + CHUNK - 1) / CHUNK;
    constexpr bool EXACT = OPF % CHUNK == 0;
    constexpr int NPAIRC = (NCHUNK + 1) / 2;             // k blocks that store two chunks each
    static_assert(NPAIRC <= NB, "the operator copy must finish within one offset");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *opl = reinterpret_cast<float *>(smem_raw);    // [2][OPF]
    __shared__ int32_t tkey[TT];
    __shared__ int32_t pinfo[189];                       // per local offset: op | (d + 8) in 4-bit fields
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int tg = wave >> 1, rh = wave & 1, h = lane >> 4;
    const int octant = blockIdx.x & 7, tile = blockIdx.x >> 3;
    int rbs[NRBH], kbs[NRBH];   // row block of each slot and its k blocks (wave-uniform)
#pragma unroll
    for (int i = 0; i < NRBH; ++i) {
        rbs[i] = TRI ? int((rbmap >> (4 * (rh * NRBH + i))) & 15u) : rh * NRBH + i;
        kbs[i] = TRI ? int((kbmap >> (4 * (rh * NRBH + i))) & 15u) : NB;
    }
    const int64_t ncell_t = int64_t(1) << (3 * (level - 1));
    const int pr0 = int(blockIdx.y) * 189 / nsplit;
    const int npair = (int(blockIdx.y) + 1) * 189 / nsplit - pr0;
    const size_t op_stride = size_t(nrb_pad) * nks * 64;
    const int per_cell = 3 * kp;
    const int side = 1 << level;
    if (tid < TT) {
        const int64_t slot = int64_t(tile) * TT + tid;
        tkey[tid] = slot < ncell_t ? int32_t((slot << 3) | octant) : -1;
    }
    if (tid < npair) {
        const int op = oct_lists[octant * 189 + pr0 + tid];
        pinfo[tid] = op | ((offsets[op * 3] + 8) << 16) | ((offsets[op * 3 + 1] + 8) << 20) |
                     ((offsets[op * 3 + 2] + 8) << 24);
    }
    __syncthreads();
    const int32_t t = tkey[tg * 16 + (lane & 15)];
    int tc[3] = {0, 0, 0};
    if (t >= 0)
        for (int d = 0; d < 3; ++d) tc[d] = demorton1(uint32_t(t), d, level);
    // this lane's source cell for local offset i (zero_cell: none), k offset of its lane group
    auto src_of = [&](int i) -> const float * {
        const int info = pinfo[i];
        int c[3];
        bool ok = t >= 0;
        for (int d = 0; d < 3; ++d) {
            c[d] = tc[d] + ((info >> (16 + 4 * d)) & 15) - 8;
            if (periodic) c[d] &= side - 1;
            else ok = ok && c[d] >= 0 && c[d] < side;
        }
        const float *sp = ok ? src + size_t(morton3(c[0], c[1], c[2], level)) * per_cell : zero_cell;
        return sp + 4 * h;
    };
    auto op_of = [&](int i) { return ops + size_t(pinfo[i] & 0xffff) * op_stride; };
    f4 B[NB][3];
    auto load_b = [&](int b, const float *sp) {
#pragma unroll
        for (int c = 0; c < 3; ++c) B[b][c] = *reinterpret_cast<const f4 *>(sp + c * kp + 16 * b);
    };
    // Operators are loaded into registers AHEAD offsets before their use: two
    // for the square form, one for the truncated form, whose row-block maps
    // leave no registers for a second set.
    constexpr int AHEAD = TRI ? 1 : 2;
    f4 stage[2 * NPAIRC];   // the chunks of the operator after the current one
    {
        const float *og = op_of(0);
        for (int e = 4 * tid; e < OPF; e += CHUNK)
            *reinterpret_cast<f4 *>(opl + e) = *reinterpret_cast<const f4 *>(og + e);
        const float *og1 = op_of(npair > 1 ? 1 : 0) + 4 * tid;
        if constexpr (AHEAD == 2)
#pragma unroll
            for (int ch = 0; ch < NCHUNK; ++ch)
                if (EXACT || ch * CHUNK + 4 * tid < OPF) stage[ch] = *reinterpret_cast<const f4 *>(og1 + ch * CHUNK);
        const float *sp = src_of(0);
#pragma unroll
        for (int b = 0; b < NB; ++b) load_b(b, sp);
    }
    V acc[NRBH][3];
#pragma unroll
    for (int i = 0; i < NRBH; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[i][c] = V{0.f, 0.f, 0.f, 0.f};
    __syncthreads();

    for (int pr = 0; pr < npair; ++pr) {
        const int cur = pr & 1;
        const bool more = pr + 1 < npair;
        const float *spn = src_of(more ? pr + 1 : pr);     // wave-uniform choice
        const float *ogn = op_of(pr + AHEAD < npair ? pr + AHEAD : npair - 1) + 4 * tid;
        float *oln = opl + (cur ^ 1) * OPF + 4 * tid;
        const float *olc = opl + cur * OPF + 4 * lane;
        // The chunks of the operator AHEAD offsets ahead are loaded first, ahead
        // of this offset's source loads.  Vector loads retire in order, so a
        // wait for a chunk also waits for every older load: issued first, the
        // chunks tie only older offsets' source loads.  AHEAD = 2: the
        // registers loaded one offset earlier go into the idle buffer, one chunk
        // per k block, so the chunks tie only source loads two offsets old.
        // AHEAD = 1: the chunks just loaded go there in the last NPAIRC k
        // blocks, two per k block, tying the previous offset's source loads
        // with NB - NPAIRC k blocks to arrive.  The loads are issued
        // unconditionally (near the end they re-read the last operator): a
        // branch around them would make the wait for a chunk cover every newer
        // load.
        f4 ahead[2 * NPAIRC];
#pragma unroll
        for (int ch = 0; ch < NCHUNK; ++ch)
            if (EXACT || ch * CHUNK + 4 * tid < OPF) {
                const f4 v = *reinterpret_cast<const f4 *>(ogn + ch * CHUNK);
                if constexpr (AHEAD == 2) ahead[ch] = v;
                else stage[ch] = v;
            }
        __builtin_amdgcn_sched_barrier(0);
        f4 aq[2][NRBH];
#pragma unroll
        for (int i = 0; i < NRBH; ++i)
            if (!TRI || kbs[i] > 0) aq[0][i] = *reinterpret_cast<const f4 *>(olc + (rbs[i] * NB) * 256);
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            // chunks [c0, c1) of the operator in `stage` go out in k block b
            const int c0 = AHEAD == 2 ? b * NCHUNK / NB : (b < NB - NPAIRC ? NCHUNK : 2 * (b - (NB - NPAIRC)));
            const int c1 = AHEAD == 2 ? (b + 1) * NCHUNK / NB : (b < NB - NPAIRC ? NCHUNK : c0 + 2);
#pragma unroll
            for (int ch = c0; ch < c1; ++ch)
                if (ch < NCHUNK && (EXACT || ch * CHUNK + 4 * tid < OPF))
                    *reinterpret_cast<f4 *>(oln + ch * CHUNK) = stage[ch];
            __builtin_amdgcn_sched_barrier(0);
            if (b + 1 < NB)
#pragma unroll
                for (int i = 0; i < NRBH; ++i)
                    if (!TRI || b + 1 < kbs[i])
                        aq[(b + 1) & 1][i] = *reinterpret_cast<const f4 *>(olc + (rbs[i] * NB + b + 1) * 256);
            // raised issue priority for the MFMA cluster: the SIMD's other wave,
            // between its own clusters, then yields to it instead of
            // interleaving its memory instructions into this one
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                for (int i = 0; i < NRBH; ++i)
                    if (!TRI || b < kbs[i])
#pragma unroll
                        for (int c = 0; c < 3; ++c)
                            acc[i][c] = Mfma<float>::op(aq[b & 1][i][s4], B[b][c][s4], acc[i][c]);
            __builtin_amdgcn_s_setprio(0);
            __builtin_amdgcn_sched_barrier(0);
            load_b(b, spn);
            __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (AHEAD == 2)
#pragma unroll
            for (int ch = 0; ch < NCHUNK; ++ch)
                if (EXACT || ch * CHUNK + 4 * tid < OPF) stage[ch] = ahead[ch];
        __syncthreads();
    }
    if (t < 0) return;
    const bool split = part != nullptr;
    float *out = split ? part + (size_t(blockIdx.y) * (size_t(1) << (3 * level)) + t) * per_cell
                       : dst + size_t(t) * per_cell;
#pragma unroll
    for (int i = 0; i < NRBH; ++i) {
        const int rb = rbs[i];
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rb * 16 + Mfma<float>::row(lane, r);
                if (row < C) {
                    float *o = out + c * kp + row;
                    *o = (accumulate && !split) ? *o + acc[i][c][r] : acc[i][c][r];
                }
            }
    }
}

// ------------------------------------------------------------- lattice ----
template <typename T>
__global__ void __launch_bounds__(256) k_lattice(int C, int kp, const double *__restrict__ tlat,
                                                 const T *__restrict__ m0, T *__restrict__ l0) {
    __shared__ double m[3 * 441];
    for (int i = threadIdx.x; i < 3 * C; i += 256) m[i] = double(m0[(i / C) * kp + (i % C)]);
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * C; i += 256) {
        const int c = i / C, row = i % C;
        double s = 0.0;
        for (int k = 0; k < C; ++k) s += tlat[size_t(row) * C + k] * m[c * C + k];
        l0[c * kp + row] = T(s);
    }
}

}  // namespace

template <typename T>
hipError_t launch_p2m(hipStream_t s, int nleaf, const void *parts, const int32_t *start, int p, int kp,
                      double inv_w, const DevTables &tab, T *m_out, const LeafMap &lm, T *mc_out,
                      const int16_t *mc_pos, int kc) {
    const MGroups grp = p2m_groups(p);
    if (grp.ng == 0) return hipErrorInvalidValue;
    const size_t smem = sizeof(T) * (size_t(64) * (grp.maxn + 1) + 64 * 3);
    const auto *pp = (const typename PartOf<T>::type *)parts;
    const dim3 grid(unsigned(nleaf) * grp.ng);
    // the degrees of the workloads at compile time, any other at run time
    switch (p) {
    case 6: hipLaunchKernelGGL((k_p2m<T, 6>), grid, dim3(64), smem, s, pp, start, nleaf, p, kp, T(inv_w), tab, grp, m_out, lm, mc_out, mc_pos, kc); break;
    case 8: hipLaunchKernelGGL((k_p2m<T, 8>), grid, dim3(64), smem, s, pp, start, nleaf, p, kp, T(inv_w), tab, grp, m_out, lm, mc_out, mc_pos, kc); break;
    case 10: hipLaunchKernelGGL((k_p2m<T, 10>), grid, dim3(64), smem, s, pp, start, nleaf, p, kp, T(inv_w), tab, grp, m_out, lm, mc_out, mc_pos, kc); break;
    default: hipLaunchKernelGGL((k_p2m<T, 0>), grid, dim3(64), smem, s, pp, start, nleaf, p, kp, T(inv_w), tab, grp, m_out, lm, mc_out, mc_pos, kc);
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_l2p(hipStream_t s, int nleaf, int n, const void *parts, const int32_t *start, int p,
                      int kp, double inv_w, double w, const DevTables &tab, const T *l_leaf, double *far,
                      const LeafMap &lm, const NearCombine &nc) {
    const int C = (p + 1) * (p + 1);
    const size_t smem = sizeof(T) * (3 * size_t(C) + 12 * size_t(tab.nu) + 12);
    const double four_pi = 12.566370614359172953850573533118;
    hipLaunchKernelGGL(k_l2p<T>, dim3(nleaf), dim3(64), smem, s, (const typename PartOf<T>::type *)parts,
                       start, n, p, kp, T(inv_w), 1.0 / (four_pi * w * w), 1.0 / (four_pi * w * w * w), tab,
                       l_leaf, far, lm, nc);
    return hipGetLastError();
}

// Tile shape: FP32 takes 32 targets per workgroup, FP64 16.  The pipelined
// form needs two staging buffers within 128 KB of LDS and at most 24 prefetch
// registers per thread; larger p falls back to one buffer and 16 targets.
struct TrShape {
    int nt, pf;   // 16-target groups; prefetch registers (0 = single buffer)
};

template <typename T>
TrShape translate_shape(int kp) {
    const int nt = sizeof(T) == 4 ? 2 : 1;
    const int tpt = kTrThreads / (16 * nt);
    const int nks = (kp + 31) / 32 * 8;
    const size_t lds = 2 * sizeof(T) * size_t(16) * nt * 3 * tr_row_stride<T>(nks);
    if (lds <= 128 * 1024 && (3 * kp + tpt - 1) / tpt <= 24) return {nt, 24};
    return {1, 0};
}

template <typename T, int NT, int PF, int NR>
void launch_translate_k(hipStream_t s, int mode, dim3 grid, size_t smem, int level, int periodic, int C, int kp,
                        int nrb, const T *ops, const int16_t *oct_lists, const int8_t *offsets, const T *src, T *dst,
                        int accumulate, int nsplit, T *part, const AdaptTr &ad) {
    const int nks = tr_nks(C);
    if (mode == 0)
        hipLaunchKernelGGL((k_translate<T, NR, NT, 0, PF>), grid, dim3(kTrThreads), smem, s, level, periodic,
                           C, kp, nrb, nks, ops, oct_lists, offsets, src, dst, accumulate, nsplit, part, ad);
    else if (mode == 1)
        hipLaunchKernelGGL((k_translate<T, NR, NT, 1, PF>), grid, dim3(kTrThreads), smem, s, level, periodic,
                           C, kp, nrb, nks, ops, oct_lists, offsets, src, dst, accumulate, 1, (T *)nullptr, ad);
    else
        hipLaunchKernelGGL((k_translate<T, NR, NT, 2, PF>), grid, dim3(kTrThreads), smem, s, level, periodic,
                           C, kp, nrb, nks, ops, oct_lists, offsets, src, dst, accumulate, 1, (T *)nullptr, ad);
}

template <typename T, int NT, int PF>
hipError_t launch_translate_rows(hipStream_t s, int mode, int nrbw, dim3 grid, size_t smem, int level,
                                 int periodic, int C, int kp, int nrb, const T *ops, const int16_t *oct_lists,
                                 const int8_t *offsets, const T *src, T *dst, int accumulate, int nsplit,
                                 T *part, const AdaptTr &ad = AdaptTr()) {
    switch (nrbw) {
        case 1: launch_translate_k<T, NT, PF, 1>(s, mode, grid, smem, level, periodic, C, kp, nrb, ops, oct_lists,
                                                 offsets, src, dst, accumulate, nsplit, part, ad); break;
        case 2: launch_translate_k<T, NT, PF, 2>(s, mode, grid, smem, level, periodic, C, kp, nrb, ops, oct_lists,
                                                 offsets, src, dst, accumulate, nsplit, part, ad); break;
        case 3: launch_translate_k<T, NT, PF, 3>(s, mode, grid, smem, level, periodic, C, kp, nrb, ops, oct_lists,
                                                 offsets, src, dst, accumulate, nsplit, part, ad); break;
        case 4: launch_translate_k<T, NT, PF, 4>(s, mode, grid, smem, level, periodic, C, kp, nrb, ops, oct_lists,
                                                 offsets, src, dst, accumulate, nsplit, part, ad); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Number of offset ranges an M2L launch at `level` is split into: enough
// workgroups to fill the chip, bounded by the partial-sum buffer.
constexpr int kTrFillWorkgroups = 1024;

int translate_splits(int level, int ttn, int kp, size_t part_elems) {
    const int64_t ncell = int64_t(1) << (3 * (level - 1));
    const int64_t wgs = (ncell + ttn - 1) / ttn * 8;
    if (wgs >= kTrFillWorkgroups) return 1;
    int ns = int((kTrFillWorkgroups + wgs - 1) / wgs);
    if (ns > 189) ns = 189;
    const size_t per_split = size_t(ncell) * 8 * 3 * kp;
    while (ns > 1 && size_t(ns) * per_split > part_elems) --ns;
    return ns;
}

hipError_t launch_split_reduce64(hipStream_t s, int level, int kp, int C, int nsplit, const double *part,
                                 double *dst, int accumulate) {
    const int64_t nelem = (int64_t(1) << (3 * level)) * 3 * kp;
    hipLaunchKernelGGL(k_split_reduce<double>, dim3(unsigned((nelem + 255) / 256)), dim3(256), 0, s, nelem, kp, C,
                       nsplit, part, dst, accumulate);
    return hipGetLastError();
}

hipError_t launch_split_reduce64_n(hipStream_t s, int64_t nelem, int kp, int C, int nsplit, const double *part,
                                   double *dst, int accumulate) {
    hipLaunchKernelGGL(k_split_reduce<double>, dim3(unsigned((nelem + 255) / 256)), dim3(256), 0, s, nelem, kp, C,
                       nsplit, part, dst, accumulate);
    return hipGetLastError();
}

hipError_t launch_split_reduce(hipStream_t s, int level, int kp, int C, int nsplit, const float *part, float *dst,
                               int accumulate) {
    const int64_t nelem = (int64_t(1) << (3 * level)) * 3 * kp;
    hipLaunchKernelGGL(k_split_reduce<float>, dim3(unsigned((nelem + 255) / 256)), dim3(256), 0, s, nelem, kp, C,
                       nsplit, part, dst, accumulate);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_translate(hipStream_t s, int mode, int level, int periodic, int p, int kp, const T *ops,
                            const int16_t *oct_lists, const int8_t *offsets, const T *src, T *dst,
                            int accumulate, T *part, size_t part_elems, const T *zero_cell, int tri) {
    const int C = (p + 1) * (p + 1);
    const int nrb = tr_nrb(C);
    const int nrbw = nrb / kTrWaves;
    const TrShape sh = translate_shape<T>(kp);
    const int ttn = 16 * sh.nt;
    int64_t ncell;
    int grid;
    if (mode == 2) {
        ncell = int64_t(1) << (3 * level);
        grid = int((ncell + ttn - 1) / ttn);
    } else {
        ncell = int64_t(1) << (3 * (level - 1));
        grid = int((ncell + ttn - 1) / ttn) * 8;
    }
    if constexpr (sizeof(T) == 4) {
        // operator-stationary M2L where its register and LDS budget allows
        const int nrbh = (pad16(C) / 16 + 1) / 2, nb = tr_nks(C) / 4;
        const bool os = mode == 0 && zero_cell != nullptr &&
                        ((nrbh == 4 && nb == 8) || (nrbh == 3 && nb == 6) || (nrbh <= 2 && nb == 4));
        if (os) {
            const int nsplit = part ? translate_splits(level, 64, kp, part_elems) : 1;
            T *pbuf = nsplit > 1 ? part : nullptr;
            const dim3 g3(unsigned((ncell + 63) / 64 * 8), unsigned(nsplit));
            const int nks = tr_nks(C);
            // truncated operators: k blocks each row block needs, and a split of the
            // row blocks over the two wave halves with balanced k blocks
            uint32_t rbmap = 0, kbmap = 0;
            if (tri) {
                int need[8], half_cost[2] = {0, 0}, half_n[2] = {0, 0};
                for (int rb = 0; rb < 2 * nrbh; ++rb) {
                    int nmin = 0;
                    while ((nmin + 1) * (nmin + 1) <= 16 * rb) ++nmin;
                    const int cols = 16 * rb < C ? (p - nmin + 1) * (p - nmin + 1) : 0;
                    need[rb] = std::min(nb, (cols + 15) / 16);
                }
                int order[8];
                for (int i = 0; i < 2 * nrbh; ++i) order[i] = i;
                std::stable_sort(order, order + 2 * nrbh, [&](int a, int b) { return need[a] > need[b]; });
                for (int k = 0; k < 2 * nrbh; ++k) {
                    const int rb = order[k];
                    int hh = half_cost[0] <= half_cost[1] ? 0 : 1;
                    if (half_n[hh] == nrbh) hh ^= 1;
                    const int slot = hh * nrbh + half_n[hh]++;
                    half_cost[hh] += need[rb];
                    rbmap |= uint32_t(rb) << (4 * slot);
                    kbmap |= uint32_t(need[rb]) << (4 * slot);
                }
            }
#define VM_M2L_OS(NRBH_, NB_)                                                                                  \
    do {                                                                                                        \
        const size_t smem = 2 * sizeof(float) * size_t(2 * NRBH_ * NB_ * 256);                                \
        if (tri)                                                                                                \
            hipLaunchKernelGGL((k_m2l_os<NRBH_, NB_, true>), g3, dim3(kTrThreads), smem, s, level, periodic, C, \
                               kp, nrb, nks, ops, oct_lists, offsets, src, dst, accumulate, nsplit, pbuf,      \
                               zero_cell, rbmap, kbmap);                                                        \
        else                                                                                                    \
            hipLaunchKernelGGL((k_m2l_os<NRBH_, NB_, false>), g3, dim3(kTrThreads), smem, s, level, periodic,   \
                               C, kp, nrb, nks, ops, oct_lists, offsets, src, dst, accumulate, nsplit, pbuf,   \
                               zero_cell, rbmap, kbmap);                                                        \
    } while (0)
            if (nb == 8) VM_M2L_OS(4, 8);
            else if (nb == 6) VM_M2L_OS(3, 6);
            else VM_M2L_OS(2, 4);
#undef VM_M2L_OS
            hipError_t e = hipGetLastError();
            if (e != hipSuccess || nsplit == 1) return e;
            const int64_t nelem = (int64_t(1) << (3 * level)) * 3 * kp;
            hipLaunchKernelGGL(k_split_reduce<T>, dim3(unsigned((nelem + 255) / 256)), dim3(256), 0, s, nelem, kp,
                               C, nsplit, (const T *)pbuf, dst, accumulate);
            return hipGetLastError();
        }
    }
    const int nsplit = (mode == 0 && part) ? translate_splits(level, ttn, kp, part_elems) : 1;
    T *pbuf = nsplit > 1 ? part : nullptr;
    const size_t smem = sizeof(T) * size_t(ttn) * 3 * tr_row_stride<T>(tr_nks(C)) * (sh.pf > 0 ? 2 : 1);
    constexpr int NTP = sizeof(T) == 4 ? 2 : 1;
    const dim3 g3(grid, nsplit);
    hipError_t e;
    if (sh.pf > 0)
        e = launch_translate_rows<T, NTP, 24>(s, mode, nrbw, g3, smem, level, periodic, C, kp, nrb, ops, oct_lists,
                                              offsets, src, dst, accumulate, nsplit, pbuf);
    else
        e = launch_translate_rows<T, 1, 0>(s, mode, nrbw, g3, smem, level, periodic, C, kp, nrb, ops, oct_lists,
                                           offsets, src, dst, accumulate, nsplit, pbuf);
    if (e != hipSuccess || nsplit == 1) return e;
    const int64_t nelem = (int64_t(1) << (3 * level)) * 3 * kp;
    hipLaunchKernelGGL(k_split_reduce<T>, dim3(unsigned((nelem + 255) / 256)), dim3(256), 0, s, nelem, kp, C,
                       nsplit, (const T *)pbuf, dst, accumulate);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_translate_adaptive(hipStream_t s, int mode, int p, int kp, const T *ops, const int16_t *oct_lists,
                                     const T *src, T *dst, int accumulate, const AdaptTr &ad, T *part,
                                     size_t part_elems) {
    const int C = (p + 1) * (p + 1);
    const int nrb = tr_nrb(C);
    const int nrbw = nrb / kTrWaves;
    const TrShape sh = translate_shape<T>(kp);
    const int ttn = 16 * sh.nt;
    AdaptTr a = ad;
    int grid;
    if (mode == 2) {
        grid = (a.ntarget + ttn - 1) / ttn;
    } else {
        a.tile_start[0] = 0;
        for (int o = 0; o < 8; ++o) a.tile_start[o + 1] = a.tile_start[o] + (a.oct_n[o] + ttn - 1) / ttn;
        grid = a.tile_start[8];
    }
    if (grid == 0) return hipSuccess;
    int nsplit = 1;
    if (mode == 0 && part != nullptr && a.part_cells > 0 && grid < kTrFillWorkgroups) {
        nsplit = (kTrFillWorkgroups + grid - 1) / grid;
        if (nsplit > 189) nsplit = 189;
        const size_t per_split = size_t(a.part_cells) * 3 * kp;
        while (nsplit > 1 && size_t(nsplit) * per_split > part_elems) --nsplit;
    }
    T *pbuf = nsplit > 1 ? part : nullptr;
    const size_t smem = sizeof(T) * size_t(ttn) * 3 * tr_row_stride<T>(tr_nks(C)) * (sh.pf > 0 ? 2 : 1);
    constexpr int NTP = sizeof(T) == 4 ? 2 : 1;
    const dim3 g3(grid, nsplit);
    hipError_t e;
    if (sh.pf > 0)
        e = launch_translate_rows<T, NTP, 24>(s, mode, nrbw, g3, smem, 0, 0, C, kp, nrb, ops, oct_lists, nullptr,
                                              src, dst, accumulate, nsplit, pbuf, a);
    else
        e = launch_translate_rows<T, 1, 0>(s, mode, nrbw, g3, smem, 0, 0, C, kp, nrb, ops, oct_lists, nullptr, src,
                                           dst, accumulate, nsplit, pbuf, a);
    if (e != hipSuccess || nsplit == 1) return e;
    const int64_t nelem = int64_t(a.part_cells) * 3 * kp;
    hipLaunchKernelGGL(k_split_reduce<T>, dim3(unsigned((nelem + 255) / 256)), dim3(256), 0, s, nelem, kp, C, nsplit,
                       (const T *)pbuf, dst + size_t(a.part_cell0) * 3 * kp, accumulate);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_lattice(hipStream_t s, int p, int kp, const double *tlat, const T *m0, T *l0) {
    const int C = (p + 1) * (p + 1);
    hipLaunchKernelGGL(k_lattice<T>, dim3(1), dim3(256), 0, s, C, kp, tlat, m0, l0);
    return hipGetLastError();
}

#define VM_INST(T)                                                                                          \
    template hipError_t launch_p2m<T>(hipStream_t, int, const void *, const int32_t *, int, int, double,    \
                                      const DevTables &, T *, const LeafMap &, T *, const int16_t *, int);  \
    template hipError_t launch_l2p<T>(hipStream_t, int, int, const void *, const int32_t *, int, int,       \
                                      double, double, const DevTables &, const T *, double *,               \
                                      const LeafMap &, const NearCombine &);                                \
    template hipError_t launch_translate<T>(hipStream_t, int, int, int, int, int, const T *,                \
                                            const int16_t *, const int8_t *, const T *, T *, int, T *,      \
                                            size_t, const T *, int);                                        \
    template hipError_t launch_lattice<T>(hipStream_t, int, int, const double *, const T *, T *);          \
    template hipError_t launch_translate_adaptive<T>(hipStream_t, int, int, int, const T *, const int16_t *,  \
                                                     const T *, T *, int, const AdaptTr &, T *, size_t);
VM_INST(double)
VM_INST(float)
#undef VM_INST

}  // namespace vmfmm
