// Near field (P2P): exact regularised Biot-Savart velocity and gradient over
// the 27 adjacent leaves (paper Sec. 3.1, last paragraph; kernel eqs. 5-8).
//
// One wave per target leaf, one target particle per lane.  Source particles
// are read at wave-uniform addresses, so they arrive through scalar loads and
// sit in SGPRs: every lane of the wave works on the same source at the same
// time with no LDS traffic.  The pair kernel, with r = x_i - x_j and rho = r/sigma:
//   q      = g(rho) / r^3,  g = erf(rho/sqrt2) - sqrt(2/pi) rho exp(-rho^2/2)
//   q'/r   = (sqrt(2/pi) sigma^-3 exp(-rho^2/2) - 3 q) / r^2
//   u     += q alpha_j x r
//   J[a][b] += (q'/r) r_a (alpha_j x r)_b + q eps_abc alpha_j,c
// For small rho both q and q'/r are even power series in rho (g is the
// integral of the Gaussian mass, g' = sqrt(2/pi) rho^2 exp(-rho^2/2)).
// A leaf's last target block of 32 or fewer particles is split over lane
// groups that share out the sources.  The epilogue adds the far field
// computed by L2P, contracts the gradient into the stretching term and
// scatters to the caller's particle order.
#include "kernels.h"

namespace vmfmm {

namespace {

constexpr double kInv4Pi = 0.079577471545947667884441881686257181;
constexpr double kSqrt2OverPi = 0.79788456080286535587989211986876373;

// a_n = (-1/2)^n / (n! (2n+3)): g / rho^3 = sqrt(2/pi) sum a_n rho^{2n}
// Horner in t = rho^2 over n = 0..NTERM-1; h1 = 2 d(h0)/dt = sum 2 n a_n t^{n-1}.
template <typename T, int NTERM>
__device__ __forceinline__ void small_rho(T t, T &h0, T &h1) {
    static_assert(NTERM >= 3 && NTERM <= 14, "series length");
    constexpr double a[14] = {
        1.0 / 3.0,
        -0.5 / 5.0,
        0.25 / (2.0 * 7.0),
        -0.125 / (6.0 * 9.0),
        0.0625 / (24.0 * 11.0),
        -0.03125 / (120.0 * 13.0),
        0.015625 / (720.0 * 15.0),
        -0.0078125 / (5040.0 * 17.0),
        0.00390625 / (40320.0 * 19.0),
        -0.001953125 / (362880.0 * 21.0),
        0.0009765625 / (3628800.0 * 23.0),
        -0.00048828125 / (39916800.0 * 25.0),
        0.000244140625 / (479001600.0 * 27.0),
        -0.0001220703125 / (6227020800.0 * 29.0),
    };
    constexpr int top = NTERM - 1;
    T s0 = T(a[top]), s1 = T(2.0 * top * a[top]);
#pragma unroll
    for (int k = top - 1; k >= 1; --k) {
        s0 = s0 * t + T(a[k]);
        s1 = s1 * t + T(2.0 * k * a[k]);
    }
    h0 = s0 * t + T(a[0]);
    h1 = s1;
}

struct Consts64 {
    double inv_sigma, inv_s2, is3, is5, thr2;
};

__device__ __forceinline__ void pair64(double r2, const Consts64 &k, double &q, double &dq) {
    if (r2 >= k.thr2) {
        const double rinv = 1.0 / sqrt(r2);
        const double r = r2 * rinv;
        const double rho = r * k.inv_sigma;
        const double e = exp(-0.5 * rho * rho);
        const double g = erf(rho * 0.70710678118654752440084436210484903) - kSqrt2OverPi * rho * e;
        const double ir2 = rinv * rinv;
        q = g * ir2 * rinv;
        dq = (kSqrt2OverPi * k.is3 * e - 3.0 * q) * ir2;
    } else {
        double h0, h1;
        small_rho<double, 9>(r2 * k.inv_s2, h0, h1);
        q = kSqrt2OverPi * k.is3 * h0;
        dq = kSqrt2OverPi * k.is5 * h1;
    }
}

struct Consts32 {
    float inv_s2, thr2;
    float ka;          // p / (sqrt2 sigma): t = 1 / (1 + ka r)
    float ke;          // -log2(e) / (2 sigma^2): exp(-rho^2/2) = 2^(ke r^2)
    float ks;          // sqrt(2/pi) / sigma: sqrt(2/pi) rho = ks r
    float kd;          // sqrt(2/pi) / sigma^3
    float kd5;         // sqrt(2/pi) / sigma^5
};

__device__ __forceinline__ Consts32 consts32(double sigma) {
    const double is = 1.0 / sigma;
    Consts32 k;
    k.inv_s2 = float(is * is);
    k.thr2 = float(sigma * sigma);
    k.ka = float(0.3275911 * 0.70710678118654752440 * is);
    k.ke = float(-0.5 * 1.4426950408889634074 * is * is);
    k.ks = float(kSqrt2OverPi * is);
    k.kd = float(kSqrt2OverPi * is * is * is);
    k.kd5 = float(kSqrt2OverPi * is * is * is * is * is);
    return k;
}

// FP32 pair kernel.  For rho < 1 the series (9 terms, truncation < 1e-9
// relative) is used; beyond, the erf of Abramowitz & Stegun 7.1.26
// (|error| <= 1.5e-7), whose exp(-s^2) factor is shared with the Gaussian term:
//   1 - g = exp(-rho^2/2) (P(t) + sqrt(2/pi) rho),  t = 1 / (1 + p rho/sqrt2);
// at rho >= 1 that gives q to 6e-7 and q'/r to 2e-6 relative.  The series
// branch diverges within a wave whenever one lane is close to the source, so
// its threshold is kept as small as that accuracy allows.  1/sigma is folded
// into the constants; the Gaussian is one hardware exp2 of r^2 ke, the
// reciprocal the hardware one (1 ulp, far below the approximation's error).
__device__ __forceinline__ void pair32(float r2, const Consts32 &k, float &q, float &dq) {
    if (r2 >= k.thr2) {
        const float rinv = __frsqrt_rn(r2);
        const float r = r2 * rinv;
        const float e = __builtin_amdgcn_exp2f(r2 * k.ke);
        const float t = __builtin_amdgcn_rcpf(fmaf(k.ka, r, 1.0f));
        const float poly = t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
        const float g = fmaf(-e, fmaf(k.ks, r, poly), 1.0f);
        const float ir2 = rinv * rinv;
        q = g * rinv * ir2;
        dq = fmaf(k.kd, e, -3.0f * q) * ir2;
    } else {
        float h0, h1;
        small_rho<float, 9>(r2 * k.inv_s2, h0, h1);
        q = k.kd * h0;
        dq = k.kd5 * h1;
    }
}

__device__ __forceinline__ int demorton(int k, int d, int level) {
    int c = 0;
    for (int b = 0; b < level; ++b) c |= ((k >> (3 * b + d)) & 1) << b;
    return c;
}

__device__ __forceinline__ int morton(int cx, int cy, int cz, int level) {
    int k = 0;
    for (int b = 0; b < level; ++b)
        k |= (((cx >> b) & 1) << (3 * b)) | (((cy >> b) & 1) << (3 * b + 1)) | (((cz >> b) & 1) << (3 * b + 2));
    return k;
}

// Writes u, dalpha/dt and J for sorted particle gi (caller index oi) from the
// near sums (velocity us - uc, rank-one gradient part Jr, S = sum q alpha) plus
// the far field.  Every near value passes through `red` on its way (the
// identity, or the sum over the lane groups of a split target block: then all
// lanes run this, and only those with `write` set store).  Streamed value by
// value, J row by row with the stretching contraction accumulated on the way,
// so that few values are live at once: the kernels' register budget, hence
// their occupancy, is set here.
template <typename A, typename R>
__device__ __forceinline__ void epilogue(const P2PArgs &a, int gi, bool write, const A us[3], const A uc[3],
                                         const A Jr[9], const A S[3], R red) {
    const size_t n = size_t(a.n);
    const int oi = write ? a.perm[gi] : 0;
    for (int b = 0; b < 3; ++b) {
        double u = red(double(us[b]) - double(uc[b])) * kInv4Pi;
        if (write) {
            if (a.have_far) u += a.far[b * n + gi];
            a.u[b * n + oi] = u;
        }
    }
    if (!a.grad && !a.dalpha) return;
    double Sd[3];
    for (int c = 0; c < 3; ++c) Sd[c] = red(double(S[c]));
    double al[3] = {0.0, 0.0, 0.0};
    if (write && a.dalpha)
        for (int c = 0; c < 3; ++c) al[c] = a.alpha[c * n + oi];
    double da[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            // antisymmetric part eps_abc S_c of the near gradient J[r][c]
            const int k = 3 - r - c;
            const double anti = r == c ? 0.0 : ((c == (r + 1) % 3) ? Sd[k] : -Sd[k]);
            double J = (red(double(Jr[3 * r + c])) + anti) * kInv4Pi;
            if (write) {
                if (a.have_far) J += a.far[(3 + 3 * r + c) * n + gi];
                if (a.grad) a.grad[(3 * r + c) * n + oi] = J;
            }
            if (a.scheme == 0) da[c] += al[r] * J;      // classic: sum_a alpha_a J[a][b]
            else da[r] += J * al[c];                     // transpose: sum_c J[b][c] alpha_c
        }
    }
    if (write && a.dalpha)
        for (int b = 0; b < 3; ++b) a.dalpha[b * n + oi] = da[b];
}

struct NoReduce {
    __device__ double operator()(double v) const { return v; }
};

// sum over the lane groups of a split block (lanes l, l ^ E, l ^ 2E, ...), fixed order
struct GroupSum {
    int E;
    __device__ double operator()(double v) const {
        for (int off = E; off < 64; off <<= 1) v += __shfl_xor(v, off);
        return v;
    }
};

// Target blocks of a leaf: whole blocks of 64 targets, one target per lane, take
// every source at a wave-uniform address (scalar loads).  A last block of
// rem <= 32 targets would leave most lanes idle, so there the wave splits into
// g = 64 / E lane groups (E = rem rounded up to a power of two): lane group k
// takes target t = lane % E against every g-th source of each neighbour leaf,
// and the groups' partial sums are combined in FP64 by a fixed butterfly.
__device__ __forceinline__ int pow2_ceil(int v) {
    int e = 1;
    while (e < v) e <<= 1;
    return e;
}

struct LeafGeom {
    int cx, cy, cz, side;
};

// neighbour nb of the target leaf: source range and the offset d (source - target cell)
__device__ __forceinline__ bool neighbour(const P2PArgs &a, const LeafGeom &L, int nb, int &js, int &je, int &dx,
                                          int &dy, int &dz) {
    dx = nb % 3 - 1;
    dy = (nb / 3) % 3 - 1;
    dz = nb / 9 - 1;
    int nx = L.cx + dx, ny = L.cy + dy, nz = L.cz + dz;
    if (a.periodic) {
        nx = (nx + L.side) % L.side;
        ny = (ny + L.side) % L.side;
        nz = (nz + L.side) % L.side;
    } else if (nx < 0 || ny < 0 || nz < 0 || nx >= L.side || ny >= L.side || nz >= L.side) {
        return false;
    }
    const int nk = morton(nx, ny, nz, a.level);
    js = a.start[nk];
    je = a.start[nk + 1];
    return true;
}

__device__ __forceinline__ void acc64(const Part64 &s, double tx, double ty, double tz, const Consts64 &k,
                                      double u[3], double Jr[9], double S[3]) {
    const double rx = tx - s.dx, ry = ty - s.dy, rz = tz - s.dz;
    const double r2 = rx * rx + ry * ry + rz * rz;
    double q, dq;
    pair64(r2, k, q, dq);
    const double c0 = s.ay * rz - s.az * ry;
    const double c1 = s.az * rx - s.ax * rz;
    const double c2 = s.ax * ry - s.ay * rx;
    u[0] += q * c0;
    u[1] += q * c1;
    u[2] += q * c2;
    S[0] += q * s.ax;
    S[1] += q * s.ay;
    S[2] += q * s.az;
    const double t0 = dq * c0, t1 = dq * c1, t2 = dq * c2;
    Jr[0] += rx * t0; Jr[1] += rx * t1; Jr[2] += rx * t2;
    Jr[3] += ry * t0; Jr[4] += ry * t1; Jr[5] += ry * t2;
    Jr[6] += rz * t0; Jr[7] += rz * t1; Jr[8] += rz * t2;
}

// Workgroups are handed to the 8 XCDs round-robin; leaf (blockIdx mod 8) *
// nleaf/8 + blockIdx/8 gives each XCD one contiguous Morton range, whose
// neighbour leaves its L2 then shares.
__device__ __forceinline__ int xcd_leaf(int nleaf) {
    const int b = blockIdx.x;
    if (nleaf % 8 != 0) return b;
    return (b & 7) * (nleaf >> 3) + (b >> 3);
}

__global__ void __launch_bounds__(64) k_p2p64(P2PArgs a, const Part64 *__restrict__ parts) {
    const int leaf = xcd_leaf(a.nleaf), lane = threadIdx.x;
    const int s0 = a.start[leaf], cnt = a.start[leaf + 1] - s0;
    if (cnt == 0) return;
    LeafGeom L;
    L.side = 1 << a.level;
    L.cx = demorton(leaf, 0, a.level);
    L.cy = demorton(leaf, 1, a.level);
    L.cz = demorton(leaf, 2, a.level);
    Consts64 k;
    k.inv_sigma = 1.0 / a.sigma;
    k.inv_s2 = k.inv_sigma * k.inv_sigma;
    k.is3 = k.inv_s2 * k.inv_sigma;
    k.is5 = k.is3 * k.inv_s2;
    k.thr2 = 0.0625 * a.sigma * a.sigma;
    const double zero[3] = {0.0, 0.0, 0.0};
    // whole-wave blocks: one target per lane, wave-uniform sources
    const int nfull = cnt - cnt % 64 + (cnt % 64 > 32 ? 64 : 0);
    for (int base = 0; base < nfull; base += 64) {
        const int rem = cnt - base;
        const bool valid = lane < rem;
        const Part64 me = parts[s0 + base + (valid ? lane : 0)];
        double u[3] = {0, 0, 0}, Jr[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, S[3] = {0, 0, 0};
        for (int nb = 0; nb < 27; ++nb) {
            int js, je, dx, dy, dz;
            if (!neighbour(a, L, nb, js, je, dx, dy, dz)) continue;
            // x_i - x_j = (delta_i - d w) - delta_j, d = source - target cell offset
            const double tx = me.dx - dx * a.w, ty = me.dy - dy * a.w, tz = me.dz - dz * a.w;
            for (int j = js; j < je; ++j) acc64(parts[j], tx, ty, tz, k, u, Jr, S);
        }
        if (valid) epilogue(a, s0 + base + lane, true, u, zero, Jr, S, NoReduce{});
    }
    // a last block of rem <= 32 targets: lane groups share out the sources
    const int rem = cnt - nfull;
    if (rem <= 0) return;
    const int E = pow2_ceil(rem);
    const int t = lane & (E - 1), gi = lane / E, ng = 64 / E;
    const bool valid = t < rem;
    const Part64 me = parts[s0 + nfull + (valid ? t : 0)];
    double u[3] = {0, 0, 0}, Jr[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, S[3] = {0, 0, 0};
    for (int nb = 0; nb < 27; ++nb) {
        int js, je, dx, dy, dz;
        if (!neighbour(a, L, nb, js, je, dx, dy, dz)) continue;
        const double tx = me.dx - dx * a.w, ty = me.dy - dy * a.w, tz = me.dz - dz * a.w;
#pragma unroll 1
        for (int j = js + gi; j < je; j += ng) acc64(parts[j], tx, ty, tz, k, u, Jr, S);
    }
    epilogue(a, s0 + nfull + t, valid && gi == 0, u, zero, Jr, S, GroupSum{E});
}

struct Acc32 {
    float us[3], uc[3], Jr[9], S[3];
};

__device__ __forceinline__ void acc32(const Part32 &s, float tx, float ty, float tz, const Consts32 &k, Acc32 &A) {
    const float rx = tx - s.dx, ry = ty - s.dy, rz = tz - s.dz;
    const float r2 = rx * rx + ry * ry + rz * rz;
    float q, dq;
    pair32(r2, k, q, dq);
    const float c[3] = {s.ay * rz - s.az * ry, s.az * rx - s.ax * rz, s.ax * ry - s.ay * rx};
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        const float y = q * c[b] - A.uc[b];
        const float t = A.us[b] + y;
        A.uc[b] = (t - A.us[b]) - y;
        A.us[b] = t;
    }
    A.S[0] += q * s.ax;
    A.S[1] += q * s.ay;
    A.S[2] += q * s.az;
    const float t0 = dq * c[0], t1 = dq * c[1], t2 = dq * c[2];
    A.Jr[0] += rx * t0; A.Jr[1] += rx * t1; A.Jr[2] += rx * t2;
    A.Jr[3] += ry * t0; A.Jr[4] += ry * t1; A.Jr[5] += ry * t2;
    A.Jr[6] += rz * t0; A.Jr[7] += rz * t1; A.Jr[8] += rz * t2;
}

// Mixed precision: FP32 pair arithmetic, Kahan-compensated velocity sums.
__global__ void __launch_bounds__(64) k_p2p32(P2PArgs a, const Part32 *__restrict__ parts) {
    const int leaf = xcd_leaf(a.nleaf), lane = threadIdx.x;
    const int s0 = a.start[leaf], cnt = a.start[leaf + 1] - s0;
    if (cnt == 0) return;
    LeafGeom L;
    L.side = 1 << a.level;
    L.cx = demorton(leaf, 0, a.level);
    L.cy = demorton(leaf, 1, a.level);
    L.cz = demorton(leaf, 2, a.level);
    const Consts32 k = consts32(a.sigma);
    const float w = float(a.w);
    // whole-wave blocks: one target per lane, wave-uniform sources
    const int nfull = cnt - cnt % 64 + (cnt % 64 > 32 ? 64 : 0);
    for (int base = 0; base < nfull; base += 64) {
        const int rem = cnt - base;
        const bool valid = lane < rem;
        const Part32 me = parts[s0 + base + (valid ? lane : 0)];
        Acc32 A;
        for (int c = 0; c < 3; ++c) A.us[c] = A.uc[c] = A.S[c] = 0.0f;
        for (int c = 0; c < 9; ++c) A.Jr[c] = 0.0f;
        for (int nb = 0; nb < 27; ++nb) {
            int js, je, dx, dy, dz;
            if (!neighbour(a, L, nb, js, je, dx, dy, dz) || js >= je) continue;
            const float tx = me.dx - float(dx) * w, ty = me.dy - float(dy) * w, tz = me.dz - float(dz) * w;
            // the next record is fetched (scalar load) while the current one is evaluated
            Part32 cur = parts[js];
#pragma unroll 2
            for (int j = js; j < je; ++j) {
                const Part32 nxt = parts[j + 1 < je ? j + 1 : j];
                acc32(cur, tx, ty, tz, k, A);
                cur = nxt;
            }
        }
        if (valid) epilogue(a, s0 + base + lane, true, A.us, A.uc, A.Jr, A.S, NoReduce{});
    }
    // a last block of rem <= 32 targets: lane groups share out the sources, their
    // partial sums are combined in FP64
    const int rem = cnt - nfull;
    if (rem <= 0) return;
    const int E = pow2_ceil(rem);
    const int t = lane & (E - 1), gi = lane / E, ng = 64 / E;
    const bool valid = t < rem;
    const Part32 me = parts[s0 + nfull + (valid ? t : 0)];
    Acc32 A;
    for (int c = 0; c < 3; ++c) A.us[c] = A.uc[c] = A.S[c] = 0.0f;
    for (int c = 0; c < 9; ++c) A.Jr[c] = 0.0f;
    for (int nb = 0; nb < 27; ++nb) {
        int js, je, dx, dy, dz;
        if (!neighbour(a, L, nb, js, je, dx, dy, dz)) continue;
        const float tx = me.dx - float(dx) * w, ty = me.dy - float(dy) * w, tz = me.dz - float(dz) * w;
#pragma unroll 1
        for (int j = js + gi; j < je; j += ng) acc32(parts[j], tx, ty, tz, k, A);
    }
    epilogue(a, s0 + nfull + t, valid && gi == 0, A.us, A.uc, A.Jr, A.S, GroupSum{E});
}

}  // namespace

hipError_t launch_p2p64(hipStream_t s, const P2PArgs &a, const Part64 *parts) {
    hipLaunchKernelGGL(k_p2p64, dim3(a.nleaf), dim3(64), 0, s, a, parts);
    return hipGetLastError();
}

hipError_t launch_p2p32(hipStream_t s, const P2PArgs &a, const Part32 *parts) {
    hipLaunchKernelGGL(k_p2p32, dim3(a.nleaf), dim3(64), 0, s, a, parts);
    return hipGetLastError();
}

}  // namespace vmfmm
