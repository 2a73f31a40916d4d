// Uniform-octree build on the GPU: Morton keys, stable LSD radix sort of
// (key, particle index), dense leaf ranges and the permutation of the
// particles into leaf order.  All passes are bandwidth-bound; the key
// arithmetic follows the documented reading bit for bit (no fused
// multiply-add in the wrap or the cell index).
#include "kernels.h"

namespace vmfmm {

namespace {

__device__ __forceinline__ double wrap_coord(double x, double lo, double len, double inv_len) {
#pragma clang fp contract(off)
    const double s = floor((x - lo) * inv_len);
    const double t = s * len;
    return x - t;
}

__device__ __forceinline__ int cell_coord(double xw, double lo, double inv_w, int side) {
#pragma clang fp contract(off)
    const double c = floor((xw - lo) * inv_w);
    if (!(c >= 0.0)) return 0;            // also catches NaN
    if (c > double(side - 1)) return side - 1;
    return int(c);
}

__device__ __forceinline__ uint32_t interleave(int cx, int cy, int cz, int level) {
    uint32_t k = 0;
    for (int b = 0; b < level; ++b) {
        k |= uint32_t((cx >> b) & 1) << (3 * b);
        k |= uint32_t((cy >> b) & 1) << (3 * b + 1);
        k |= uint32_t((cz >> b) & 1) << (3 * b + 2);
    }
    return k;
}

__device__ __forceinline__ int deinterleave(uint32_t k, int d, int level) {
    int c = 0;
    for (int b = 0; b < level; ++b) c |= int((k >> (3 * b + d)) & 1u) << b;
    return c;
}

__global__ void __launch_bounds__(256) k_keys(int n, const double *__restrict__ x, TreeGeom g, int check,
                                              uint32_t *__restrict__ keys, int32_t *__restrict__ idx,
                                              int *__restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int side = 1 << g.level;
    int c[3];
    bool bad = false;
    for (int d = 0; d < 3; ++d) {
        const double x0 = x[size_t(d) * n + i];
        double xv = x0;
        if (g.periodic) xv = wrap_coord(x0, g.lo[d], g.box_len, g.inv_len);
        c[d] = cell_coord(xv, g.lo[d], g.inv_w, side);
        if (check) {
            if (!isfinite(x0)) bad = true;
            if (!g.periodic && !(x0 >= g.lo[d] && x0 <= g.lo[d] + g.box_len)) bad = true;
        }
    }
    if (bad) atomicOr(flag, 1);
    keys[i] = interleave(c[0], c[1], c[2], g.level);
    idx[i] = i;
}

__global__ void __launch_bounds__(256) k_iota(int n, int32_t *__restrict__ idx, uint32_t *__restrict__ keys) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        idx[i] = i;
        keys[i] = 0u;
    }
}

// Per-tile digit histogram: hist[digit * nblocks + block].
__global__ void __launch_bounds__(kRadixThreads) k_radix_hist(int n, int shift, int bits,
                                                             const uint32_t *__restrict__ keys,
                                                             uint32_t *__restrict__ hist) {
    __shared__ uint32_t cnt[256];
    const int nb = 1 << bits;
    for (int b = threadIdx.x; b < nb; b += kRadixThreads) cnt[b] = 0;
    __syncthreads();
    const int base = blockIdx.x * kRadixTile;
    const uint32_t mask = uint32_t(nb - 1);
    for (int it = 0; it < kRadixItems; ++it) {
        const int e = base + it * kRadixThreads + threadIdx.x;
        if (e < n) atomicAdd(&cnt[(keys[e] >> shift) & mask], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += kRadixThreads) hist[size_t(b) * gridDim.x + blockIdx.x] = cnt[b];
}

// Exclusive scan of `total` counts in three coalesced steps: each block scans
// a tile of kScanTile entries and records the tile total; one block scans the
// totals; each block adds its tile's offset.
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *sh, uint32_t &total) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const uint32_t w = t >= off ? sh[t - off] : 0u;
        __syncthreads();
        sh[t] += w;
        __syncthreads();
    }
    total = sh[kScanThreads - 1];
    const uint32_t excl = sh[t] - v;
    __syncthreads();
    return excl;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(int total, uint32_t *__restrict__ data,
                                                            uint32_t *__restrict__ tile_sums) {
    __shared__ uint32_t sh[kScanThreads];
    const int base = blockIdx.x * kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < total ? data[base + i] : 0u;
        s += v[i];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, sh, tot);
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < total) data[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_sums(int ntiles, uint32_t *__restrict__ tile_sums) {
    __shared__ uint32_t sh[kScanThreads];
    uint32_t carry = 0;
    for (int b = 0; b < ntiles; b += kScanThreads) {
        const int i = b + threadIdx.x;
        const uint32_t v = i < ntiles ? tile_sums[i] : 0u;
        uint32_t tot;
        const uint32_t e = block_exclusive_scan(v, sh, tot);
        if (i < ntiles) tile_sums[i] = carry + e;
        carry += tot;
    }
}

__global__ void __launch_bounds__(kScanThreads) k_scan_add(int total, uint32_t *__restrict__ data,
                                                          const uint32_t *__restrict__ tile_sums) {
    const uint32_t off = tile_sums[blockIdx.x];
    const int base = blockIdx.x * kScanTile;
    for (int i = threadIdx.x; i < kScanTile; i += kScanThreads)
        if (base + i < total) data[base + i] += off;
}

// Stable scatter: wave w of a block owns the contiguous quarter of its tile,
// processed in rounds of 64 consecutive keys; ranks among equal digits come
// from ballots, so equal keys keep their input order.
__global__ void __launch_bounds__(kRadixThreads) k_radix_scatter(int n, int shift, int bits,
                                                                const uint32_t *__restrict__ kin,
                                                                const int32_t *__restrict__ vin,
                                                                uint32_t *__restrict__ kout,
                                                                int32_t *__restrict__ vout,
                                                                const uint32_t *__restrict__ offs) {
    __shared__ uint32_t whist[kRadixThreads / 64][256];
    const int nb = 1 << bits;
    const uint32_t mask = uint32_t(nb - 1);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int b = threadIdx.x; b < 4 * 256; b += kRadixThreads) (&whist[0][0])[b] = 0;
    __syncthreads();
    const int base = blockIdx.x * kRadixTile + wave * (kRadixItems * 64);
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    uint32_t key[kRadixItems];
    int32_t val[kRadixItems];
    uint32_t rank[kRadixItems];
#pragma unroll
    for (int it = 0; it < kRadixItems; ++it) {
        const int e = base + it * 64 + lane;
        const bool valid = e < n;
        const uint32_t k = valid ? kin[e] : 0u;
        const uint32_t d = (k >> shift) & mask;
        uint64_t m = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            m &= bit ? bb : ~bb;
        }
        const uint32_t r = __popcll(m & lt);
        const uint32_t prev = valid ? whist[wave][d] : 0u;
        // all lanes have read `prev` before the leader (lowest lane of the
        // group) stores: the store depends on the loaded value
        if (valid && r == 0) whist[wave][d] = prev + uint32_t(__popcll(m));
        key[it] = k;
        val[it] = valid ? vin[e] : 0;
        rank[it] = prev + r;
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += kRadixThreads) {
        uint32_t s = offs[size_t(b) * gridDim.x + blockIdx.x];
        for (int w = 0; w < kRadixThreads / 64; ++w) {
            const uint32_t t = whist[w][b];
            whist[w][b] = s;
            s += t;
        }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < kRadixItems; ++it) {
        const int e = base + it * 64 + lane;
        if (e < n) {
            const uint32_t d = (key[it] >> shift) & mask;
            const uint32_t pos = whist[wave][d] + rank[it];
            if (pos < uint32_t(n)) {   // always true for a consistent histogram
                kout[pos] = key[it];
                vout[pos] = val[it];
            }
        }
    }
}

// start[c] = first sorted index with key >= c, for c = 0..nleaf (start[nleaf] = n).
__global__ void __launch_bounds__(256) k_ranges(int n, int nleaf, const uint32_t *__restrict__ keys,
                                                int32_t *__restrict__ start) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t k = keys[i];
    const int64_t kp = i == 0 ? -1 : int64_t(keys[i - 1]);
    for (int64_t c = kp + 1; c <= k; ++c) start[c] = i;
    if (i == n - 1)
        for (int64_t c = k + 1; c <= nleaf; ++c) start[c] = n;
}

__global__ void __launch_bounds__(256) k_permute(int n, const double *__restrict__ x,
                                                 const double *__restrict__ alpha,
                                                 const int32_t *__restrict__ perm,
                                                 const uint32_t *__restrict__ keys, TreeGeom g,
                                                 Part64 *__restrict__ p64, Part32 *__restrict__ p32) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int j = perm[i];
    if (j < 0 || j >= n) return;   // never for a valid permutation
    const uint32_t k = keys[i];
    double dl[3], al[3];
    for (int d = 0; d < 3; ++d) {
        double xv = x[size_t(d) * n + j];
        if (g.periodic) xv = wrap_coord(xv, g.lo[d], g.box_len, g.inv_len);
        const int c = deinterleave(k, d, g.level);
        const double centre = g.lo[d] + (double(c) + 0.5) * g.w;
        dl[d] = xv - centre;
        al[d] = alpha[size_t(d) * n + j];
    }
    if (p64) {
        Part64 r;
        r.dx = dl[0]; r.dy = dl[1]; r.dz = dl[2];
        r.ax = al[0]; r.ay = al[1]; r.az = al[2];
        r.pad0 = 0.0; r.pad1 = 0.0;
        p64[i] = r;
    }
    if (p32) {
        Part32 r;
        r.dx = float(dl[0]); r.dy = float(dl[1]); r.dz = float(dl[2]);
        r.ax = float(al[0]); r.ay = float(al[1]); r.az = float(al[2]);
        r.pad0 = 0.0f; r.pad1 = 0.0f;
        p32[i] = r;
    }
}

inline int blocks(int n, int t) { return (n + t - 1) / t; }

}  // namespace

hipError_t launch_keys(hipStream_t s, int n, const double *x, const TreeGeom &g, int check,
                       uint32_t *keys, int32_t *idx, int *flag) {
    hipLaunchKernelGGL(k_keys, dim3(blocks(n, 256)), dim3(256), 0, s, n, x, g, check, keys, idx, flag);
    return hipGetLastError();
}

hipError_t launch_iota(hipStream_t s, int n, int32_t *idx, uint32_t *keys) {
    hipLaunchKernelGGL(k_iota, dim3(blocks(n, 256)), dim3(256), 0, s, n, idx, keys);
    return hipGetLastError();
}

hipError_t launch_radix_pass(hipStream_t s, int n, int shift, int bits, const uint32_t *kin,
                             const int32_t *vin, uint32_t *kout, int32_t *vout, uint32_t *hist) {
    const int nblk = blocks(n, kRadixTile);
    hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(kRadixThreads), 0, s, n, shift, bits, kin, hist);
    const int total = nblk << bits;
    const int ntiles = (total + kScanTile - 1) / kScanTile;
    uint32_t *tile_sums = hist + size_t(nblk) * 256;   // the histogram buffer carries room for the tile sums
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kScanThreads), 0, s, total, hist, tile_sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, ntiles, tile_sums);
    hipLaunchKernelGGL(k_scan_add, dim3(ntiles), dim3(kScanThreads), 0, s, total, hist, (const uint32_t *)tile_sums);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(kRadixThreads), 0, s, n, shift, bits, kin, vin,
                       kout, vout, (const uint32_t *)hist);
    return hipGetLastError();
}

hipError_t launch_exclusive_scan(hipStream_t s, int total, uint32_t *data, uint32_t *tile_sums) {
    if (total <= 0) return hipSuccess;
    const int ntiles = (total + kScanTile - 1) / kScanTile;
    hipLaunchKernelGGL(k_scan_tiles, dim3(ntiles), dim3(kScanThreads), 0, s, total, data, tile_sums);
    hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(kScanThreads), 0, s, ntiles, tile_sums);
    hipLaunchKernelGGL(k_scan_add, dim3(ntiles), dim3(kScanThreads), 0, s, total, data, (const uint32_t *)tile_sums);
    return hipGetLastError();
}

hipError_t launch_ranges(hipStream_t s, int n, int nleaf, const uint32_t *keys, int32_t *start) {
    hipLaunchKernelGGL(k_ranges, dim3(blocks(n, 256)), dim3(256), 0, s, n, nleaf, keys, start);
    return hipGetLastError();
}

hipError_t launch_permute(hipStream_t s, int n, const double *x, const double *alpha,
                          const int32_t *perm, const uint32_t *keys, const TreeGeom &g,
                          Part64 *p64, Part32 *p32) {
    hipLaunchKernelGGL(k_permute, dim3(blocks(n, 256)), dim3(256), 0, s, n, x, alpha, perm, keys, g, p64, p32);
    return hipGetLastError();
}

}  // namespace vmfmm
