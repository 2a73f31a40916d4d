// M2L in FP32 by reflection orbits (paper Sec. 3.1, eq. 11: the multipole-to-
// local translation of the interaction list).
//
// The 189 offsets of an octant's interaction list fall into 56 orbits under
// the reflections of the axes along which the list is symmetric; all offsets
// of an orbit share one operator up to the sign matrices P_R (kernels.h).  A
// target's local expansion is then
//   L_a += sum_orbits sum_b T_ab Y_{a^b, b},  Y_{x, b} = sum_R chi_x(R) M_{R d, b},
// where a, b run over the coefficient classes, d is the orbit's representative
// and R its reflections: one operator application per orbit instead of one per
// offset, and blocks T_ab with a ^ b along an axis where d is zero vanish.  The
// octant's own reflection is folded into per-octant operator copies.
//
// Work split: a workgroup of 12 waves takes 64 same-octant target cells; wave
// w serves targets 16 (w / 3) .. +15 and component w % 3, so no source is
// loaded twice.  Per orbit the operator's nonzero blocks sit in LDS (two
// buffers: the next orbit's copy is spread over the current orbit's k blocks,
// one barrier per orbit).  Per k block a lane loads its target's sources of
// the orbit's members (one 16-byte quad each), transforms them in registers
// and feeds the class blocks of the block's column to the MFMAs; the next k
// block's sources are loaded before the MFMAs of the current one.
#include "kernels.h"

#include <type_traits>

namespace vmfmm {
namespace {


template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<N, I + 1>(f);
    }
}

// bits of v (< 2^10) spread to every third bit
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ __forceinline__ uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v | (v >> 2)) & 0x030c30c3u;
    v = (v | (v >> 4)) & 0x0300f00fu;
    v = (v | (v >> 8)) & 0x030000ffu;
    v = (v | (v >> 16)) & 0x3ffu;
    return v;
}

// Elements [0, npack) from M (cell-major, 3 components of kc), then the 3 kc
// elements of the zero cell at element zero_off.
template <typename T>
__global__ void __launch_bounds__(256) k_sym_pack(int64_t npack, int64_t zero_off, int kp, int kc,
                                                  const T *__restrict__ M, const int16_t *__restrict__ mc_src,
                                                  T *__restrict__ Mc) {
    const int64_t e = int64_t(blockIdx.x) * 256 + threadIdx.x;
    if (e >= npack + 3 * kc) return;
    if (e >= npack) {
        Mc[zero_off + (e - npack)] = T(0);
        return;
    }
    const int q = int(e % kc);
    const int64_t cc = e / kc;   // cell * 3 + component
    const int src = mc_src[q];
    Mc[e] = src >= 0 ? M[cc * kp + src] : T(0);
}

constexpr int kSymWaves = 12;
constexpr int kSymThreads = 64 * kSymWaves;
constexpr int kSymTargets = 64;

template <int P>
__global__ void __launch_bounds__(kSymThreads) k_m2l_sym(int level, int periodic, int kp,
                                                                    const float *__restrict__ mc, uint32_t zero_off,
                                                                    const float *__restrict__ ops,
                                                                    const int32_t *__restrict__ op_off,
                                                                    const int32_t *__restrict__ orbits,
                                                                    const int16_t *__restrict__ row_std,
                                                                    float *__restrict__ dst, int accumulate,
                                                                    int nsplit, float *__restrict__ part) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    constexpr SymLayout SL = sym_layout(P);
    constexpr int NB = SL.nblk, KC = 16 * NB;
    static_assert(NB > 0, "degree without a class layout");
    constexpr int NT = kSymThreads, TT = kSymTargets;
    constexpr int OPF = 16 * SL.C * NB;        // floats of a full orbit (every block)
    constexpr int BUF = OPF + 64;              // + slack for the row over-reads of short blocks
    constexpr int CELL = 3 * KC;               // floats per cell of mc
    static_assert(NB * NT * 4 >= OPF, "the operator copy must finish within one orbit");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    float *opl = reinterpret_cast<float *>(smem_raw);   // [2][BUF]
    __shared__ int32_t sorb[kSymOrbits];
    __shared__ int32_t soff[kSymOrbits + 1];
    __shared__ int16_t srow[KC];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int comp = wave % 3, tg = wave / 3;
    const int h = lane >> 4, col = lane & 15;
    const int octant = blockIdx.x & 7, tile = blockIdx.x >> 3;
    const int o0 = int(blockIdx.y) * kSymOrbits / nsplit;
    const int o1 = (int(blockIdx.y) + 1) * kSymOrbits / nsplit;
    const int64_t ncell_t = int64_t(1) << (3 * (level - 1));
    const int side = 1 << level;

    if (tid < kSymOrbits) sorb[tid] = orbits[tid];
    if (tid <= kSymOrbits) soff[tid] = op_off[octant * (kSymOrbits + 1) + tid];
    for (int i = tid; i < KC; i += NT) srow[i] = row_std[i];
    if (tid < 64) {
        opl[OPF + tid] = 0.0f;
        opl[BUF + OPF + tid] = 0.0f;
    }
    {
        const int b0 = op_off[octant * (kSymOrbits + 1) + o0];
        const int n4 = (op_off[octant * (kSymOrbits + 1) + o0 + 1] - b0) / 4;
        for (int q = tid; q < n4; q += NT)
            *reinterpret_cast<f4 *>(opl + 4 * q) = *reinterpret_cast<const f4 *>(ops + b0 + 4 * q);
    }
    const int64_t slot = int64_t(tile) * TT + tg * 16 + col;
    const bool tvalid = slot < ncell_t;
    const uint32_t tkey = tvalid ? uint32_t((slot << 3) | octant) : 0u;
    const int tc[3] = {int(compact3(tkey)), int(compact3(tkey >> 1)), int(compact3(tkey >> 2))};
    __syncthreads();

    // byte offsets (relative to mc, with the lane group's quad) of the member
    // sources of orbit o; slot r is the reflection of the axes in r, present
    // when r lies within G
    uint32_t mo[8];
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(mc), 0, -1, 0x00020000);
    auto members = [&](int o) {
        const int info = sorb[o];
        const int G = (info >> 6) & 7;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (r & ~G) {
                mo[r] = zero_off * 4u + uint32_t(16 * h);
                continue;
            }
            bool ok = tvalid;
            uint32_t key = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int rep = (info >> (2 * a)) & 3;
                int d = ((r >> a) & 1) ? -rep : rep;
                if ((octant >> a) & 1) d = -d;
                int c = tc[a] + d;
                if (periodic) c &= side - 1;
                else ok = ok && c >= 0 && c < side;
                key |= spread3(uint32_t(c)) << a;
            }
            mo[r] = (ok ? key * uint32_t(CELL) : zero_off) * 4u + uint32_t(16 * h);
        }
    };
    // the lane's quad of k block b of every member; absent slots read the zero
    // cell (loads issued unconditionally keep the wait counts static)
    f4 val[8];
    auto load_block = [&](int b) {
        const uint32_t cb = uint32_t((comp * KC + 16 * b) * 4);
#pragma unroll
        for (int r = 0; r < 8; ++r)
            val[r] = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(rsrc, int(mo[r] + cb), 0, 0));
    };
    // Walsh-Hadamard transform over the reflection slots: y[x] = sum_r chi_x(r) v[r];
    // along an axis outside G the partner slots are zero and the stage copies
    auto wht = [&](f4 (&y)[8], int G) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int bit = 1 << a;
            if (G & bit) {
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    if (!(r & bit)) {
                        const f4 u = y[r], v = y[r | bit];
                        y[r] = u + v;
                        y[r | bit] = u - v;
                    }
            } else {
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    if (!(r & bit)) y[r | bit] = y[r];
            }
        }
    };

    typedef float v4 __attribute__((ext_vector_type(4)));
    v4 acc[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) acc[i] = v4{0.f, 0.f, 0.f, 0.f};

    if (o0 < o1) {
        members(o0);
        load_block(0);
    }
    for (int o = o0; o < o1; ++o) {
        const int cur = (o - o0) & 1;
        const float *olc = opl + cur * BUF;
        float *oln = opl + (cur ^ 1) * BUF;
        const bool more = o + 1 < o1;
        const int nn4 = more ? (soff[o + 2] - soff[o + 1]) / 4 : 0;
        const float *ogn = ops + (more ? soff[o + 1] : 0);
        const int info = sorb[o];
        const int G = (info >> 6) & 7, Z = (info >> 9) & 7;
        int off = 0;   // LDS offset of column block B of this orbit (floats)
        f4 stage;
        static_for<NB>([&](auto bi) {
            constexpr int B = decltype(bi)::value;
            // the next orbit's operator: chunk B - 1 out to LDS, chunk B in
            if constexpr (B > 0) {
                const int q = (B - 1) * NT + tid;
                if (q < nn4) *reinterpret_cast<f4 *>(oln + 4 * q) = stage;
            }
            {
                const int q = B * NT + tid;
                stage = *reinterpret_cast<const f4 *>(ogn + 4 * (q < nn4 ? q : 0));
            }
            if constexpr (B + 1 == NB) members(more ? o + 1 : o);
            // transform into y, load the next k block into val, then the class
            // blocks of column B against y
            f4 y[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) y[r] = val[r];
            wht(y, G);
            load_block(B + 1 < NB ? B + 1 : 0);
            static_for<8>([&](auto xi) {
                constexpr int X = decltype(xi)::value;
                if (!(X & Z)) {
                    static_for<NB>([&](auto ai) {
                        constexpr int A = decltype(ai)::value;
                        if constexpr (SL.bcls[A] == (SL.bcls[B] ^ X)) {
                            const f4 aq = *reinterpret_cast<const f4 *>(olc + off + 4 * (h * SL.bnv[A] + col));
                            off += 16 * SL.bnv[A];
                            static_for<SL.bsteps[B]>([&](auto si) {
                                constexpr int S = decltype(si)::value;
                                acc[A] = __builtin_amdgcn_mfma_f32_16x16x4f32(aq[S], y[X][S], acc[A], 0, 0, 0);
                            });
                        }
                    });
                }
            });
        });
        {
            const int q = (NB - 1) * NT + tid;
            if (q < nn4) *reinterpret_cast<f4 *>(oln + 4 * q) = stage;
        }
        __syncthreads();
    }
    if (!tvalid) return;
    const bool split = part != nullptr;
    float *out = (split ? part + (size_t(blockIdx.y) * (size_t(1) << (3 * level)) + tkey) * 3 * kp
                        : dst + size_t(tkey) * 3 * kp) + comp * kp;
    static_for<NB>([&](auto ai) {
        constexpr int A = decltype(ai)::value;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = 4 * h + r;
            if (e < SL.bnv[A]) {
                float *o = out + srow[16 * A + e];
                *o = (accumulate && !split) ? *o + acc[A][r] : acc[A][r];
            }
        }
    });
}

// FP64 form.  An orbit's operator (up to 139 KB) does not fit twice in LDS,
// so it streams through a ring of kRing column slices (slice (o, B): the class
// blocks of column B), one barrier per slice: while slice k is multiplied, the
// workgroup copies slice k + kRing - 1 into the slot slice k - 1 left.  Each k
// block runs as two halves of two k steps (a lane's 16-byte half quad per
// member), transformed in place; a half's sources for the next step are loaded
// right after its MFMAs.  Blocks are stored as [half][lane group][row][2].
constexpr int kRing = 8;

// AD: the targets and sources of an adaptive tree's level (SymAdapt) instead
// of a uniform level's cells.
template <int P, bool AD>
__global__ void __launch_bounds__(kSymThreads) k_m2l_sym64(int level, int periodic, int kp,
                                                           const double *__restrict__ mc, uint32_t zero_off,
                                                           const double *__restrict__ ops,
                                                           const int32_t *__restrict__ sl_off,
                                                           const int32_t *__restrict__ orbits,
                                                           const int16_t *__restrict__ row_std,
                                                           double *__restrict__ dst, int accumulate, int nsplit,
                                                           double *__restrict__ part, SymAdapt ad) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    typedef double d4 __attribute__((ext_vector_type(4)));
    constexpr SymLayout SL = sym_layout(P);
    constexpr int NB = SL.nblk, KC = 16 * NB, CELL = 3 * KC;
    static_assert(NB > 0, "degree without a class layout");
    constexpr int NT = kSymThreads, TT = kSymTargets;
    constexpr int SLICE = 16 * SL.C;           // doubles of the largest slice (every class block)
    constexpr int SLOT = SLICE + 32;           // + slack for the row over-reads of short blocks
    constexpr int NSL = kSymOrbits * NB + 1;   // slice offsets per octant
    static_assert(SLICE <= 4 * NT, "a slice is copied in two 16-byte chunks per thread");
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double *ring = reinterpret_cast<double *>(smem_raw);   // [kRing][SLOT]
    __shared__ int32_t sorb[kSymOrbits];
    __shared__ int32_t ssl[NSL];
    __shared__ int16_t srow[KC];
    __shared__ int16_t svs[AD ? 343 : 1];   // adaptive: slot of offset d in the octant's list

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int comp = wave % 3, tg = wave / 3;
    const int h = lane >> 4, col = lane & 15;
    int octant, tile;
    int64_t ncell_t;
    if constexpr (AD) {
        // octant groups of the level: tile_start[o] .. tile_start[o + 1] - 1
        octant = 0;
        while (octant < 7 && int(blockIdx.x) >= ad.tile_start[octant + 1]) ++octant;
        tile = int(blockIdx.x) - ad.tile_start[octant];
        ncell_t = ad.oct_n[octant];
    } else {
        octant = blockIdx.x & 7;
        tile = blockIdx.x >> 3;
        ncell_t = int64_t(1) << (3 * (level - 1));
    }
    const int o0 = int(blockIdx.y) * kSymOrbits / nsplit;
    const int o1 = (int(blockIdx.y) + 1) * kSymOrbits / nsplit;
    const int nk = (o1 - o0) * NB;
    const int side = 1 << level;

    if constexpr (AD)
        for (int i = tid; i < 343; i += NT) svs[i] = ad.vslot[octant * 343 + i];
    if (tid < kSymOrbits) sorb[tid] = orbits[tid];
    for (int i = tid; i < NSL; i += NT) ssl[i] = sl_off[octant * NSL + i];
    for (int i = tid; i < KC; i += NT) srow[i] = row_std[i];
    for (int i = tid; i < kRing * 32; i += NT) ring[(i / 32) * SLOT + SLICE + i % 32] = 0.0;
    __syncthreads();
    // the first kRing - 1 slices
    for (int k = 0; k < kRing - 1 && k < nk; ++k) {
        const int g0 = ssl[o0 * NB + k], n2 = (ssl[o0 * NB + k + 1] - g0) / 2;
        for (int q = tid; q < n2; q += NT)
            *reinterpret_cast<d2 *>(ring + k * SLOT + 2 * q) = *reinterpret_cast<const d2 *>(ops + g0 + 2 * q);
    }
    const int64_t slot = int64_t(tile) * TT + tg * 16 + col;
    const bool tvalid = slot < ncell_t;
    // uniform: the target's key at the level; adaptive: its cell index
    const uint32_t tkey = !tvalid ? 0u : AD ? uint32_t(ad.tcell[ad.oct_base[octant] + slot])
                                          : uint32_t((slot << 3) | octant);
    const int tc[3] = {int(compact3(tkey)), int(compact3(tkey >> 1)), int(compact3(tkey >> 2))};
    __syncthreads();

    uint32_t mo[8];   // byte offsets of the member sources (+ the lane group's quad)
    const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(mc), 0, -1, 0x00020000);
    auto members = [&](int o) {
        const int info = sorb[o];
        if constexpr (AD) {
            // the source of each member offset from the target's table row
            const int32_t *row = ad.vtab + size_t(tvalid ? int(tkey) - ad.cell0 : 0) * 189;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                int src = -1;
                if (!(r & ~((info >> 6) & 7)) && tvalid) {
                    int idx = 0, mul = 1;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const int rep = (info >> (2 * a)) & 3;
                        int d = ((r >> a) & 1) ? -rep : rep;
                        if ((octant >> a) & 1) d = -d;
                        idx += (d + 3) * mul;
                        mul *= 7;
                    }
                    const int sl = svs[idx];   // every member offset is in the octant's list
                    src = sl >= 0 ? row[sl] : -1;
                }
                mo[r] = (src >= 0 ? uint32_t(src) * uint32_t(CELL) : zero_off) * 8u + uint32_t(32 * h);
            }
            return;
        }
        const int G = (info >> 6) & 7;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            if (r & ~G) {
                mo[r] = zero_off * 8u + uint32_t(32 * h);
                continue;
            }
            bool ok = tvalid;
            uint32_t key = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int rep = (info >> (2 * a)) & 3;
                int d = ((r >> a) & 1) ? -rep : rep;
                if ((octant >> a) & 1) d = -d;
                int c = tc[a] + d;
                if (periodic) c &= side - 1;
                else ok = ok && c >= 0 && c < side;
                key |= spread3(uint32_t(c)) << a;
            }
            mo[r] = (ok ? key * uint32_t(CELL) : zero_off) * 8u + uint32_t(32 * h);
        }
    };
    d2 val[8];   // the lane's half quad of every member for the current step
    auto load_half = [&](int b, int half) {
        const uint32_t cb = uint32_t((comp * KC + 16 * b + 2 * half) * 8);
#pragma unroll
        for (int r = 0; r < 8; ++r)
            val[r] = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rsrc, int(mo[r] + cb), 0, 0));
    };
    auto wht = [&](int G) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int bit = 1 << a;
            if (G & bit) {
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    if (!(r & bit)) {
                        const d2 u = val[r], v = val[r | bit];
                        val[r] = u + v;
                        val[r | bit] = u - v;
                    }
            } else {
#pragma unroll
                for (int r = 0; r < 8; ++r)
                    if (!(r & bit)) val[r | bit] = val[r];
            }
        }
    };

    d4 acc[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) acc[i] = d4{0.0, 0.0, 0.0, 0.0};

    if (o0 < o1) {
        members(o0);
        load_half(0, 0);
    }
    for (int o = o0; o < o1; ++o) {
        const bool more = o + 1 < o1;
        const int info = sorb[o];
        const int G = (info >> 6) & 7, Z = (info >> 9) & 7;
        static_for<NB>([&](auto bi) {
            constexpr int B = decltype(bi)::value;
            constexpr int HALVES = SL.bsteps[B] > 2 ? 2 : 1;
            const int k = (o - o0) * NB + B;
            // slice k + kRing - 1 in (16-byte chunks q = tid, tid + NT)
            const int kc = k + kRing - 1;
            const bool has = kc < nk;
            const int g0 = has ? ssl[o0 * NB + kc] : 0;
            const int n2 = has ? (ssl[o0 * NB + kc + 1] - g0) / 2 : 0;
            const d2 st0 = *reinterpret_cast<const d2 *>(ops + g0 + 2 * (tid < n2 ? tid : 0));
            const d2 st1 = *reinterpret_cast<const d2 *>(ops + g0 + 2 * (tid + NT < n2 ? tid + NT : 0));
            const double *sl = ring + (k % kRing) * SLOT;
            static_for<HALVES>([&](auto hi) {
                constexpr int HALF = decltype(hi)::value;
                wht(G);
                int boff = 0;
                static_for<8>([&](auto xi) {
                    constexpr int X = decltype(xi)::value;
                    if (!(X & Z)) {
                        static_for<NB>([&](auto ai) {
                            constexpr int A = decltype(ai)::value;
                            if constexpr (SL.bcls[A] == (SL.bcls[B] ^ X)) {
                                const d2 aq = *reinterpret_cast<const d2 *>(
                                    sl + boff + 2 * ((HALF * 4 + h) * SL.bnv[A] + col));
                                boff += 16 * SL.bnv[A];
                                static_for<2>([&](auto si) {
                                    constexpr int S = decltype(si)::value;
                                    if constexpr (2 * HALF + S < SL.bsteps[B])
                                        acc[A] = __builtin_amdgcn_mfma_f64_16x16x4f64(aq[S], val[X][S], acc[A], 0,
                                                                                      0, 0);
                                });
                            }
                        });
                    }
                });
                // the sources of the next step: this block's second half, the next
                // block's first, or the next orbit's first
                if constexpr (HALF + 1 < HALVES) {
                    load_half(B, HALF + 1);
                } else if constexpr (B + 1 < NB) {
                    load_half(B + 1, 0);
                } else {
                    members(more ? o + 1 : o);
                    load_half(0, 0);
                }
            });
            double *dsl = ring + (kc % kRing) * SLOT;
            if (tid < n2) *reinterpret_cast<d2 *>(dsl + 2 * tid) = st0;
            if (tid + NT < n2) *reinterpret_cast<d2 *>(dsl + 2 * (tid + NT)) = st1;
            __syncthreads();
        });
    }
    if (!tvalid) return;
    const bool split = part != nullptr;
    const size_t tslot = AD ? size_t(tkey) - size_t(ad.part_cell0) : size_t(tkey);
    const size_t pstride = AD ? size_t(ad.part_cells) : (size_t(1) << (3 * level));
    double *out = (split ? part + (size_t(blockIdx.y) * pstride + tslot) * 3 * kp
                         : dst + size_t(tkey) * 3 * kp) + comp * kp;
    static_for<NB>([&](auto ai) {
        constexpr int A = decltype(ai)::value;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = h + 4 * r;   // the FP64 MFMA's output row of lane group h, element r
            if (e < SL.bnv[A]) {
                double *o = out + srow[16 * A + e];
                *o = (accumulate && !split) ? *o + acc[A][r] : acc[A][r];
            }
        }
    });
}

}  // namespace

bool m2l_sym_supported(int p) { return p == 10; }

template <typename T>
hipError_t launch_sym_pack_range(hipStream_t s, int64_t npack, int64_t zero_cell, int kp, int kc, const T *M,
                                 const int16_t *mc_src, T *Mc) {
    const int64_t nelem = (npack + 1) * 3 * kc;
    hipLaunchKernelGGL(k_sym_pack<T>, dim3(unsigned((nelem + 255) / 256)), dim3(256), 0, s, npack * 3 * kc,
                       zero_cell * 3 * kc, kp, kc, M, mc_src, Mc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sym_pack(hipStream_t s, int64_t ncells, int kp, int kc, const T *M, const int16_t *mc_src, T *Mc) {
    return launch_sym_pack_range<T>(s, ncells, ncells, kp, kc, M, mc_src, Mc);
}
template hipError_t launch_sym_pack<float>(hipStream_t, int64_t, int, int, const float *, const int16_t *, float *);
template hipError_t launch_sym_pack<double>(hipStream_t, int64_t, int, int, const double *, const int16_t *,
                                            double *);
template hipError_t launch_sym_pack_range<float>(hipStream_t, int64_t, int64_t, int, int, const float *,
                                                 const int16_t *, float *);
template hipError_t launch_sym_pack_range<double>(hipStream_t, int64_t, int64_t, int, int, const double *,
                                                  const int16_t *, double *);

hipError_t launch_m2l_sym64(hipStream_t s, int level, int periodic, int p, int kp, const double *mc,
                            int64_t zero_cell, const double *ops, const int32_t *sl_off, const int32_t *orbits,
                            const int16_t *row_std, double *dst, int accumulate, double *part, size_t part_elems) {
    if (!m2l_sym_supported(p) || level < 1) return hipErrorInvalidValue;
    constexpr SymLayout SL = sym_layout(10);
    constexpr int KC = 16 * SL.nblk;
    if ((uint64_t(zero_cell) + 1) * 3 * KC * sizeof(double) > (uint64_t(1) << 32)) return hipErrorInvalidValue;
    const int64_t ncell_t = int64_t(1) << (3 * (level - 1));
    const size_t smem = sizeof(double) * size_t(kRing) * size_t(16 * SL.C + 32);
    int nsplit = part ? translate_splits(level, kSymTargets, kp, part_elems) : 1;
    if (nsplit > kSymOrbits) nsplit = kSymOrbits;
    double *pbuf = nsplit > 1 ? part : nullptr;
    const dim3 grid(unsigned((ncell_t + kSymTargets - 1) / kSymTargets * 8), unsigned(nsplit));
    hipLaunchKernelGGL((k_m2l_sym64<10, false>), grid, dim3(kSymThreads), smem, s, level, periodic, kp, mc,
                       uint32_t(zero_cell * 3 * KC), ops, sl_off, orbits, row_std, dst, accumulate, nsplit, pbuf,
                       SymAdapt());
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nsplit == 1) return e;
    return launch_split_reduce64(s, level, kp, SL.C, nsplit, pbuf, dst, accumulate);
}

hipError_t launch_m2l_sym64_adaptive(hipStream_t s, int p, int kp, const double *mc, int64_t zero_cell,
                                     const double *ops, const int32_t *sl_off, const int32_t *orbits,
                                     const int16_t *row_std, double *dst, int accumulate, const SymAdapt &ad_in,
                                     double *part, size_t part_elems) {
    if (!m2l_sym_supported(p)) return hipErrorInvalidValue;
    constexpr SymLayout SL = sym_layout(10);
    constexpr int KC = 16 * SL.nblk;
    if ((uint64_t(zero_cell) + 1) * 3 * KC * sizeof(double) > (uint64_t(1) << 32)) return hipErrorInvalidValue;
    SymAdapt ad = ad_in;
    ad.tile_start[0] = 0;
    for (int o = 0; o < 8; ++o) ad.tile_start[o + 1] = ad.tile_start[o] + (ad.oct_n[o] + kSymTargets - 1) / kSymTargets;
    const int grid = ad.tile_start[8];
    if (grid == 0) return hipSuccess;
    // orbit-range splits: a workgroup holds a compute unit (its LDS), so the
    // level takes ceil(grid nsplit / CUs) rounds of ceil(56 / nsplit) orbits;
    // the smallest nsplit with the fewest orbit-rounds that the partial-sum
    // buffer holds
    int nsplit = 1;
    if (part != nullptr && ad.part_cells > 0) {
        static int ncu = 0;
        if (ncu == 0) {
            int dev = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
                ncu = 256;
        }
        const size_t per_split = size_t(ad.part_cells) * 3 * kp;
        int64_t best = -1;
        for (int ns = 1; ns <= kSymOrbits && size_t(ns) * per_split <= part_elems; ++ns) {
            const int64_t rounds = (int64_t(grid) * ns + ncu - 1) / ncu;
            const int64_t cost = rounds * ((kSymOrbits + ns - 1) / ns);
            if (best < 0 || cost < best) {
                best = cost;
                nsplit = ns;
            }
        }
    }
    double *pbuf = nsplit > 1 ? part : nullptr;
    const size_t smem = sizeof(double) * size_t(kRing) * size_t(16 * SL.C + 32);
    hipLaunchKernelGGL((k_m2l_sym64<10, true>), dim3(unsigned(grid), unsigned(nsplit)), dim3(kSymThreads), smem, s,
                       0, 0, kp, mc, uint32_t(zero_cell * 3 * KC), ops, sl_off, orbits, row_std, dst, accumulate,
                       nsplit, pbuf, ad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nsplit == 1) return e;
    const int64_t nelem = int64_t(ad.part_cells) * 3 * kp;
    return launch_split_reduce64_n(s, nelem, kp, SL.C, nsplit, pbuf, dst + size_t(ad.part_cell0) * 3 * kp,
                                   accumulate);
}

hipError_t launch_m2l_sym(hipStream_t s, int level, int periodic, int p, int kp, const float *mc, int64_t zero_cell,
                          const float *ops, const int32_t *op_off, const int32_t *orbits, const int16_t *row_std,
                          float *dst, int accumulate, float *part, size_t part_elems) {
    if (!m2l_sym_supported(p) || level < 1) return hipErrorInvalidValue;
    constexpr SymLayout SL = sym_layout(10);
    constexpr int KC = 16 * SL.nblk;
    // byte offsets into mc (the zero cell included) must fit 32 bits
    if ((uint64_t(zero_cell) + 1) * 3 * KC * sizeof(float) > (uint64_t(1) << 32)) return hipErrorInvalidValue;
    const int64_t ncell_t = int64_t(1) << (3 * (level - 1));
    const size_t smem = 2 * sizeof(float) * size_t(16 * SL.C * SL.nblk + 64);
    int nsplit = part ? translate_splits(level, kSymTargets, kp, part_elems) : 1;
    if (nsplit > kSymOrbits) nsplit = kSymOrbits;
    float *pbuf = nsplit > 1 ? part : nullptr;
    const dim3 grid(unsigned((ncell_t + kSymTargets - 1) / kSymTargets * 8), unsigned(nsplit));
    hipLaunchKernelGGL(k_m2l_sym<10>, grid, dim3(kSymThreads), smem, s, level, periodic, kp, mc,
                       uint32_t(zero_cell * 3 * KC), ops, op_off, orbits, row_std, dst, accumulate, nsplit, pbuf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nsplit == 1) return e;
    return launch_split_reduce(s, level, kp, SL.C, nsplit, pbuf, dst, accumulate);
}

}  // namespace vmfmm
