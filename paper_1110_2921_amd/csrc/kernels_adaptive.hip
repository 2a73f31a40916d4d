// Adaptive tree of the hybrid treecode-FMM (Sec. 3.2): construction level by
// level from the particles sorted at the finest level, the stack-based dual
// traversal that turns touching cell pairs into P2P, M2L (cell-cell), M2P and
// P2L (cell-particle) interactions, and the two cell-particle kernels.
//
// Cells are numbered level by level, ascending key inside a level.  A cell is
// split when it holds more than ncrit particles above max_level; only its
// non-empty children exist.  Two cells interact through expansions when their
// closed cubes (the source shifted by its image) do not touch, an integer test
// on the finest grid.
//
// Traversal: a cell's partners are the touching (cell, image) pairs it hands to
// its children unresolved: same-level cells and coarser leaves, at most the 27
// neighbour positions of the cell.  A cell's candidates are its parent's
// partners, split ones replaced by their children (the root: itself and, when
// periodic, its 26 images).  A candidate that does not touch the cell is an
// M2L source when it has the cell's level, and a P2L source when it is a
// coarser leaf and the cell is split.  Cell-particle interactions need a split
// cell on the cell side (a cell of at most ncrit particles is cheaper taken
// particle by particle), so any other candidate -- touching, or a coarser leaf
// apart from a leaf cell -- is a P2P source when both are leaves, a partner
// when the cell is split, and when only the candidate is split its subtree is
// walked with an explicit stack: split cells that do not touch the leaf are
// M2P sources, its leaves (touching or not) P2P sources, touching split cells
// are opened.  Each (target particle, source particle, image) triple is then
// covered by exactly one interaction.
#include <cstdio>

#include "device_harmonics.h"
#include "kernels.h"

namespace vmfmm {

namespace {

using dev::irregular_packed;
using dev::irregular_packed_orders;

__device__ __forceinline__ int ad_coord(uint32_t k, int d, int level) {
    int c = 0;
    for (int b = 0; b < level; ++b) c |= int((k >> (3 * b + d)) & 1u) << b;
    return c;
}

__device__ __forceinline__ bool ad_leaf(const AdTreeView &t, int c) {
    return t.count[c] <= t.ncrit || t.level[c] >= t.max_level;
}

// image shift code (sx+1) + 3 (sy+1) + 9 (sz+1) -> component d
__device__ __forceinline__ int shift_of(int code, int d) {
    return d == 0 ? code % 3 - 1 : (d == 1 ? (code / 3) % 3 - 1 : code / 9 - 1);
}

// Do the closed cubes of a and of b shifted by image `code` touch?
__device__ __forceinline__ bool touching(const AdTreeView &t, int a, int b, int code) {
    const int la = t.level[a], lb = t.level[b], M = t.max_level;
    const int na = 1 << (M - la), nb = 1 << (M - lb);
    for (int d = 0; d < 3; ++d) {
        const int ca = ad_coord(t.key[a], d, la) << (M - la);
        const int cb = (ad_coord(t.key[b], d, lb) << (M - lb)) + shift_of(code, d) * (1 << M);
        if (ca > cb + nb || cb > ca + na) return false;
    }
    return true;
}

__device__ __forceinline__ void centre(const AdTreeView &t, int c, double out[3]) {
    if (t.ctr) {
        for (int d = 0; d < 3; ++d) out[d] = t.ctr[4 * size_t(c) + d];
        return;
    }
    const int l = t.level[c];
    const double w = ldexp(t.box_len, -l);
    for (int d = 0; d < 3; ++d) out[d] = t.lo[d] + (double(ad_coord(t.key[c], d, l)) + 0.5) * w;
}

// sort key of each cell for the octant groups of all levels at once:
// level * 8 + octant (a stable sort keeps the key order inside a group)
__global__ void __launch_bounds__(256) k_ad_group_keys(AdTreeView t, int ncell, uint32_t *__restrict__ keys,
                                                       int32_t *__restrict__ idx) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    keys[c] = uint32_t(t.level[c]) * 8u + (t.key[c] & 7u);
    idx[c] = c;
}

// the first position of each (level, octant) group, from the sort pass's
// scanned histogram (digit-major, block 0 first), and the cell count
__global__ void k_ad_group_starts(int ngroup, int nblk, int ncell, const uint32_t *__restrict__ offs,
                                  int *__restrict__ starts) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < ngroup) starts[g] = int(offs[size_t(g) * nblk]);
    if (g == 0) starts[ngroup] = ncell;
}

// per cell: its P2P entries' source ranges and frame shifts
__global__ void __launch_bounds__(64) k_ad_p2p_meta(AdTreeView t, int ncell, const uint32_t *__restrict__ off,
                                                    const uint32_t *__restrict__ cnt,
                                                    const int32_t *__restrict__ src, const int8_t *__restrict__ code,
                                                    P2PMeta *__restrict__ meta) {
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= ncell) return;
    const uint32_t e0 = off[a], e1 = e0 + cnt[a];
    if (e1 == e0) return;
    double ca[3];
    centre(t, a, ca);
    for (uint32_t e = e0; e < e1; ++e) {
        const int b = src[e], cd = code[e];
        double cb[3];
        centre(t, b, cb);
        P2PMeta m;
        m.dx = cb[0] + shift_of(cd, 0) * t.box_len - ca[0];
        m.dy = cb[1] + shift_of(cd, 1) * t.box_len - ca[1];
        m.dz = cb[2] + shift_of(cd, 2) * t.box_len - ca[2];
        m.js = t.start[b];
        m.je = m.js + t.count[b];
        meta[e] = m;
    }
}

__global__ void __launch_bounds__(256) k_ad_centres(AdTreeView t, int ncell, double *__restrict__ ctr) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    t.ctr = nullptr;
    double v[3];
    centre(t, c, v);
    for (int d = 0; d < 3; ++d) ctr[4 * size_t(c) + d] = v[d];
    ctr[4 * size_t(c) + 3] = 0.0;
}

// ------------------------------------------------------------- construction ----
__global__ void k_ad_root(AdTreeView t, int n) {
    if (threadIdx.x != 0) return;
    int32_t *child = const_cast<int32_t *>(t.child);
    const_cast<uint32_t *>(t.key)[0] = 0u;
    const_cast<int32_t *>(t.level)[0] = 0;
    const_cast<int32_t *>(t.start)[0] = 0;
    const_cast<int32_t *>(t.count)[0] = n;
    const_cast<int32_t *>(t.parent)[0] = -1;
    for (int o = 0; o < 8; ++o) child[o] = -1;
}

// slot 8 (c - off) + o: particle range of child o of cell c (empty unless c is split)
__global__ void __launch_bounds__(256) k_ad_children(AdTreeView t, int off, int ncl, const uint32_t *__restrict__ fine,
                                                     int32_t *__restrict__ sstart, int32_t *__restrict__ scount,
                                                     uint32_t *__restrict__ flag) {
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= 8 * ncl) return;
    const int c = off + slot / 8, o = slot % 8;
    int s0 = 0, cnt = 0;
    const int l = t.level[c];
    if (!ad_leaf(t, c)) {
        const int shift = 3 * (t.max_level - l - 1);
        const uint32_t want = (t.key[c] << 3) | uint32_t(o);
        const int a = t.start[c], e = a + t.count[c];
        // first position with prefix >= want, then first with prefix > want
        int lo = a, hi = e;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if ((fine[mid] >> shift) < want) lo = mid + 1;
            else hi = mid;
        }
        int lo2 = lo, hi2 = e;
        while (lo2 < hi2) {
            const int mid = (lo2 + hi2) >> 1;
            if ((fine[mid] >> shift) <= want) lo2 = mid + 1;
            else hi2 = mid;
        }
        s0 = lo;
        cnt = lo2 - lo;
    }
    sstart[slot] = s0;
    scount[slot] = cnt;
    flag[slot] = cnt > 0 ? 1u : 0u;
}

__global__ void __launch_bounds__(256) k_ad_emit(AdTreeView t, int off, int ncl, const int32_t *__restrict__ sstart,
                                                 const int32_t *__restrict__ scount, const uint32_t *__restrict__ rank,
                                                 int *__restrict__ nnext) {
    const int slot = blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= 8 * ncl) return;
    const int c = off + slot / 8, o = slot % 8;
    const int next0 = off + ncl;
    if (slot == 8 * ncl - 1) *nnext = int(rank[slot]) + (scount[slot] > 0 ? 1 : 0);
    int32_t *child = const_cast<int32_t *>(t.child);
    if (scount[slot] == 0) {
        child[8 * c + o] = -1;
        return;
    }
    const int idx = next0 + int(rank[slot]);
    const_cast<uint32_t *>(t.key)[idx] = (t.key[c] << 3) | uint32_t(o);
    const_cast<int32_t *>(t.level)[idx] = t.level[c] + 1;
    const_cast<int32_t *>(t.start)[idx] = sstart[slot];
    const_cast<int32_t *>(t.count)[idx] = scount[slot];
    const_cast<int32_t *>(t.parent)[idx] = c;
    child[8 * c + o] = idx;
}

// the children of the last level's cells do not exist
__global__ void __launch_bounds__(256) k_ad_no_children(AdTreeView t, int off, int ncl) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 8 * ncl) return;
    const_cast<int32_t *>(t.child)[8 * off + i] = -1;
}

// ------------------------------------------------------------------ leaves ----
__global__ void __launch_bounds__(256) k_ad_leaf_mark(AdTreeView t, int ncell, int32_t *__restrict__ leaf_at) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ncell || !ad_leaf(t, c)) return;
    leaf_at[t.start[c]] = c;
}

__global__ void __launch_bounds__(256) k_ad_leaf_flag(int n, const int32_t *__restrict__ leaf_at,
                                                      uint32_t *__restrict__ flag) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = leaf_at[i] >= 0 ? 1u : 0u;
}

__global__ void __launch_bounds__(256) k_ad_leaf_compact(AdTreeView t, int n, const int32_t *__restrict__ leaf_at,
                                                         const uint32_t *__restrict__ rank, int32_t *__restrict__ lcell,
                                                         int32_t *__restrict__ lstart, int32_t *__restrict__ llev,
                                                         int *__restrict__ nleaf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = leaf_at[i];
    if (i == n - 1) {
        const int tot = int(rank[i]) + (c >= 0 ? 1 : 0);
        *nleaf = tot;
        lstart[tot] = n;
    }
    if (c < 0) return;
    const int r = int(rank[i]);
    lcell[r] = c;
    lstart[r] = i;
    llev[r] = t.level[c];
}

__device__ __forceinline__ double wrap1(double x, double lo, double len, double inv_len) {
#pragma clang fp contract(off)
    const double s = floor((x - lo) * inv_len);
    const double tt = s * len;
    return x - tt;
}

// one workgroup per leaf: records of its particles relative to its centre
__global__ void __launch_bounds__(64) k_ad_permute(AdTreeView t, int n, const double *__restrict__ x,
                                                   const double *__restrict__ alpha, const int32_t *__restrict__ perm,
                                                   const int32_t *__restrict__ lcell, Part64 *__restrict__ parts) {
    const int c = lcell[blockIdx.x];
    double ctr[3];
    centre(t, c, ctr);
    const int s0 = t.start[c], cnt = t.count[c];
    for (int k = threadIdx.x; k < cnt; k += 64) {
        const int i = s0 + k, j = perm[i];
        double dl[3], al[3];
        for (int d = 0; d < 3; ++d) {
            double xv = x[size_t(d) * n + j];
            if (t.periodic) xv = wrap1(xv, t.lo[d], t.box_len, t.inv_len);
            dl[d] = xv - ctr[d];
            al[d] = alpha[size_t(d) * n + j];
        }
        Part64 r;
        r.dx = dl[0]; r.dy = dl[1]; r.dz = dl[2];
        r.ax = al[0]; r.ay = al[1]; r.az = al[2];
        r.pad0 = 0.0; r.pad1 = 0.0;
        parts[i] = r;
    }
}

// --------------------------------------------------------------- traversal ----
constexpr int kAdStack = 128;
constexpr int kM2LSlots = 189;

// exclusive prefix over the wave's lanes (lane order) and the wave's total
__device__ __forceinline__ uint32_t wave_scan(uint32_t v, uint32_t &total) {
    const int lane = threadIdx.x & 63;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    total = __shfl(x, 63, 64);
    return x - v;
}

// One wave per cell a of level l.  Candidate c of a's list is (parent partner
// c / 8, child c % 8); a leaf partner stands for itself at c % 8 == 0 (the
// root: itself under each of its images).  The lanes classify the candidates
// 64 at a time; each lane walks its own candidate's subtree when that is
// needed.  List entries go to the cell's lists in candidate order: in the
// filling pass every lane first counts its entries, the wave's prefix sums
// place them, and the lane classifies again, writing.
__global__ void __launch_bounds__(64) k_ad_traverse(AdTreeView t, AdLists ls, int lvl, int off, int ncl, int pass,
                                                    int vcell0, int ncell) {
    const int a = off + int(blockIdx.x);
    // lvl < 0: cells of every level in one launch (the filling pass, whose
    // partners are all known), each at its own level
    const int l = lvl >= 0 ? lvl : t.level[a];
    const int lane = threadIdx.x;
    const bool leaf_a = ad_leaf(t, a);
    const int oct = int(t.key[a] & 7u);
    int ca[3];
    for (int d = 0; d < 3; ++d) ca[d] = ad_coord(t.key[a], d, l);
    bool bad = false;
    int stack[kAdStack];

    // classify candidate b: with write == false count the list entries into
    // cnt, with write == true store them from pos on (and the M2L slot)
    auto classify = [&](int b, int code, bool write, uint32_t (&pos)[3], uint32_t (&cnt)[3], bool &partner) {
        auto put = [&](int k, int src) {
            if (write) {
                ls.src[k][pos[k]] = src;
                ls.code[k][pos[k]] = int8_t(code);
                ++pos[k];
            } else {
                ++cnt[k];
            }
        };
        const int lb = t.level[b];
        // apart: cell-cell between cells of one level; particle-cell from a
        // coarser leaf b only into a split cell a -- a leaf a takes b's
        // particles directly, the cheaper of the two for cells of <= ncrit
        if (!touching(t, a, b, code) && (lb == l || !leaf_a)) {
            if (lb == l) {
                if (write) {
                    int idx = 0, mul = 1;
                    bool out = false;
                    for (int d = 0; d < 3; ++d) {
                        const int dd = ad_coord(t.key[b], d, l) + shift_of(code, d) * (1 << l) - ca[d];
                        if (dd < -3 || dd > 3) out = true;
                        idx += (dd + 3) * mul;
                        mul *= 7;
                    }
                    const int slot = out ? -1 : ls.vslot[oct * 343 + idx];
                    if (slot < 0) bad = true;
                    else ls.vtab[size_t(a - vcell0) * kM2LSlots + slot] = b;
                }
            } else {
                put(2, b);      // P2L: b is a coarser leaf
            }
            return;
        }
        const bool leaf_b = ad_leaf(t, b);
        if (leaf_a && leaf_b) {
            put(0, b);
        } else if (leaf_a) {
            // walk b's subtree: split cells apart from a are M2P sources,
            // its leaves (apart or touching) P2P sources
            int sp = 0;
            for (int o = 0; o < 8; ++o) {
                const int e = t.child[8 * b + o];
                if (e >= 0) {
                    if (sp < kAdStack) stack[sp++] = e;
                    else bad = true;
                }
            }
            while (sp > 0) {
                const int e = stack[--sp];
                const bool leaf_e = ad_leaf(t, e);
                if (!leaf_e && !touching(t, a, e, code)) {
                    put(1, e);   // M2P from a split cell only
                } else if (leaf_e) {
                    put(0, e);
                } else {
                    for (int o = 0; o < 8; ++o) {
                        const int f = t.child[8 * e + o];
                        if (f >= 0) {
                            if (sp < kAdStack) stack[sp++] = f;
                            else bad = true;
                        }
                    }
                }
            }
        } else {
            partner = true;     // a is split: the pair goes to a's children
        }
    };

    int P = -1, ncand;
    if (l == 0) {
        ncand = t.periodic ? 27 : 1;
    } else {
        P = t.parent[a];
        ncand = 8 * ls.npart[P];
    }
    uint32_t base[3] = {0u, 0u, 0u};
    if (pass == 1)
        for (int k = 0; k < 3; ++k) base[k] = ls.off[size_t(k) * ncell + a];
    uint32_t nent[3] = {0u, 0u, 0u};
    int np = 0;
    for (int c0 = 0; c0 < ncand; c0 += 64) {
        const int c = c0 + lane;
        int b = -1, code = 13;
        if (c < ncand) {
            if (l == 0) {
                b = 0;
                code = t.periodic ? c : 13;
            } else {
                const int B = ls.part[size_t(P) * 27 + (c >> 3)];
                code = ls.pcode[size_t(P) * 27 + (c >> 3)];
                b = ad_leaf(t, B) ? ((c & 7) == 0 ? B : -1) : t.child[8 * B + (c & 7)];
            }
        }
        uint32_t cnt[3] = {0u, 0u, 0u}, pos[3];
        bool partner = false;
        if (b >= 0) classify(b, code, false, pos, cnt, partner);
        uint32_t tot[3], ptot;
        uint32_t pre[3];
        for (int k = 0; k < 3; ++k) pre[k] = wave_scan(cnt[k], tot[k]);
        const uint32_t pp = wave_scan(partner ? 1u : 0u, ptot);
        if (pass == 0 && partner) {
            const int slot = np + int(pp);
            if (slot < 27) {
                ls.part[size_t(a) * 27 + slot] = b;
                ls.pcode[size_t(a) * 27 + slot] = int8_t(code);
            } else {
                bad = true;
            }
        }
        if (pass == 1 && b >= 0) {
            for (int k = 0; k < 3; ++k) pos[k] = base[k] + nent[k] + pre[k];
            bool unused = false;
            classify(b, code, true, pos, cnt, unused);
        }
        for (int k = 0; k < 3; ++k) nent[k] += tot[k];
        np += int(ptot);
    }
    if (pass == 0 && lane == 0) {
        ls.npart[a] = np < 27 ? np : 27;
        for (int k = 0; k < 3; ++k) ls.cnt[size_t(k) * ncell + a] = nent[k];
    }
    if (bad) atomicExch(ls.err, 1);
}

// ------------------------------------------------------------ cell-particle ----
// P2L: one workgroup per target cell with a P2L list.  Lane j takes the
// conjugated irregular harmonics of source particle j (relative to the target
// centre, in target widths) into its LDS row; lanes then sum the rows per
// coefficient, weighted by the particles' strengths, and add the result to the
// cell's local expansion (which already holds L2L and M2L).
__global__ void __launch_bounds__(64) k_ad_p2l(AdTreeView t, AdLists ls, int off, int ncl, int ncell, int p, int kp,
                                               DevTables tab, const Part64 *__restrict__ parts,
                                               double *__restrict__ L) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int a = off + blockIdx.x;
    const uint32_t e0 = ls.off[size_t(2) * ncell + a];
    const uint32_t e1 = e0 + ls.cnt[size_t(2) * ncell + a];
    if (e1 == e0) return;
    const int C = (p + 1) * (p + 1), lane = threadIdx.x;
    const int stride = C + 1;
    double *rows = reinterpret_cast<double *>(smem_raw);   // [64][C + 1]
    double *al = rows + 64 * stride;                       // [64][3]
    double ca[3];
    centre(t, a, ca);
    const double inv_w = ldexp(t.inv_len, t.level[a]);
    constexpr int kMaxC = 4;   // coefficients per lane: C <= 256 (p <= 15)
    double acc[kMaxC][3];
    for (int q = 0; q < kMaxC; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.0;
    for (uint32_t e = e0; e < e1; ++e) {
        const int b = ls.src[2][e], code = ls.code[2][e];
        double cb[3];
        centre(t, b, cb);
        // source position relative to the target centre: delta_j + (c_b + s L - c_a)
        double sh[3];
        for (int d = 0; d < 3; ++d) sh[d] = cb[d] + shift_of(code, d) * t.box_len - ca[d];
        const int s0 = t.start[b], cnt = t.count[b];
        for (int base = 0; base < cnt; base += 64) {
            const int nj = min(64, cnt - base);
            if (lane < nj) {
                const Part64 q = parts[s0 + base + lane];
                const double X = (q.dx + sh[0]) * inv_w, Y = (q.dy + sh[1]) * inv_w, Z = (q.dz + sh[2]) * inv_w;
                irregular_packed<double>(X, Y, Z, p, tab.c1_64, tab.c2_64, tab.diag_64, -1.0, rows + lane * stride, 1);
                al[lane * 3 + 0] = q.ax;
                al[lane * 3 + 1] = q.ay;
                al[lane * 3 + 2] = q.az;
            }
            __syncthreads();
            for (int q = 0; q < kMaxC; ++q) {
                const int cidx = lane + 64 * q;
                if (cidx >= C) break;
                for (int j = 0; j < nj; ++j) {
                    const double v = rows[j * stride + cidx];
                    acc[q][0] += al[j * 3 + 0] * v;
                    acc[q][1] += al[j * 3 + 1] * v;
                    acc[q][2] += al[j * 3 + 2] * v;
                }
            }
            __syncthreads();
        }
    }
    for (int q = 0; q < kMaxC; ++q) {
        const int cidx = lane + 64 * q;
        if (cidx >= C) break;
        for (int k = 0; k < 3; ++k) L[(size_t(a) * 3 + k) * kp + cidx] += acc[q][k];
    }
}

// M2P: one workgroup per block of 16 targets of a leaf with an M2P list.
// For each source cell the lane writes the balanced irregular harmonics of its
// particle's offset from the source centre (degree p + 2) into its LDS column,
// forms the degree <= 2 local expansion about the particle from the table
// (rows x (col, harm, weight)), and the table's evaluation matrix G turns
// those coefficients into u and J at the particle, added to far[12][n].
constexpr int kM2PMaxRow = 9;
constexpr int kM2PChunk = 2;   // list entries per M2P work item

__global__ void __launch_bounds__(64) k_ad_m2p(AdTreeView t, AdLists ls, const int4 *__restrict__ items,
                                               const int32_t *__restrict__ lcell,
                                               const int32_t *__restrict__ lstart, int n, int ncell, int p, int kp,
                                               int nrow, int nharm, DevTables tab, const int32_t *__restrict__ rowptr,
                                               const int32_t *__restrict__ col, const int32_t *__restrict__ harm,
                                               const double *__restrict__ wt, const double *__restrict__ G,
                                               const Part64 *__restrict__ parts, const double *__restrict__ M,
                                               double *__restrict__ far, double *__restrict__ part) {
    // Particle pi of the item's 16 has lanes 4 pi .. 4 pi + 3: lane j computes
    // the harmonic orders m = j (mod 4) and sums every fourth term of each
    // local row, and the lanes' partial rows are added by two butterflies.
    // LDS holds the 16 particles' harmonics and the source cell's multipole.
    // Item (leaf, first target, chunk c, chunks): 16 targets against entries
    // c kM2PChunk .. of the leaf's list, so that the few leaves with M2P lists
    // still give the chip many short waves; with several chunks the outputs go
    // to part[item][12][16] and k_ad_m2p_reduce adds them in chunk order.
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int4 it = items[blockIdx.x];
    const int a = lcell[it.x];
    const uint32_t l0 = ls.off[size_t(1) * ncell + a];
    const uint32_t l1 = l0 + ls.cnt[size_t(1) * ncell + a];
    const uint32_t e0 = l0 + uint32_t(it.z) * kM2PChunk;
    const uint32_t e1 = e0 + kM2PChunk < l1 ? e0 + kM2PChunk : l1;
    if (e1 <= e0) return;
    const int lane = threadIdx.x, pi = lane >> 2, j = lane & 3;
    double *hs = reinterpret_cast<double *>(smem_raw);     // [nharm][16]
    double *mb = hs + size_t(nharm) * 16;                   // [3][kp]
    double ca[3];
    centre(t, a, ca);
    const int s0 = lstart[it.x], cnt = lstart[it.x + 1] - s0;
    {
        const int base = it.y;
        const bool valid = base + pi < cnt;
        const Part64 me = parts[s0 + base + (valid ? pi : 0)];
        double out[3] = {0.0, 0.0, 0.0};                    // outputs j, j + 4, j + 8
        for (uint32_t e = e0; e < e1; ++e) {
            const int b = ls.src[1][e], code = ls.code[1][e];
            double cb[3];
            centre(t, b, cb);
            const int lb = t.level[b];
            const double inv_w = ldexp(t.inv_len, lb);
            __syncthreads();
            for (int k = lane; k < 3 * kp; k += 64) mb[k] = M[size_t(b) * 3 * kp + k];
            // particle relative to the source centre: delta_i + (c_a - c_b - s L)
            const double X = (me.dx + (ca[0] - cb[0] - shift_of(code, 0) * t.box_len)) * inv_w;
            const double Y = (me.dy + (ca[1] - cb[1] - shift_of(code, 1) * t.box_len)) * inv_w;
            const double Z = (me.dz + (ca[2] - cb[2] - shift_of(code, 2) * t.box_len)) * inv_w;
            irregular_packed_orders<double>(X, Y, Z, p + 2, tab.c1_64, tab.c2_64, tab.diag_64, 1.0, j, 4, hs + pi,
                                            16);
            __syncthreads();
            double loc[3][kM2PMaxRow];
#pragma unroll
            for (int r = 0; r < kM2PMaxRow; ++r) {
                double s0v = 0.0, s1v = 0.0, s2v = 0.0;
                if (r < nrow) {
                    const int k1 = rowptr[r + 1];
                    int k = rowptr[r] + j;
                    // this lane's terms four apart, eight at a time
                    for (; k + 28 < k1; k += 32) {
                        int cc[8], hh[8];
                        double ww[8], hv[8];
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            cc[i] = col[k + 4 * i];
                            hh[i] = harm[k + 4 * i];
                            ww[i] = wt[k + 4 * i];
                        }
#pragma unroll
                        for (int i = 0; i < 8; ++i) hv[i] = ww[i] * hs[hh[i] * 16 + pi];
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            s0v += hv[i] * mb[cc[i]];
                            s1v += hv[i] * mb[kp + cc[i]];
                            s2v += hv[i] * mb[2 * kp + cc[i]];
                        }
                    }
                    for (; k < k1; k += 4) {
                        const double hv = wt[k] * hs[harm[k] * 16 + pi];
                        const int c = col[k];
                        s0v += hv * mb[c];
                        s1v += hv * mb[kp + c];
                        s2v += hv * mb[2 * kp + c];
                    }
                }
                // the four lanes' partial sums, fixed order
                s0v += __shfl_xor(s0v, 1);
                s1v += __shfl_xor(s1v, 1);
                s2v += __shfl_xor(s2v, 1);
                s0v += __shfl_xor(s0v, 2);
                s1v += __shfl_xor(s1v, 2);
                s2v += __shfl_xor(s2v, 2);
                loc[0][r] = s0v;
                loc[1][r] = s1v;
                loc[2][r] = s2v;
            }
            const double su = 0.079577471545947667884 * inv_w * inv_w, sj = su * inv_w;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int o = j + 4 * i;
                double v = 0.0;
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int r = 0; r < kM2PMaxRow; ++r)
                        if (r < nrow) v += G[size_t(o) * 3 * nrow + k * nrow + r] * loc[k][r];
                out[i] += v * (o < 3 ? su : sj);
            }
        }
        if (it.w > 1) {
            // this chunk's share, summed over the chunks by k_ad_m2p_reduce
#pragma unroll
            for (int i = 0; i < 3; ++i) part[(size_t(blockIdx.x) * 12 + j + 4 * i) * 16 + pi] = out[i];
        } else if (valid) {
            const size_t gi = size_t(s0) + base + pi;
#pragma unroll
            for (int i = 0; i < 3; ++i) far[size_t(j + 4 * i) * n + gi] += out[i];
        }
    }
}

// M2P work items of leaf i: blocks of 16 targets times chunks of kM2PChunk
// entries of its M2P list
__device__ __forceinline__ int m2p_items_of(int i, const int32_t *__restrict__ lstart,
                                            const int32_t *__restrict__ lcell, const uint32_t *__restrict__ cnt1,
                                            int &nb, int &nch) {
    const uint32_t len = cnt1[lcell[i]];
    nb = (lstart[i + 1] - lstart[i] + 15) / 16;
    nch = int((len + kM2PChunk - 1) / kM2PChunk);
    return nb * nch;
}

__global__ void __launch_bounds__(256) k_ad_m2p_count(int nleaf, const int32_t *__restrict__ lstart,
                                                      const int32_t *__restrict__ lcell,
                                                      const uint32_t *__restrict__ cnt1, uint32_t *__restrict__ ni) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int nb, nch;
    if (i < nleaf) ni[i] = uint32_t(m2p_items_of(i, lstart, lcell, cnt1, nb, nch));
}

// after the exclusive scan: the item count (last leaf's offset + its items)
__global__ void k_ad_m2p_total(int nleaf, const int32_t *__restrict__ lstart, const int32_t *__restrict__ lcell,
                               const uint32_t *__restrict__ cnt1, const uint32_t *__restrict__ ioff,
                               int *__restrict__ nitem) {
    int nb, nch;
    *nitem = nleaf == 0 ? 0 : int(ioff[nleaf - 1]) + m2p_items_of(nleaf - 1, lstart, lcell, cnt1, nb, nch);
}

__global__ void __launch_bounds__(256) k_ad_m2p_fill(int nleaf, const int32_t *__restrict__ lstart,
                                                     const int32_t *__restrict__ lcell,
                                                     const uint32_t *__restrict__ cnt1,
                                                     const uint32_t *__restrict__ ioff, int4 *__restrict__ items) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nleaf) return;
    int nb, nch;
    if (m2p_items_of(i, lstart, lcell, cnt1, nb, nch) == 0) return;
    for (int b = 0; b < nb; ++b)
        for (int c = 0; c < nch; ++c) items[ioff[i] + b * nch + c] = make_int4(i, 16 * b, c, nch);
}

// the chunks of a target block (consecutive items) summed in chunk order
__global__ void __launch_bounds__(64) k_ad_m2p_reduce(const int4 *__restrict__ items,
                                                      const int32_t *__restrict__ lstart, int n,
                                                      const double *__restrict__ part, double *__restrict__ far) {
    const int4 it = items[blockIdx.x];
    if (it.z != 0 || it.w <= 1) return;
    const int s0 = lstart[it.x], cnt = lstart[it.x + 1] - s0;
    for (int v = threadIdx.x; v < 12 * 16; v += 64) {
        const int o = v / 16, pi = v % 16;
        if (it.y + pi >= cnt) continue;
        double sum = 0.0;
        for (int c = 0; c < it.w; ++c) sum += part[(size_t(blockIdx.x + c) * 12 + o) * 16 + pi];
        far[size_t(o) * n + s0 + it.y + pi] += sum;
    }
}

// target blocks of bs per leaf (none for a leaf whose gate count is zero,
// when a gate is given), then the (leaf, first target) items
__device__ __forceinline__ int leaf_blocks(int i, const int32_t *__restrict__ lstart,
                                           const int32_t *__restrict__ lcell, const uint32_t *__restrict__ gate,
                                           int bs) {
    if (gate != nullptr && gate[lcell[i]] == 0u) return 0;
    return (lstart[i + 1] - lstart[i] + bs - 1) / bs;
}

__global__ void __launch_bounds__(256) k_ad_block_count(int nleaf, const int32_t *__restrict__ lstart,
                                                        const int32_t *__restrict__ lcell,
                                                        const uint32_t *__restrict__ gate, int bs,
                                                        uint32_t *__restrict__ nb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nleaf) nb[i] = uint32_t(leaf_blocks(i, lstart, lcell, gate, bs));
}

__global__ void __launch_bounds__(256) k_ad_block_fill(int nleaf, const int32_t *__restrict__ lstart,
                                                       const int32_t *__restrict__ lcell,
                                                       const uint32_t *__restrict__ gate, int bs,
                                                       const uint32_t *__restrict__ boff, int2 *__restrict__ items,
                                                       int *__restrict__ nitem) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nleaf) return;
    const int nb = leaf_blocks(i, lstart, lcell, gate, bs);
    if (i == nleaf - 1) *nitem = int(boff[i]) + nb;
    for (int b = 0; b < nb; ++b) items[boff[i] + b] = make_int2(i, bs * b);
}

inline int blocks(int n, int t) { return (n + t - 1) / t; }

}  // namespace

hipError_t launch_ad_groups(hipStream_t s, const AdTreeView &t, int ncell, int nlev, uint32_t *ka, int32_t *va,
                            uint32_t *kb, int32_t *vb, uint32_t *hist, int *starts) {
    if (ncell == 0 || nlev * 8 > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_ad_group_keys, dim3(blocks(ncell, 256)), dim3(256), 0, s, t, ncell, ka, va);
    int bits = 0;
    while ((1 << bits) < nlev * 8) ++bits;
    hipError_t e = launch_radix_pass(s, ncell, 0, bits, ka, va, kb, vb, hist);
    if (e != hipSuccess) return e;
    const int nblk = (ncell + kRadixTile - 1) / kRadixTile;
    hipLaunchKernelGGL(k_ad_group_starts, dim3(blocks(nlev * 8, 256)), dim3(256), 0, s, nlev * 8, nblk, ncell,
                       (const uint32_t *)hist, starts);
    return hipGetLastError();
}

hipError_t launch_ad_p2p_meta(hipStream_t s, const AdTreeView &t, int ncell, const uint32_t *off,
                              const uint32_t *cnt, const int32_t *src, const int8_t *code, P2PMeta *meta) {
    if (ncell == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ad_p2p_meta, dim3(blocks(ncell, 64)), dim3(64), 0, s, t, ncell, off, cnt, src, code, meta);
    return hipGetLastError();
}

hipError_t launch_ad_centres(hipStream_t s, const AdTreeView &t, int ncell, double *ctr) {
    if (ncell == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ad_centres, dim3(blocks(ncell, 256)), dim3(256), 0, s, t, ncell, ctr);
    return hipGetLastError();
}

hipError_t launch_ad_root(hipStream_t s, const AdTreeView &t, int n) {
    hipLaunchKernelGGL(k_ad_root, dim3(1), dim3(64), 0, s, t, n);
    return hipGetLastError();
}

hipError_t launch_ad_level(hipStream_t s, const AdTreeView &t, int off, int ncl, const uint32_t *fine,
                           int32_t *sstart, int32_t *scount, uint32_t *rank, uint32_t *tile_sums, int *nnext) {
    const int slots = 8 * ncl;
    hipLaunchKernelGGL(k_ad_children, dim3(blocks(slots, 256)), dim3(256), 0, s, t, off, ncl, fine, sstart, scount,
                       rank);
    hipError_t e = launch_exclusive_scan(s, slots, rank, tile_sums);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ad_emit, dim3(blocks(slots, 256)), dim3(256), 0, s, t, off, ncl,
                       (const int32_t *)sstart, (const int32_t *)scount, (const uint32_t *)rank, nnext);
    return hipGetLastError();
}

hipError_t launch_ad_no_children(hipStream_t s, const AdTreeView &t, int off, int ncl) {
    hipLaunchKernelGGL(k_ad_no_children, dim3(blocks(8 * ncl, 256)), dim3(256), 0, s, t, off, ncl);
    return hipGetLastError();
}

hipError_t launch_ad_leaves(hipStream_t s, const AdTreeView &t, int ncell, int n, int32_t *leaf_at, uint32_t *rank,
                            uint32_t *tile_sums, int32_t *lcell, int32_t *lstart, int32_t *llev, int *nleaf_out) {
    hipError_t e = hipMemsetAsync(leaf_at, 0xff, sizeof(int32_t) * size_t(n), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ad_leaf_mark, dim3(blocks(ncell, 256)), dim3(256), 0, s, t, ncell, leaf_at);
    hipLaunchKernelGGL(k_ad_leaf_flag, dim3(blocks(n, 256)), dim3(256), 0, s, n, (const int32_t *)leaf_at, rank);
    e = launch_exclusive_scan(s, n, rank, tile_sums);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ad_leaf_compact, dim3(blocks(n, 256)), dim3(256), 0, s, t, n, (const int32_t *)leaf_at,
                       (const uint32_t *)rank, lcell, lstart, llev, nleaf_out);
    return hipGetLastError();
}

hipError_t launch_ad_permute(hipStream_t s, const AdTreeView &t, int n, const double *x, const double *alpha,
                             const int32_t *perm, int nleaf, const int32_t *lcell, Part64 *parts) {
    hipLaunchKernelGGL(k_ad_permute, dim3(nleaf), dim3(64), 0, s, t, n, x, alpha, perm, lcell, parts);
    return hipGetLastError();
}

hipError_t launch_ad_traverse(hipStream_t s, const AdTreeView &t, const AdLists &ls, int l, int off, int ncl,
                              int pass, int vcell0, int ncell) {
    if (ncl == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ad_traverse, dim3(ncl), dim3(64), 0, s, t, ls, l, off, ncl, pass, vcell0, ncell);
    return hipGetLastError();
}

hipError_t launch_ad_p2l(hipStream_t s, const AdTreeView &t, const AdLists &ls, int off, int ncl, int ncell, int p,
                         int kp, const DevTables &tab, const Part64 *parts, double *L) {
    const int C = (p + 1) * (p + 1);
    const size_t smem = sizeof(double) * (size_t(64) * (C + 1) + 64 * 3);
    hipLaunchKernelGGL(k_ad_p2l, dim3(ncl), dim3(64), smem, s, t, ls, off, ncl, ncell, p, kp, tab, parts, L);
    return hipGetLastError();
}

hipError_t launch_ad_m2p(hipStream_t s, const AdTreeView &t, const AdLists &ls, int nitem, const int4 *items,
                         const int32_t *lcell, const int32_t *lstart, int n, int ncell, int p, int kp, int nrow,
                         int nharm, const DevTables &tab, const int32_t *rowptr, const int32_t *col,
                         const int32_t *harm, const double *w, const double *G, const Part64 *parts, const double *M,
                         double *far, double *part) {
    if (nitem == 0) return hipSuccess;
    const size_t smem = sizeof(double) * (size_t(nharm) * 16 + size_t(3) * kp);
    hipLaunchKernelGGL(k_ad_m2p, dim3(nitem), dim3(64), smem, s, t, ls, items, lcell, lstart, n, ncell, p, kp, nrow,
                       nharm, tab, rowptr, col, harm, w, G, parts, M, far, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ad_m2p_reduce, dim3(nitem), dim3(64), 0, s, items, lstart, n, (const double *)part, far);
    return hipGetLastError();
}

hipError_t launch_ad_m2p_count(hipStream_t s, int nleaf, const int32_t *lstart, const int32_t *lcell,
                               const uint32_t *cnt1, uint32_t *ioff, uint32_t *tile_sums, int *nitem_out) {
    hipLaunchKernelGGL(k_ad_m2p_count, dim3(blocks(nleaf, 256)), dim3(256), 0, s, nleaf, lstart, lcell, cnt1, ioff);
    hipError_t e = launch_exclusive_scan(s, nleaf, ioff, tile_sums);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ad_m2p_total, dim3(1), dim3(1), 0, s, nleaf, lstart, lcell, cnt1, (const uint32_t *)ioff,
                       nitem_out);
    return hipGetLastError();
}

hipError_t launch_ad_m2p_fill(hipStream_t s, int nleaf, const int32_t *lstart, const int32_t *lcell,
                              const uint32_t *cnt1, const uint32_t *ioff, int4 *items) {
    hipLaunchKernelGGL(k_ad_m2p_fill, dim3(blocks(nleaf, 256)), dim3(256), 0, s, nleaf, lstart, lcell, cnt1, ioff,
                       items);
    return hipGetLastError();
}

hipError_t launch_ad_blocks(hipStream_t s, int nleaf, const int32_t *lstart, const int32_t *lcell,
                            const uint32_t *gate, int bs, uint32_t *rank, uint32_t *tile_sums, int2 *items,
                            int *nitem_out) {
    hipLaunchKernelGGL(k_ad_block_count, dim3(blocks(nleaf, 256)), dim3(256), 0, s, nleaf, lstart, lcell, gate, bs,
                       rank);
    hipError_t e = launch_exclusive_scan(s, nleaf, rank, tile_sums);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ad_block_fill, dim3(blocks(nleaf, 256)), dim3(256), 0, s, nleaf, lstart, lcell, gate, bs,
                       (const uint32_t *)rank, items, nitem_out);
    return hipGetLastError();
}

}  // namespace vmfmm
