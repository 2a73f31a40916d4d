// Launchers of the gfx950 kernels (defined in the .hip files) and the
// device-side layouts they share with the host driver.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace vmfmm {

// Sorted particle record: position relative to its leaf centre, strength.
struct __align__(64) Part64 { double dx, dy, dz, ax, ay, az, pad0, pad1; };
struct __align__(32) Part32 { float dx, dy, dz, ax, ay, az, pad0, pad1; };

struct TreeGeom {
    double lo[3];
    double box_len;
    double inv_len;   // fl(1 / box_len)
    double inv_w;     // 2^level * inv_len
    double w;         // box_len * 2^-level (leaf width)
    int level;
    int periodic;
};

// --- tree build (kernels_tree.hip) ----------------------------------------
constexpr int kRadixThreads = 256;
constexpr int kRadixItems = 16;
constexpr int kRadixTile = kRadixThreads * kRadixItems;

hipError_t launch_keys(hipStream_t s, int n, const double *x, const TreeGeom &g, int check,
                       uint32_t *keys, int32_t *idx, int *flag);
hipError_t launch_radix_pass(hipStream_t s, int n, int shift, int bits, const uint32_t *kin,
                             const int32_t *vin, uint32_t *kout, int32_t *vout, uint32_t *hist);
hipError_t launch_ranges(hipStream_t s, int n, int nleaf, const uint32_t *keys, int32_t *start);
hipError_t launch_permute(hipStream_t s, int n, const double *x, const double *alpha,
                          const int32_t *perm, const uint32_t *keys, const TreeGeom &g,
                          Part64 *p64, Part32 *p32);
hipError_t launch_iota(hipStream_t s, int n, int32_t *idx, uint32_t *keys);
// In-place exclusive prefix sum of data[0..total); tile_sums holds at least
// scan_tile_sums(total) words of scratch.
hipError_t launch_exclusive_scan(hipStream_t s, int total, uint32_t *data, uint32_t *tile_sums);
inline int scan_tile_sums(int total) { return (total + 4095) / 4096 + 1; }

// --- expansions (kernels_fmm.hip) -------------------------------------------
struct DevTables {
    // recurrence constants for balanced regular harmonics (index n(n+1)/2 + m)
    const double *c1_64, *c2_64, *diag_64;
    const float *c1_32, *c2_32, *diag_32;
    // L2P sparse table: rows (3 nu + 9 ng) x width, stored entry-major [width][rows]
    const int32_t *l2p_idx;
    const double *l2p_w64;
    const float *l2p_w32;
    int l2p_width, nu, ng;
};

// Leaves of an adaptive tree in particle order: leaf i holds the sorted
// particles start[i] .. start[i+1]-1, sits at tree level lev[i] (its width
// box_len 2^-lev) and keeps its expansions in cell slot cell[i].  The uniform
// tree passes none (cell == nullptr): leaf i is then cell i at one width.
struct LeafMap {
    const int32_t *cell = nullptr;
    const int32_t *lev = nullptr;
    double box_len = 0.0, inv_len = 0.0;
};

// With mc_out, the multipoles go also to the class-major copy of the orbit M2L
// (mc_out[leaf][3][kc], position mc_pos[standard index]).
template <typename T>
hipError_t launch_p2m(hipStream_t s, int nleaf, const void *parts, const int32_t *start,
                      int p, int kp, double inv_w, const DevTables &tab, T *m_out,
                      const LeafMap &lm = LeafMap(), T *mc_out = nullptr, const int16_t *mc_pos = nullptr,
                      int kc = 0);

// With `near` set, L2P adds the far field it evaluates to the near field a P2P
// launch stored there (P2PArgs::near, sorted order) and writes u, grad and
// dalpha in caller order, exactly as the P2P epilogue combines them; `far` is
// then not written.
struct NearCombine {
    const double *near = nullptr;
    const int32_t *perm = nullptr;   // caller index of each sorted target
    const double *alpha = nullptr;   // caller order [3][n] (stretching)
    double *u = nullptr, *dalpha = nullptr, *grad = nullptr;
    int scheme = 0;
};

template <typename T>
hipError_t launch_l2p(hipStream_t s, int nleaf, int n, const void *parts, const int32_t *start,
                      int p, int kp, double inv_w, double w, const DevTables &tab,
                      const T *l_leaf, double *far, const LeafMap &lm = LeafMap(),
                      const NearCombine &nc = NearCombine());

// Generic translation GEMM on MFMA: mode 0 = M2L, 1 = L2L, 2 = M2M.
// `part` (part_elems elements of T, may be null) is scratch for M2L launches
// split over the offsets at coarse levels; without it no split is made.
// `zero_cell` (may be null) points at tr_zero_elems(kp) zeros; with it the
// FP32 M2L takes its operator-stationary form, which also needs
// tr_slack_elems(kp) readable elements after the end of `src`.  `tri`: the
// operators are truncated to n + n' <= p (zero elsewhere); the
// operator-stationary form then skips their zero tiles.
template <typename T>
hipError_t launch_translate(hipStream_t s, int mode, int level, int periodic, int p, int kp,
                            const T *ops, const int16_t *oct_lists, const int8_t *offsets,
                            const T *src, T *dst, int accumulate, T *part = nullptr,
                            size_t part_elems = 0, const T *zero_cell = nullptr, int tri = 0);
inline size_t tr_slack_elems(int kp) { return size_t((kp + 31) / 32 * 32 - kp) + 4; }
inline size_t tr_zero_elems(int kp) { return size_t(3) * kp + tr_slack_elems(kp) + 4; }

template <typename T>
hipError_t launch_lattice(hipStream_t s, int p, int kp, const double *tlat, const T *m0, T *l0);

// The translation GEMMs on an adaptive tree's cells (same MFMA kernel, the
// targets and sources from tables instead of a dense level):
//   M2L: cells tcell[oct_base[o] ..] of octant o (8 groups, key order), source
//        of pair i of target t in stab[(t - cell0) 189 + i] (-1: none), pair i
//        the i-th operator of the octant's list;
//   L2L: the same octant groups, source the parent parent[t];
//   M2M: cells tcell[0 .. ntarget) in any order, pairs the 8 children
//        child[8 t + o] (-1: none); targets without children are skipped.
struct AdaptTr {
    const int32_t *tcell = nullptr;
    int oct_base[8] = {0, 0, 0, 0, 0, 0, 0, 0};       // M2L / L2L: group o is tcell[oct_base[o] ..]
    int oct_n[8] = {0, 0, 0, 0, 0, 0, 0, 0};          //   of oct_n[o] cells
    int tile_start[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  //   first workgroup of each group
    int ntarget = 0;                                   // M2M: tcell[0 .. ntarget)
    int cell0 = 0;                                     // M2L: first cell of the stab rows
    const int32_t *stab = nullptr, *parent = nullptr, *child = nullptr;
    int part_cell0 = 0, part_cells = 0;                // M2L splits: the level's cells [part_cell0, + part_cells)
};
// M2L (mode 0) with a partial-sum buffer `part` of part_elems elements: the 189
// offsets are split over up to 189 workgroups per target tile when a level has
// too few tiles to fill the chip, and the partial sums are added in fixed order
template <typename T>
hipError_t launch_translate_adaptive(hipStream_t s, int mode, int p, int kp, const T *ops, const int16_t *oct_lists,
                                     const T *src, T *dst, int accumulate, const AdaptTr &ad, T *part = nullptr,
                                     size_t part_elems = 0);

// --- near field (kernels_p2p.hip) ---------------------------------------------
struct P2PArgs {
    int n, nleaf, level, periodic, scheme, have_far;   // n: number of targets
    double w, sigma;
    const int32_t *start;    // source leaf ranges
    const int32_t *tstart;   // target leaf ranges (= start at the particles)
    const void *tparts;      // target records, the sources' record type (= the sources at the particles)
    const int32_t *perm;     // caller index of each sorted target
    const double *alpha;  // caller order [3][n] (stretching contraction in FP64)
    const double *far;    // sorted order: u[3][n], then J[9][n]
    double *u, *dalpha, *grad;   // caller order
    // non-null: the near field only, in sorted order, to near[15][n] (u, the
    // raw gradient sums, the strength sums q alpha; rows 3.. only with grad or
    // dalpha), combined with the far field afterwards by L2P (NearCombine)
    double *near = nullptr;
};
hipError_t launch_p2p64(hipStream_t s, const P2PArgs &a, const Part64 *parts);
hipError_t launch_p2p32(hipStream_t s, const P2PArgs &a, const Part32 *parts);

// Near field of an adaptive tree: work item w is the target block items[w] =
// (leaf i in particle order, first target of the block in the leaf; blocks
// of 64); leaf i is cell lcell[i] with particles lstart[i] .. lstart[i+1]-1,
// its sources the leaves of its P2P list, entries off[c] .. off[c] + cnt[c] - 1
// of (src, code) with image shift codes; cells' particle ranges, keys and
// levels from the tree.  Same combine and output as launch_p2p64 (a.n,
// a.perm, a.alpha, a.far, a.u, a.dalpha, a.grad, a.scheme, a.have_far,
// a.sigma are used).
struct AdTreeView;
// One P2P list entry of an adaptive target leaf: the source leaf's sorted
// particle range and D = centre_b + s L - centre_a, which takes the source
// records (relative to their leaf's centre) into the target leaf's frame.
struct __align__(32) P2PMeta {
    double dx, dy, dz;
    int js, je;
};
hipError_t launch_p2p64_list(hipStream_t s, const P2PArgs &a, int nitem, const int2 *items, const int32_t *lcell,
                             const int32_t *lstart, const uint32_t *off, const uint32_t *cnt, const P2PMeta *meta,
                             const Part64 *parts);

// --- RBF interpolation (kernels_rbf.hip) --------------------------------------------
struct GaussArgs {
    int n, nleaf, level, periodic;   // n: number of targets
    double w, sigma;
    const int32_t *start;            // source leaf ranges
    const int32_t *tstart;           // target leaf ranges (the source ranges for sums at the particles)
    const void *tparts;              // target records (positions), same record type as the sources
    double *out;                     // target sorted order [3][n]
};
// Gaussian sums at the targets of the strengths held in the source records' a-fields
hipError_t launch_gauss(hipStream_t s, const GaussArgs &a, const void *parts, int mixed);
// records' a-fields <- gamma (sorted order [3][n])
hipError_t launch_pack(hipStream_t s, int n, const double *gamma, void *parts, int mixed);
hipError_t launch_gather3(hipStream_t s, int n, const int32_t *perm, const double *src, double *dst);
// cell centres of the ng^3 lattice, site (ix ng + iy) ng + iz, [3][ng^3]
hipError_t launch_lattice_sites(hipStream_t s, int ng, const double lo[3], double h, double *out);
hipError_t launch_scatter3(hipStream_t s, int n, const int32_t *perm, const double *src, double scale, double *dst);

constexpr int kRbfDotBlocks = 512;
constexpr int kRbfMaxVecs = 32;
struct RbfCoefs {
    double alpha[3];
    double c[3 * kRbfMaxVecs];   // c[3 j + component]
};
// out[3 j + c] = <w_c, v_{j,c}>, j < k <= kRbfMaxVecs, v_j = V + j ldv, fixed
// reduction order; `partial` holds 3 k kRbfDotBlocks doubles
hipError_t launch_multidot(hipStream_t s, int n, const double *w, const double *V, int64_t ldv, int k,
                           double *partial, double *out);
// w_c <- alpha_c w_c + sum_{j < k} c_{j,c} v_{j,c}
hipError_t launch_multiaxpy(hipStream_t s, int n, double *w, const double *V, int64_t ldv, int k,
                            const RbfCoefs &c);

// --- energy spectrum (kernels_spectrum.hip) -----------------------------------------
// power (+)= weighted |U|^2 scale over the ng x ng x (ng/2+1) half spectrum U (double2)
hipError_t launch_spec_power(hipStream_t s, int ng, const void *U, double scale, int first, double *power);
// E[s] = sum of power over list[start[s] .. start[s+1]), s < nshell
hipError_t launch_shell_sum(hipStream_t s, int nshell, const int32_t *start, const int32_t *list,
                            const double *power, double *E);

// --- adjoint (kernels_adjoint.hip) ------------------------------------------------
template <typename T>
hipError_t launch_l2p_adj(hipStream_t s, int nleaf, int n, const void *parts, const int32_t *start,
                          const int32_t *perm, const double *ubar, int p, int kp, double inv_w, double w,
                          const DevTables &tab, const int32_t *t_idx, const T *t_w, int width, T *lbar);
template <typename T>
hipError_t launch_p2m_adj(hipStream_t s, int nleaf, int n, const void *parts, const int32_t *start, int p, int kp,
                          double inv_w, const DevTables &tab, const int32_t *g_idx, const T *g_w, int width,
                          const T *mbar, double *adj);
hipError_t launch_parts_with64(hipStream_t s, int n, const Part64 *in, const int32_t *perm, const double *ubar,
                               Part64 *out);
hipError_t launch_parts_with32(hipStream_t s, int n, const Part32 *in, const int32_t *perm, const double *ubar,
                               Part32 *out);
hipError_t launch_adj_combine(hipStream_t s, int n, const int32_t *perm, const double *ubar, const double *alpha,
                              const double *J, const double *v, const double *Jv, const double *adj, double *xbar,
                              double *abar);

// --- time stepping and diagnostics (kernels_step.hip) --------------------------
hipError_t launch_rk_stage1(hipStream_t s, int n, double *x, double *a, const double *u, const double *sv,
                            double dt, double *xs, double *as);
hipError_t launch_rk_stage2(hipStream_t s, int n, double *x, double *a, const double *u, const double *sv,
                            double dt, const TreeGeom &g);
int diag_blocks(int n);
hipError_t launch_diagnostics(hipStream_t s, int n, const double *u, const double *J, const double *a,
                              double h3, double *part, double *out);
// Device address, on `device` (which must be current), of the static partial-sum
// array of the allocation-free diagnostics; looked up once per device.
hipError_t diag_scratch(int device, double **ptr);
size_t diag_scratch_bytes();

// --- adaptive tree (kernels_adaptive.hip) ------------------------------------------
// Cells level-major, ascending key inside a level; a cell is split when it
// holds more than ncrit particles above max_level (then it has >= 1 child).
struct AdTreeView {
    const uint32_t *key;
    const int32_t *level, *start, *count, *parent, *child;   // child: [cell][8], -1 absent
    int ncrit, max_level, periodic;
    double lo[3], box_len, inv_len;
    const double *ctr = nullptr;   // [cell][4] centres (x, y, z, 0) once launch_ad_centres has run
};
// Interaction lists: partners (unresolved touching pairs a cell hands to its
// children), the M2L table, and P2P / M2P / P2L lists in CSR form.
struct AdLists {
    int32_t *part;            // [cell][27] partner cell
    int8_t *pcode;            // [cell][27] partner image shift code
    int32_t *npart;           // [cell]
    int32_t *vtab;            // [cell][189]: M2L source per slot of the cell's octant list, -1 none
    const int16_t *vslot;     // [8][343] slot of offset d in octant o's M2L list (-1: not in it)
    uint32_t *cnt;            // [3][ncell] counts of the P2P, M2P, P2L lists (counting pass)
    const uint32_t *off;      // [3][ncell] exclusive offsets into the payload (filling pass)
    int32_t *src[3];          // list payloads (one buffer): source cell
    int8_t *code[3];          //   and its image shift code (sx+1) + 3 (sy+1) + 9 (sz+1)
    int *err;                 // set on a partner overflow or an M2L offset outside the list
};
hipError_t launch_ad_root(hipStream_t s, const AdTreeView &t, int n);
// Octant groups of every level at once: the cells sorted stably by
// (level, octant) into vb (ka, va, kb scratch of ncell words; hist the radix
// histogram, as for a pass over ncell keys), starts[level * 8 + octant] the
// first position of each group and starts[8 nlev] = ncell (device ints).
hipError_t launch_ad_groups(hipStream_t s, const AdTreeView &t, int ncell, int nlev, uint32_t *ka, int32_t *va,
                            uint32_t *kb, int32_t *vb, uint32_t *hist, int *starts);
// meta[e] of every P2P list entry e of the ncell cells (list 0 of off / cnt)
hipError_t launch_ad_p2p_meta(hipStream_t s, const AdTreeView &t, int ncell, const uint32_t *off,
                              const uint32_t *cnt, const int32_t *src, const int8_t *code, P2PMeta *meta);
// the centres of the ncell cells into ctr[cell][4] (the cell-particle and near
// field kernels read them instead of decoding keys)
hipError_t launch_ad_centres(hipStream_t s, const AdTreeView &t, int ncell, double *ctr);
// children of the cells [off, off + ncl) of one level; writes the next level's
// cells from off + ncl on, and their number to *nnext
hipError_t launch_ad_level(hipStream_t s, const AdTreeView &t, int off, int ncl, const uint32_t *fine_keys,
                           int32_t *slot_start, int32_t *slot_count, uint32_t *rank, uint32_t *tile_sums,
                           int *nnext);
// marks the cells [off, off + ncl) of the last level as childless
hipError_t launch_ad_no_children(hipStream_t s, const AdTreeView &t, int off, int ncl);
// leaves in particle order: lcell, lstart (nleaf + 1), llev; *nleaf_out
hipError_t launch_ad_leaves(hipStream_t s, const AdTreeView &t, int ncell, int n, int32_t *leaf_at, uint32_t *rank,
                            uint32_t *tile_sums, int32_t *lcell, int32_t *lstart, int32_t *llev, int *nleaf_out);
// target blocks of bs of the leaves (particle order): items (leaf, first
// target), their number in *nitem_out; with a gate (per cell, indexed through
// lcell) only the leaves whose gate count is non-zero; rank / tile_sums
// scratch of nleaf words
hipError_t launch_ad_blocks(hipStream_t s, int nleaf, const int32_t *lstart, const int32_t *lcell,
                            const uint32_t *gate, int bs, uint32_t *rank, uint32_t *tile_sums, int2 *items,
                            int *nitem_out);
// sorted FP64 records relative to each leaf's centre
hipError_t launch_ad_permute(hipStream_t s, const AdTreeView &t, int n, const double *x, const double *alpha,
                             const int32_t *perm, int nleaf, const int32_t *lcell, Part64 *parts);
// dual traversal of the cells [off, off + ncl) of level l (l < 0: each cell at
// its own level, for pass 1 over cells of several levels): pass 0 counts the
// list entries and records the partners, pass 1 fills the lists (entries of
// list k of cell c at off[k ncell + c] ..) and the M2L table (row c - vcell0)
hipError_t launch_ad_traverse(hipStream_t s, const AdTreeView &t, const AdLists &ls, int l, int off, int ncl,
                              int pass, int vcell0, int ncell);
// P2L: local expansions of the cells [off, off + ncl) (holding L2L and M2L)
// += the particles of the source leaves of their P2L lists
hipError_t launch_ad_p2l(hipStream_t s, const AdTreeView &t, const AdLists &ls, int off, int ncl, int ncell, int p,
                         int kp, const DevTables &tab, const Part64 *parts, double *L);
// M2P: far[12][n] of the particles of the target blocks `items` += the
// derivatives of the source cells' multipoles (m2p_table layout; tab's
// recurrence of degree >= p + 2)
hipError_t launch_ad_m2p(hipStream_t s, const AdTreeView &t, const AdLists &ls, int nitem, const int4 *items,
                         const int32_t *lcell, const int32_t *lstart, int n, int ncell, int p, int kp, int nrow, int nharm,
                         const DevTables &tab, const int32_t *rowptr, const int32_t *col, const int32_t *harm,
                         const double *w, const double *G, const Part64 *parts, const double *M, double *far,
                         double *part);
// M2P work items (leaf, first target, chunk, chunks): blocks of 16 targets of
// the leaves with an M2P list times chunks of its entries.  count: per-leaf
// item counts scanned into ioff (nleaf words; tile_sums scratch) and the total
// in *nitem_out; fill: the items (needs the total's room: nitem int4).  M2P
// takes part (nitem x 12 x 16 doubles) for the chunks' shares.
hipError_t launch_ad_m2p_count(hipStream_t s, int nleaf, const int32_t *lstart, const int32_t *lcell,
                               const uint32_t *cnt1, uint32_t *ioff, uint32_t *tile_sums, int *nitem_out);
hipError_t launch_ad_m2p_fill(hipStream_t s, int nleaf, const int32_t *lstart, const int32_t *lcell,
                              const uint32_t *cnt1, const uint32_t *ioff, int4 *items);

// rows of the translation-operator GEMM tile
inline int pad16(int c) { return (c + 15) / 16 * 16; }
inline int pad4(int c) { return (c + 3) / 4 * 4; }
// Per-component stride of the expansion buffers, [cell][3][kp]: C rounded up to
// a multiple of 32, so that every k block of 16 coefficients is one aligned
// half of a 128-byte line (FP32) and the MFMA K padding is part of the layout.
inline int coef_stride(int c) { return (c + 31) / 32 * 32; }

// Operator fragment layout of the translation GEMMs: [op][row block][k block]
// [64 lanes][4], row blocks padded to whole groups of 8 (one per wave), k
// steps (4 coefficients each) padded to a multiple of 8, the padding zero, so
// no guard is needed inside the MFMA loop.  A k block is four k steps: lane l
// of row block rb holds, for k step 4b+s, element (rb*16 + l%16,
// tr_col(4b+s, l/16)) of the operator at position s of its 16-byte quad:
// k step 4b+s takes column 16b + 4h + s in lane group h.
constexpr int kTrWaveCount = 8;
inline int tr_nrb(int C) { return (pad16(C) / 16 + kTrWaveCount - 1) / kTrWaveCount * kTrWaveCount; }
inline int tr_nks(int C) { return (pad4(C) + 31) / 32 * 8; }
inline size_t tr_frag(int C) { return size_t(tr_nrb(C)) * tr_nks(C) * 64; }
inline int tr_col(int ks, int h) { return 16 * (ks >> 2) + 4 * h + (ks & 3); }


// --- reflection-symmetric M2L (kernels_m2l_sym.hip) ---------------------------
// Reflecting the configuration in the plane x = 0 (y = 0, z = 0) multiplies each
// real coefficient of the basis by a sign: (-1)^m for Re Rb_n^m and -(-1)^m for
// Im (x), +1 for Re and -1 for Im (y), (-1)^(n+m) for both (z).  The three signs
// give every coefficient a class c in 0..7 (bit a set: sign -1 under the
// reflection of axis a), and the M2L operator of a reflected offset R d is
// P_R T_d P_R with P_R = diag(chi_c(R)), chi_c(R) = (-1)^popcount(c & R).  The
// M2L of the offsets of one reflection orbit therefore needs one operator: its
// block (a, b) between classes a and b meets the sources of the orbit combined
// with the character of a ^ b (a Walsh-Hadamard transform over the orbit).
//
// Class-major layout: class c holds its coefficients in ascending standard
// index, in ceil(size / 16) blocks of 16; block k of the layout is of class
// bcls[k], with bnv[k] valid elements starting at rank brank0[k] of its class,
// which take the first bsteps[k] = ceil(bnv / 4) of the block's four k steps
// (element e of a block sits at position 4 (e % 4) + e / 4).
constexpr int kSymMaxBlk = 16;
struct SymLayout {
    int p = 0, C = 0, nblk = 0;
    int csize[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int bcls[kSymMaxBlk] = {}, bnv[kSymMaxBlk] = {}, bsteps[kSymMaxBlk] = {}, brank0[kSymMaxBlk] = {};
};

// class of the coefficient at standard index i (n n for m = 0, n n + 2m - 1 for
// Re, n n + 2m for Im)
constexpr int sym_class(int i) {
    int n = 0;
    while ((n + 1) * (n + 1) <= i) ++n;
    const int r = i - n * n;
    const int m = (r + 1) / 2, im = (r > 0 && r % 2 == 0) ? 1 : 0;
    return ((m & 1) ^ im) | (im << 1) | (((n + m) & 1) << 2);
}

// nblk = 0 when a class needs more than kSymMaxBlk blocks in total
constexpr SymLayout sym_layout(int p) {
    SymLayout L;
    L.p = p;
    L.C = (p + 1) * (p + 1);
    for (int i = 0; i < L.C; ++i) ++L.csize[sym_class(i)];
    int k = 0;
    for (int c = 0; c < 8; ++c)
        for (int r = 0; r < L.csize[c]; r += 16) {
            if (k == kSymMaxBlk) {
                L.nblk = 0;
                return L;
            }
            L.bcls[k] = c;
            L.brank0[k] = r;
            L.bnv[k] = L.csize[c] - r < 16 ? L.csize[c] - r : 16;
            L.bsteps[k] = (L.bnv[k] + 3) / 4;
            ++k;
        }
    L.nblk = k;
    return L;
}

// The 56 orbits of the octant-0 interaction list under the reflections that
// keep it (axes with |d_a| = 1 or 2): representative r (components 0..3,
// source - target, largest >= 2), packed rx | ry << 2 | rz << 4 | G << 6 | Z << 9
// with G the axes of the orbit's reflections and Z the axes where r_a = 0.
constexpr int kSymOrbits = 56;
// coarsest level the orbit kernel runs (coarser levels have too few target cells
// to fill the chip without splitting every workgroup down to one orbit)
constexpr int kSymMinLevel = 4;

// Mc[cell][3][16 nblk] (FP32) from the standard-layout multipoles of `ncells`
// cells (M[cell][3][kp]): mc_src[16 k + q] is the standard index held at
// position q of block k (-1: zero).  Cell `ncells` of Mc is written as zeros.
template <typename T>
hipError_t launch_sym_pack(hipStream_t s, int64_t ncells, int kp, int kc, const T *M, const int16_t *mc_src, T *Mc);
// The same for the first npack cells only, the zero cell at index zero_cell.
template <typename T>
hipError_t launch_sym_pack_range(hipStream_t s, int64_t npack, int64_t zero_cell, int kp, int kc, const T *M,
                                 const int16_t *mc_src, T *Mc);
// Offset-range splits of an M2L launch of `level` with `ttn` targets per
// workgroup (enough workgroups to fill the chip, within part_elems), and the
// fixed-order sum of the splits' partials into dst (rows < C).
int translate_splits(int level, int ttn, int kp, size_t part_elems);
hipError_t launch_split_reduce(hipStream_t s, int level, int kp, int C, int nsplit, const float *part, float *dst,
                               int accumulate);
hipError_t launch_split_reduce64(hipStream_t s, int level, int kp, int C, int nsplit, const double *part,
                                 double *dst, int accumulate);
// the same over nelem = cells * 3 * kp elements of dst (the cells of a split launch)
hipError_t launch_split_reduce64_n(hipStream_t s, int64_t nelem, int kp, int C, int nsplit, const double *part,
                                   double *dst, int accumulate);
// True if the symmetric M2L kernel is built for degree p.
bool m2l_sym_supported(int p);
// M2L at `level` (FP32): dst[cell] (+)= sum over the interaction list, from the
// class-major multipoles mc of the level (zero_cell: index of a zero cell,
// relative to mc), operators ops (per octant, orbit-compact, offsets op_off
// [8][57] in floats), orbit table `orbits`, output map row_std[16 nblk].
// Splits over orbit ranges with partial sums in `part` as launch_translate.
hipError_t launch_m2l_sym(hipStream_t s, int level, int periodic, int p, int kp, const float *mc, int64_t zero_cell,
                          const float *ops, const int32_t *op_off, const int32_t *orbits, const int16_t *row_std,
                          float *dst, int accumulate, float *part, size_t part_elems);

// Targets and sources of one level of an adaptive tree for the FP64 orbit
// M2L: the level's cells grouped by octant, tcell[oct_base[o] ..] of oct_n[o]
// cells (global cell indices); vtab[cell - cell0][189] the source cell of each
// slot of the cell's octant list (-1: none), vslot[8][343] the slot of offset
// d = source - target (index (dx+3) + 7 (dy+3) + 49 (dz+3)) in octant o's list;
// split partials indexed by cell - part_cell0 over part_cells cells.
struct SymAdapt {
    const int32_t *tcell = nullptr, *vtab = nullptr;
    const int16_t *vslot = nullptr;
    int tile_start[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // set by the launcher
    int oct_base[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int oct_n[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int cell0 = 0, part_cell0 = 0, part_cells = 0;
};

// FP64 form of launch_m2l_sym: class-major FP64 multipoles mc (zero_cell as
// there), operators per octant stored per column slice, sl_off[8][56 nblk + 1]
// the offsets (doubles) of the slices of orbit o, column b at o nblk + b.
hipError_t launch_m2l_sym64(hipStream_t s, int level, int periodic, int p, int kp, const double *mc,
                            int64_t zero_cell, const double *ops, const int32_t *sl_off, const int32_t *orbits,
                            const int16_t *row_std, double *dst, int accumulate, double *part, size_t part_elems);
// The same for one level of an adaptive tree: mc the class-major multipoles of
// every cell (zero_cell: their count), dst the locals of every cell; the
// level's orbit ranges split over workgroups (partials in `part`) when its
// tiles do not fill the chip.
hipError_t launch_m2l_sym64_adaptive(hipStream_t s, int p, int kp, const double *mc, int64_t zero_cell,
                                     const double *ops, const int32_t *sl_off, const int32_t *orbits,
                                     const int16_t *row_std, double *dst, int accumulate, const SymAdapt &ad,
                                     double *part, size_t part_elems);

}  // namespace vmfmm
