// Host driver of the C ABI declared in include/vmfmm.h: argument checks,
// workspace and operator caches, and the launch sequence of one evaluation
// (tree -> P2M -> M2M -> lattice -> L2L/M2L per level -> L2P -> P2P).
#include "../../include/vmfmm.h"

#include <hip/hip_runtime.h>
#include <hipfft/hipfft.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <utility>
#include <vector>

#include "kernels.h"
#include "operators.h"

using namespace vmfmm;

namespace {

constexpr size_t kTrPartBytes = size_t(64) << 20;   // scratch of split M2L launches
constexpr size_t kAdSplitElems = size_t(32) << 20;  // doubles of the adaptive M2L partial sums (256 MiB)
constexpr int kAdSymMinCells = 256;   // adaptive levels with fewer cells keep the dense M2L

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (ptr) (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    // grows (never shrinks); new memory is zero-filled when `zero`
    hipError_t reserve(size_t want, bool zero = false) {
        if (want <= bytes && ptr) return hipSuccess;
        release();
        if (want == 0) want = 256;
        hipError_t e = hipMalloc(&ptr, want);
        if (e != hipSuccess) {
            ptr = nullptr;
            return e;
        }
        bytes = want;
        if (zero) e = hipMemset(ptr, 0, want);
        return e;
    }
    template <typename T> T *as() const { return static_cast<T *>(ptr); }
};

template <typename T>
hipError_t upload(DevBuf &b, const std::vector<T> &v) {
    hipError_t e = b.reserve(v.size() * sizeof(T));
    if (e != hipSuccess) return e;
    return hipMemcpy(b.ptr, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

// Operator matrices swizzled into MFMA A fragments: [op][rb][kb][64][4],
// quad element s of lane l is (rb*16 + l%16, tr_col(4 kb + s, l/16)) of the
// zero-padded operator.
template <typename T>
void swizzle(const std::vector<double> &m, int C, std::vector<T> &out, size_t base) {
    const int nrb = tr_nrb(C), nkb = tr_nks(C) / 4;
    for (int rb = 0; rb < nrb; ++rb)
        for (int kb = 0; kb < nkb; ++kb)
            for (int l = 0; l < 64; ++l)
                for (int q = 0; q < 4; ++q) {
                    const int row = rb * 16 + (l & 15), col = tr_col(4 * kb + q, l >> 4);
                    const double v = (row < C && col < C) ? m[size_t(row) * C + col] : 0.0;
                    out[base + ((size_t(rb) * nkb + kb) * 64 + l) * 4 + q] = T(v);
                }
}

struct OpSet {
    int p = -1;
    DevBuf m2l64, m2l32, m2m64, m2m32, l2l64, l2l32;
    DevBuf c1_64, c2_64, dg_64, c1_32, c2_32, dg_32;
    DevBuf l2p_idx, l2p_w64, l2p_w32;
    int width = 0, nu = 0, ng = 0;
    // adjoint: transposed operators and tables (built on first use)
    bool adj_ready = false;
    DevBuf m2lT64, m2lT32, m2mT64, m2mT32, l2lT64, l2lT32;
    DevBuf t_idx, t_w64, t_w32, g_idx, g_w64, g_w32;
    int width_t = 0, width_g = 0;
    // M2L operators truncated to n + n' <= p, and their transposes (built on first use)
    bool tri_ready = false, tri_adj_ready = false;
    DevBuf m2lt64, m2lt32, m2lTt64, m2lTt32;
    // reflection-orbit M2L (square truncation; built on first use): class maps and
    // orbits, and the operators of the forward gather and of the adjoint one
    struct SymOps {
        bool ready = false;
        DevBuf ops, off, ops64, sl64;
    };
    bool sym_ready = false;
    DevBuf sym_orb, sym_mcsrc, sym_row, sym_mcpos;   // sym_mcpos[standard index] = class-major position
    SymOps sym[2];
};

// Zeroes the entries of a C x C operator that pair target degree n (row) with
// source degree n' (column) beyond n + n' <= p.
void triangular(std::vector<double> &m, int C, int p) {
    auto deg = [](int i) { int n = 0; while ((n + 1) * (n + 1) <= i) ++n; return n; };
    for (int i = 0; i < C; ++i)
        for (int j = 0; j < C; ++j)
            if (deg(i) + deg(j) > p) m[size_t(i) * C + j] = 0.0;
}

}  // namespace

struct vm_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    // the near field runs on `side` while the far field runs on `stream`:
    // fork and join by events (default priority, non-blocking)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    std::string err;

    // workspace
    DevBuf keys_a, keys_b, vals_a, vals_b, hist, start, p64, p32, far, flag, mbuf, lbuf;
    DevBuf nearf;    // near field [15][n] of a P2P launch overlapped with the far field
    DevBuf trpart;   // partial sums of M2L launches split over the offsets (coarse levels)
    DevBuf zeros;    // a zero expansion cell read in place of missing M2L sources
    DevBuf mcbuf;    // class-major multipoles of every level for the reflection-orbit M2L
    DevBuf rk_u, rk_s, rk_x, rk_a, diag;
    DevBuf adj_u, adj_J, adj_v, adj_Jv, adj_far, adj_p64, adj_p32;
    DevBuf rbf_b, rbf_x, rbf_V, rbf_part, rbf_dots;   // RBF solve: right side, iterate, Krylov basis, reductions
    // second tree over a distinct target set (Gaussian sums at other points)
    DevBuf t_keys_a, t_keys_b, t_vals_a, t_vals_b, t_start, t_p64, t_p32;
    DevBuf rin_y, rin_w, run_J;   // reinitialisation: lattice sites, vorticity there; loop: gradient
    // energy spectrum: FFT plan and shell lists for one lattice size
    hipfftHandle fft_plan = 0;
    int fft_ng = -1, spec_ng = -1, spec_kmax = -1;
    DevBuf spec_in, spec_U, spec_power, spec_start, spec_list;
    std::map<std::pair<int, int>, std::unique_ptr<DevBuf>> lattice_t;
    int layout_p = -1, layout_prec = -1;   // layout of mbuf/lbuf
    // the particle tree's generation (bumped by every build) and what the last
    // evaluation at the particles was called with, for vm_fmm_adjoint_reuse
    uint64_t tree_gen = 0;
    struct {
        bool valid = false;
        const double *x = nullptr, *alpha = nullptr;
        int64_t n = 0;
        double sigma = 0.0;
        int p = 0, level = 0;
        vm_opts opts{};
        uint64_t gen = 0;
    } last_eval;
    // results of the last evaluation, for the debug views
    uint32_t *last_keys = nullptr;
    int32_t *last_perm = nullptr;
    int64_t last_n = 0;
    int last_level = -1;
    int last_p = -1, last_mixed = 0, last_far = 0;
    // the L2P launch of the last evaluation, re-run by vm_debug_far (the far
    // field goes straight into the outputs otherwise)
    struct {
        bool valid = false;
        int nleaf = 0, n = 0, p = 0, kp = 0, mixed = 0;
        double inv_w = 0.0, w = 0.0;
        const void *tparts = nullptr, *lptr = nullptr;
        const int32_t *tstart = nullptr;
        DevTables tab{};
    } last_l2p;

    // device-time accounting
    bool timing = false;
    std::vector<hipEvent_t> events;              // pool, two per timed launch
    std::vector<std::pair<int, int>> timed;      // (phase, first event index)

    // adaptive tree of vm_fmm_eval_adaptive: cells, leaves, lists and
    // expansions of the last call (kept for the debug views), construction
    // scratch and the tables of the cell-particle kernels
    struct Adaptive {
        DevBuf key, level, start, count, parent, child;        // cells
        DevBuf sstart, scount, rank, tsum, ints;                // construction scratch, device counters
        DevBuf leaf_at, lcell, lstart, llev, iota, items;       // leaves in particle order, target blocks
        DevBuf items16, m2p_off, m2p_part;                      // M2P work items, their offsets, partial sums
        DevBuf tpart;                                           // M2L partial sums of the offset splits
        DevBuf mc;                                              // class-major multipoles (orbit M2L)
        DevBuf ctr;                                             // cell centres
        DevBuf gk, gv;                                          // octant-group sort scratch
        DevBuf p2p_meta;                                        // P2P entries' source ranges and frame shifts
        DevBuf part, pcode, npart, vtab, cnt, off, src, code;   // traversal
        DevBuf tcell, M, L, parts;
        DevBuf rec_c1, rec_c2, rec_dg;                          // recurrence of degree p + 2
        DevBuf m2p_rowptr, m2p_col, m2p_harm, m2p_w, m2p_G, vslot;
        int rec_p = -1, m2p_p = -1, m2p_nrow = 0, m2p_nharm = 0;
        size_t cell_cap = 0;
        bool valid = false;
        int n = 0, ncell = 0, nleaf = 0, max_level = 0, ncrit = 0, periodic = 0;
        std::vector<int> level_off;                             // first cell of each level, then the end
    } ad;

    // operator caches
    std::map<int, std::unique_ptr<OpSet>> ops;
    std::map<std::pair<int, int>, std::unique_ptr<DevBuf>> lattice;
    DevBuf offsets, octlists;
    bool tables_ready = false;
};

namespace {

vm_status fail(vm_ctx *c, vm_status s, const std::string &msg) {
    if (c) c->err = msg;
    return s;
}

vm_status hip_fail(vm_ctx *c, hipError_t e, const char *what) {
    const vm_status s = (e == hipErrorOutOfMemory) ? VM_ENOMEM : VM_EDEVICE;
    return fail(c, s, std::string(what) + ": " + hipGetErrorString(e));
}

#define VM_HIP(call, what)                              \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, what); \
    } while (0)

// Brackets one launch with a pair of events when timing is enabled.
struct Timed {
    vm_ctx *ctx;
    hipStream_t st;
    int ev = -1;
    Timed(vm_ctx *c, int phase) : Timed(c, phase, c->stream) {}
    Timed(vm_ctx *c, int phase, hipStream_t stream) : ctx(c), st(stream) {
        if (!ctx->timing || ctx->timed.size() >= 65536) return;
        const size_t need = 2 * (ctx->timed.size() + 1);
        while (ctx->events.size() < need) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            ctx->events.push_back(e);
        }
        ev = int(2 * ctx->timed.size());
        ctx->timed.push_back({phase, ev});
        (void)hipEventRecord(ctx->events[ev], st);
    }
    void stop() {
        if (ev >= 0) (void)hipEventRecord(ctx->events[ev + 1], st);
        ev = -1;
    }
    ~Timed() { stop(); }
};

// Device order of each octant's 189 offsets: grouped by the parity of d
// (the parity class of the source cells), (dz, dy, dx) order inside a
// group.  Consecutive offsets then read source cells one parent apart,
// which the workgroups of an XCD share in L2; the plain (dz, dy, dx) order
// alternates between disjoint parity classes.
std::vector<int16_t> device_octant_lists() {
    const OffsetTable &t = offset_table();
    std::vector<int16_t> lists(8 * 189);
    for (int o = 0; o < 8; ++o) {
        int16_t *l = lists.data() + o * 189;
        std::memcpy(l, t.list[o], sizeof(t.list[o]));
        auto cls = [&](int16_t i) { return (t.d[i][0] & 1) | ((t.d[i][1] & 1) << 1) | ((t.d[i][2] & 1) << 2); };
        std::stable_sort(l, l + 189, [&](int16_t a, int16_t b) { return cls(a) < cls(b); });
    }
    return lists;
}

vm_status ensure_tables(vm_ctx *ctx) {
    if (ctx->tables_ready) return VM_OK;
    const OffsetTable &t = offset_table();
    std::vector<int8_t> offs(316 * 3);
    std::memcpy(offs.data(), t.d, sizeof(t.d));
    const std::vector<int16_t> lists = device_octant_lists();
    VM_HIP(upload(ctx->offsets, offs), "upload offsets");
    VM_HIP(upload(ctx->octlists, lists), "upload octant lists");
    ctx->tables_ready = true;
    return VM_OK;
}

vm_status ensure_ops(vm_ctx *ctx, int p, OpSet **out) {
    auto it = ctx->ops.find(p);
    if (it != ctx->ops.end()) {
        *out = it->second.get();
        return VM_OK;
    }
    auto set = std::make_unique<OpSet>();
    set->p = p;
    const int C = ncoef(p);
    const size_t frag = tr_frag(C);
    const OffsetTable &t = offset_table();
    std::vector<double> m(size_t(C) * C);
    {
        std::vector<double> o64(316 * frag);
        std::vector<float> o32(316 * frag);
        for (int i = 0; i < 316; ++i) {
            const double D[3] = {-double(t.d[i][0]), -double(t.d[i][1]), -double(t.d[i][2])};
            m2l_matrix(p, D, 1.0, 1.0, m.data());
            swizzle(m, C, o64, i * frag);
            swizzle(m, C, o32, i * frag);
        }
        VM_HIP(upload(set->m2l64, o64), "upload M2L");
        VM_HIP(upload(set->m2l32, o32), "upload M2L");
    }
    {
        std::vector<double> a64(8 * frag), b64(8 * frag);
        std::vector<float> a32(8 * frag), b32(8 * frag);
        for (int o = 0; o < 8; ++o) {
            const double d[3] = {((o & 1) - 0.5) * 0.5, (((o >> 1) & 1) - 0.5) * 0.5, (((o >> 2) & 1) - 0.5) * 0.5};
            m2m_matrix(p, d, 0.5, 1.0, m.data());
            swizzle(m, C, a64, o * frag);
            swizzle(m, C, a32, o * frag);
            l2l_matrix(p, d, 1.0, 0.5, m.data());
            swizzle(m, C, b64, o * frag);
            swizzle(m, C, b32, o * frag);
        }
        VM_HIP(upload(set->m2m64, a64), "upload M2M");
        VM_HIP(upload(set->m2m32, a32), "upload M2M");
        VM_HIP(upload(set->l2l64, b64), "upload L2L");
        VM_HIP(upload(set->l2l32, b32), "upload L2L");
    }
    {
        const RecTable r = rec_table(p);
        std::vector<float> f1(r.c1.begin(), r.c1.end()), f2(r.c2.begin(), r.c2.end()), fd(r.diag.begin(), r.diag.end());
        VM_HIP(upload(set->c1_64, r.c1), "upload rec");
        VM_HIP(upload(set->c2_64, r.c2), "upload rec");
        VM_HIP(upload(set->dg_64, r.diag), "upload rec");
        VM_HIP(upload(set->c1_32, f1), "upload rec");
        VM_HIP(upload(set->c2_32, f2), "upload rec");
        VM_HIP(upload(set->dg_32, fd), "upload rec");
    }
    {
        // entry-major on the device ([entry][row]): the L2P kernel's lanes take
        // consecutive rows, so each entry's loads are coalesced
        const L2PTable l = l2p_table(p);
        const int rows = 3 * l.nu + 9 * l.ng;
        std::vector<int32_t> idx(l.idx.size());
        std::vector<double> w64(l.w.size());
        for (int r = 0; r < rows; ++r)
            for (int e = 0; e < l.width; ++e) {
                idx[size_t(e) * rows + r] = l.idx[size_t(r) * l.width + e];
                w64[size_t(e) * rows + r] = l.w[size_t(r) * l.width + e];
            }
        std::vector<float> w32(w64.begin(), w64.end());
        VM_HIP(upload(set->l2p_idx, idx), "upload L2P table");
        VM_HIP(upload(set->l2p_w64, w64), "upload L2P table");
        VM_HIP(upload(set->l2p_w32, w32), "upload L2P table");
        set->width = l.width;
        set->nu = l.nu;
        set->ng = l.ng;
    }
    *out = set.get();
    ctx->ops[p] = std::move(set);
    return VM_OK;
}

vm_status ensure_lattice(vm_ctx *ctx, int p, int K, const double **out) {
    const auto key = std::make_pair(p, K);
    auto it = ctx->lattice.find(key);
    if (it == ctx->lattice.end()) {
        const int C = ncoef(p);
        std::vector<double> m(size_t(C) * C);
        lattice_matrix(p, K, m.data());
        auto b = std::make_unique<DevBuf>();
        VM_HIP(upload(*b, m), "upload lattice operator");
        it = ctx->lattice.emplace(key, std::move(b)).first;
    }
    *out = it->second->as<double>();
    return VM_OK;
}

vm_status ensure_adj_ops(vm_ctx *ctx, OpSet *set) {
    if (set->adj_ready) return VM_OK;
    const int p = set->p;
    const int C = ncoef(p);
    const size_t frag = tr_frag(C);
    const OffsetTable &t = offset_table();
    std::vector<double> m(size_t(C) * C), mt(size_t(C) * C);
    auto transpose = [&]() {
        for (int i = 0; i < C; ++i)
            for (int j = 0; j < C; ++j) mt[size_t(j) * C + i] = m[size_t(i) * C + j];
    };
    {
        // operator for offset d applied in the adjoint gather is T_{-d}^T
        std::vector<double> o64(316 * frag);
        std::vector<float> o32(316 * frag);
        for (int i = 0; i < 316; ++i) {
            const double D[3] = {double(t.d[i][0]), double(t.d[i][1]), double(t.d[i][2])};   // target - source of -d
            m2l_matrix(p, D, 1.0, 1.0, m.data());
            transpose();
            swizzle(mt, C, o64, i * frag);
            swizzle(mt, C, o32, i * frag);
        }
        VM_HIP(upload(set->m2lT64, o64), "upload M2L^T");
        VM_HIP(upload(set->m2lT32, o32), "upload M2L^T");
    }
    {
        std::vector<double> a64(8 * frag), b64(8 * frag);
        std::vector<float> a32(8 * frag), b32(8 * frag);
        for (int o = 0; o < 8; ++o) {
            const double d[3] = {((o & 1) - 0.5) * 0.5, (((o >> 1) & 1) - 0.5) * 0.5, (((o >> 2) & 1) - 0.5) * 0.5};
            m2m_matrix(p, d, 0.5, 1.0, m.data());
            transpose();
            swizzle(mt, C, a64, o * frag);
            swizzle(mt, C, a32, o * frag);
            l2l_matrix(p, d, 1.0, 0.5, m.data());
            transpose();
            swizzle(mt, C, b64, o * frag);
            swizzle(mt, C, b32, o * frag);
        }
        VM_HIP(upload(set->m2mT64, a64), "upload M2M^T");
        VM_HIP(upload(set->m2mT32, a32), "upload M2M^T");
        VM_HIP(upload(set->l2lT64, b64), "upload L2L^T");
        VM_HIP(upload(set->l2lT32, b32), "upload L2L^T");
    }
    {
        const AdjTables a = adj_tables(p);
        std::vector<float> tw(a.t_w.begin(), a.t_w.end()), gw(a.g_w.begin(), a.g_w.end());
        VM_HIP(upload(set->t_idx, a.t_idx), "upload adjoint tables");
        VM_HIP(upload(set->t_w64, a.t_w), "upload adjoint tables");
        VM_HIP(upload(set->t_w32, tw), "upload adjoint tables");
        VM_HIP(upload(set->g_idx, a.g_idx), "upload adjoint tables");
        VM_HIP(upload(set->g_w64, a.g_w), "upload adjoint tables");
        VM_HIP(upload(set->g_w32, gw), "upload adjoint tables");
        set->width_t = a.width_t;
        set->width_g = a.width_g;
    }
    set->adj_ready = true;
    return VM_OK;
}

// M2L operators truncated to n + n' <= p (forward: `adjoint` 0; transposed: 1).
vm_status ensure_tri_ops(vm_ctx *ctx, OpSet *set, int adjoint) {
    if (adjoint ? set->tri_adj_ready : set->tri_ready) return VM_OK;
    const int p = set->p;
    const int C = ncoef(p);
    const size_t frag = tr_frag(C);
    const OffsetTable &t = offset_table();
    std::vector<double> m(size_t(C) * C), mt(size_t(C) * C);
    std::vector<double> o64(316 * frag);
    std::vector<float> o32(316 * frag);
    for (int i = 0; i < 316; ++i) {
        // forward: offset d (source - target) takes T(-d); the adjoint gather T(d)^T
        const double sg = adjoint ? 1.0 : -1.0;
        const double D[3] = {sg * double(t.d[i][0]), sg * double(t.d[i][1]), sg * double(t.d[i][2])};
        m2l_matrix(p, D, 1.0, 1.0, m.data());
        triangular(m, C, p);
        if (adjoint) {
            for (int a = 0; a < C; ++a)
                for (int b = 0; b < C; ++b) mt[size_t(b) * C + a] = m[size_t(a) * C + b];
            swizzle(mt, C, o64, i * frag);
            swizzle(mt, C, o32, i * frag);
        } else {
            swizzle(m, C, o64, i * frag);
            swizzle(m, C, o32, i * frag);
        }
    }
    VM_HIP(upload(adjoint ? set->m2lTt64 : set->m2lt64, o64), "upload truncated M2L");
    VM_HIP(upload(adjoint ? set->m2lTt32 : set->m2lt32, o32), "upload truncated M2L");
    (adjoint ? set->tri_adj_ready : set->tri_ready) = true;
    return VM_OK;
}

// Tables of the reflection-orbit M2L for degree p: the class-major maps, the
// 56 orbits of the octant-0 list and, per octant, the nonzero class blocks of
// each orbit's operator with the octant's reflection folded in, in the order
// the kernel consumes them (column block b, then class offset x, then the row
// blocks of class bcls[b] ^ x), each block as 4 lane groups x its valid rows x
// 4 k steps.
// adjoint 0: the forward gather, operator T_d for offset d (source - target);
// adjoint 1: the adjoint gather, T_{-d}^T, which has the same reflection
// structure (the transpose of P T P is P T^T P).
vm_status ensure_sym_ops(vm_ctx *ctx, OpSet *set, int adjoint) {
    if (set->sym[adjoint].ready) return VM_OK;
    const int p = set->p, C = ncoef(p);
    const SymLayout SL = sym_layout(p);
    if (SL.nblk == 0) return VM_EINVAL;
    const int NB = SL.nblk, KC = 16 * NB;
    std::vector<int> members[8];
    for (int i = 0; i < C; ++i) members[sym_class(i)].push_back(i);
    std::vector<int16_t> mc_src(KC, -1), row_std(KC, -1);
    for (int k = 0; k < NB; ++k)
        for (int e = 0; e < SL.bnv[k]; ++e) {
            const int idx = members[SL.bcls[k]][SL.brank0[k] + e];
            mc_src[16 * k + 4 * (e % 4) + e / 4] = int16_t(idx);   // element e at k step e / 4 of lane group e % 4
            row_std[16 * k + e] = int16_t(idx);
        }
    std::vector<int32_t> orb;
    std::vector<std::array<int, 3>> reps;
    for (int z = 0; z < 4; ++z)
        for (int y = 0; y < 4; ++y)
            for (int x = 0; x < 4; ++x) {
                if (std::max(x, std::max(y, z)) < 2) continue;
                const int r[3] = {x, y, z};
                int G = 0, Z = 0;
                for (int a = 0; a < 3; ++a) {
                    if (r[a] == 1 || r[a] == 2) G |= 1 << a;
                    if (r[a] == 0) Z |= 1 << a;
                }
                orb.push_back(x | (y << 2) | (z << 4) | (G << 6) | (Z << 9));
                reps.push_back({x, y, z});
            }
    if (int(orb.size()) != kSymOrbits) return VM_EINVAL;
    auto chi = [](int c, int refl) { return (__builtin_popcount(unsigned(c & refl)) & 1) ? -1.0 : 1.0; };
    // FP32: per block [lane group][row][k step]; FP64: [half][lane group][row][2 k steps],
    // with the offsets of every column slice (orbit o, column b at o NB + b)
    std::vector<float> ops;
    std::vector<double> ops64;
    std::vector<int32_t> off(8 * (kSymOrbits + 1)), sl(8 * (kSymOrbits * NB + 1));
    std::vector<double> T(size_t(C) * C);
    for (int o = 0; o < 8; ++o)
        for (int j = 0; j < kSymOrbits; ++j) {
            off[o * (kSymOrbits + 1) + j] = int32_t(ops.size());
            // operator of the representative offset d (source - target): D = target - source;
            // the adjoint gather takes the transpose of the operator of -d
            const double sd = adjoint ? 1.0 : -1.0;
            const double D[3] = {sd * reps[j][0], sd * reps[j][1], sd * reps[j][2]};
            m2l_matrix(p, D, 1.0, 1.0, T.data());
            if (adjoint)
                for (int r = 0; r < C; ++r)
                    for (int c = r + 1; c < C; ++c) std::swap(T[size_t(r) * C + c], T[size_t(c) * C + r]);
            const int Z = (orb[j] >> 9) & 7;
            for (int b = 0; b < NB; ++b) {
                sl[o * (kSymOrbits * NB + 1) + j * NB + b] = int32_t(ops64.size());
                for (int x = 0; x < 8; ++x) {
                    if (x & Z) continue;
                    for (int a = 0; a < NB; ++a) {
                        if (SL.bcls[a] != (SL.bcls[b] ^ x)) continue;
                        const double sg = chi(SL.bcls[a], o) * chi(SL.bcls[b], o);
                        auto val = [&](int e, int h, int st) {
                            const int cidx = mc_src[16 * b + 4 * h + st];
                            return cidx >= 0 ? sg * T[size_t(row_std[16 * a + e]) * C + cidx] : 0.0;
                        };
                        for (int h = 0; h < 4; ++h)
                            for (int e = 0; e < SL.bnv[a]; ++e)
                                for (int st = 0; st < 4; ++st) ops.push_back(float(val(e, h, st)));
                        for (int half = 0; half < 2; ++half)
                            for (int h = 0; h < 4; ++h)
                                for (int e = 0; e < SL.bnv[a]; ++e)
                                    for (int st = 0; st < 2; ++st) ops64.push_back(val(e, h, 2 * half + st));
                    }
                }
            }
        }
    for (int o = 0; o < 8; ++o) {
        off[o * (kSymOrbits + 1) + kSymOrbits] = int32_t(ops.size());
        sl[o * (kSymOrbits * NB + 1) + kSymOrbits * NB] = int32_t(ops64.size());
    }
    OpSet::SymOps &so = set->sym[adjoint];
    VM_HIP(upload(so.ops, ops), "upload symmetric M2L");
    VM_HIP(upload(so.ops64, ops64), "upload symmetric M2L");
    VM_HIP(upload(so.sl64, sl), "upload symmetric M2L");
    VM_HIP(upload(so.off, off), "upload symmetric M2L");
    if (!set->sym_ready) {
        VM_HIP(upload(set->sym_orb, orb), "upload symmetric M2L");
        VM_HIP(upload(set->sym_mcsrc, mc_src), "upload symmetric M2L");
        VM_HIP(upload(set->sym_row, row_std), "upload symmetric M2L");
        std::vector<int16_t> mc_pos(coef_stride(C), -1);
        for (int q = 0; q < KC; ++q)
            if (mc_src[q] >= 0) mc_pos[mc_src[q]] = int16_t(q);
        VM_HIP(upload(set->sym_mcpos, mc_pos), "upload symmetric M2L");
        set->sym_ready = true;
    }
    so.ready = true;
    return VM_OK;
}

vm_status ensure_lattice_t(vm_ctx *ctx, int p, int K, const double **out) {
    const auto key = std::make_pair(p, K);
    auto it = ctx->lattice_t.find(key);
    if (it == ctx->lattice_t.end()) {
        const int C = ncoef(p);
        std::vector<double> m(size_t(C) * C), mt(size_t(C) * C);
        lattice_matrix(p, K, m.data());
        for (int i = 0; i < C; ++i)
            for (int j = 0; j < C; ++j) mt[size_t(j) * C + i] = m[size_t(i) * C + j];
        auto b = std::make_unique<DevBuf>();
        VM_HIP(upload(*b, mt), "upload lattice operator");
        it = ctx->lattice_t.emplace(key, std::move(b)).first;
    }
    *out = it->second->as<double>();
    return VM_OK;
}

bool misaligned(const void *q) { return q && (reinterpret_cast<uintptr_t>(q) & 7u); }

// Checks shared by the entry points that build the tree.
vm_status check_common(vm_ctx *ctx, int64_t n, double sigma, int level, const vm_opts *opts) {
    if (!opts) return fail(ctx, VM_EINVAL, "opts is NULL");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(ctx, VM_EINVAL, "n out of range [1, 2^31)");
    if (!(sigma > 0.0) || !std::isfinite(sigma)) return fail(ctx, VM_EINVAL, "sigma must be positive");
    if (level < 0 || level > VM_MAX_LEVEL) return fail(ctx, VM_EINVAL, "level out of range [0, 10]");
    if (!(opts->box_len > 0.0) || !std::isfinite(opts->box_len))
        return fail(ctx, VM_EINVAL, "box_len must be positive");
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(opts->box_lo[d])) return fail(ctx, VM_EINVAL, "box_lo must be finite");
    if (opts->periodic < 0 || opts->periodic > 4) return fail(ctx, VM_EINVAL, "periodic out of range [0, 4]");
    if (opts->precision != VM_FP64 && opts->precision != VM_MIXED)
        return fail(ctx, VM_EINVAL, "unknown precision");
    if (opts->truncation != VM_SQUARE && opts->truncation != VM_TRIANGULAR)
        return fail(ctx, VM_EINVAL, "unknown truncation");
    return VM_OK;
}

// The buffers one tree lives in: the particle (source) tree, or a second
// tree over a distinct set of target points.
struct TreeBufs {
    DevBuf *keys_a, *keys_b, *vals_a, *vals_b, *start, *p64, *p32;
};
TreeBufs source_bufs(vm_ctx *c) {
    return {&c->keys_a, &c->keys_b, &c->vals_a, &c->vals_b, &c->start, &c->p64, &c->p32};
}
TreeBufs target_bufs(vm_ctx *c) {
    return {&c->t_keys_a, &c->t_keys_b, &c->t_vals_a, &c->t_vals_b, &c->t_start, &c->t_p64, &c->t_p32};
}

// With check_domain: clears the flag the key kernels raise.
vm_status clear_flag(vm_ctx *ctx, const vm_opts *opts) {
    VM_HIP(ctx->flag.reserve(sizeof(int)), "alloc flag");
    if (opts->check_domain) VM_HIP(hipMemsetAsync(ctx->flag.ptr, 0, sizeof(int), ctx->stream), "clear flag");
    return VM_OK;
}

// With check_domain: reads the flag the key kernel raised (synchronises).
vm_status check_flag(vm_ctx *ctx, const vm_opts *opts) {
    if (!opts->check_domain) return VM_OK;
    int flag = 0;
    VM_HIP(hipMemcpyAsync(&flag, ctx->flag.ptr, sizeof(int), hipMemcpyDeviceToHost, ctx->stream), "read flag");
    VM_HIP(hipStreamSynchronize(ctx->stream), "synchronize");
    if (flag) return fail(ctx, VM_EDOMAIN, "non-finite or out-of-box position");
    return VM_OK;
}

// Morton keys of the particles at `level` and their stable LSD radix sort
// (Sec. 3.1 tree): on return `kin` holds the sorted keys and `vin` the caller
// index of each sorted particle (both in b's key / value buffers, which must
// hold ni entries, with ctx->hist sized for ni).  clear_flag must have run.
vm_status sort_particles(vm_ctx *ctx, const TreeBufs &b, int ni, const double *x, int level, const vm_opts *opts,
                         TreeGeom &g, uint32_t *&kin, int32_t *&vin) {
    hipStream_t s = ctx->stream;
    for (int d = 0; d < 3; ++d) g.lo[d] = opts->box_lo[d];
    g.box_len = opts->box_len;
    g.inv_len = 1.0 / opts->box_len;
    g.inv_w = std::ldexp(g.inv_len, level);
    g.w = std::ldexp(opts->box_len, -level);
    g.level = level;
    g.periodic = opts->periodic > 0;
    kin = b.keys_a->as<uint32_t>();
    vin = b.vals_a->as<int32_t>();
    uint32_t *kout = b.keys_b->as<uint32_t>();
    int32_t *vout = b.vals_b->as<int32_t>();
    VM_HIP(launch_keys(s, ni, x, g, opts->check_domain, kin, vin, ctx->flag.as<int>()), "keys");
    const int total_bits = 3 * level;
    if (total_bits > 0) {
        const int npass = (total_bits + 7) / 8;
        const int bits = (total_bits + npass - 1) / npass;
        for (int shift = 0; shift < total_bits; shift += bits) {
            const int nb = std::min(bits, total_bits - shift);
            VM_HIP(launch_radix_pass(s, ni, shift, nb, kin, vin, kout, vout, ctx->hist.as<uint32_t>()), "radix sort");
            std::swap(kin, kout);
            std::swap(vin, vout);
        }
    }
    return VM_OK;
}

// Tree of the particles (Sec. 3.1): Morton keys, stable LSD radix sort, leaf
// ranges and the sorted particle records (positions relative to their leaf
// centres, `alpha` in the strength fields), in the precision of opts, in the
// buffers `b`.  On return `perm` holds the caller index of each sorted
// particle, `parts` the records.  The particle tree (`record`) is kept for
// the debug views.  clear_flag must have run first.
vm_status build_tree(vm_ctx *ctx, const TreeBufs &b, int ni, const double *x, const double *alpha, int level,
                     const vm_opts *opts, TreeGeom &g, int32_t *&perm, void *&parts, bool record) {
    hipStream_t s = ctx->stream;
    const int mixed = opts->precision == VM_MIXED;
    const int64_t nleaf = int64_t(1) << (3 * level);
    const size_t n = size_t(ni);
    const int nblk = (ni + kRadixTile - 1) / kRadixTile;
    VM_HIP(b.keys_a->reserve(sizeof(uint32_t) * n), "alloc keys");
    VM_HIP(b.keys_b->reserve(sizeof(uint32_t) * n), "alloc keys");
    VM_HIP(b.vals_a->reserve(sizeof(int32_t) * n), "alloc perm");
    VM_HIP(b.vals_b->reserve(sizeof(int32_t) * n), "alloc perm");
    // digit counts [256][nblk] followed by the scan's tile sums
    VM_HIP(ctx->hist.reserve(sizeof(uint32_t) * (size_t(nblk) * 256 + size_t(nblk) * 256 / 4096 + 256)),
           "alloc histogram");
    VM_HIP(b.start->reserve(sizeof(int32_t) * size_t(nleaf + 1)), "alloc leaf ranges");
    // one record to spare: the FP32 P2P prefetches one record past a block's end
    if (mixed) VM_HIP(b.p32->reserve(sizeof(Part32) * (size_t(n) + 1)), "alloc particles");
    else VM_HIP(b.p64->reserve(sizeof(Part64) * n), "alloc particles");

    int32_t *start = b.start->as<int32_t>();
    uint32_t *kin = nullptr;
    int32_t *vin = nullptr;
    Timed tm(ctx, VM_PH_TREE);
    if (vm_status st = sort_particles(ctx, b, ni, x, level, opts, g, kin, vin); st != VM_OK) return st;
    VM_HIP(launch_ranges(s, ni, int(nleaf), kin, start), "leaf ranges");
    VM_HIP(launch_permute(s, ni, x, alpha, vin, kin, g, mixed ? nullptr : b.p64->as<Part64>(),
                          mixed ? b.p32->as<Part32>() : nullptr), "permute");
    if (record) {
        ++ctx->tree_gen;
        ctx->last_eval.valid = false;
        ctx->last_keys = kin;
        ctx->last_perm = vin;
        ctx->last_n = int64_t(ni);
        ctx->last_level = level;
        ctx->last_p = -1;
        ctx->last_far = 0;
        ctx->last_l2p.valid = false;
    }
    perm = vin;
    parts = mixed ? b.p32->ptr : b.p64->ptr;
    return VM_OK;
}

// Gaussian sums of the particles (x, gamma) at the m points y (y == nullptr:
// at the particles themselves), into omega [3][m] in y's order.  The
// particle tree is kept for the debug views; y gets a tree of its own.
vm_status gauss_impl(vm_ctx *ctx, int ni, const double *x, const double *gamma, int mi, const double *y,
                     double sigma, int level, const vm_opts *opts, double *omega) {
    hipStream_t s = ctx->stream;
    const int mixed = opts->precision == VM_MIXED;
    VM_HIP(ctx->rbf_b.reserve(sizeof(double) * 3 * size_t(mi)), "alloc gaussian sum");
    if (vm_status st = clear_flag(ctx, opts); st != VM_OK) return st;
    TreeGeom g;
    int32_t *perm = nullptr;
    void *parts = nullptr;
    // the records carry gamma as their strengths
    if (vm_status st = build_tree(ctx, source_bufs(ctx), ni, x, gamma, level, opts, g, perm, parts, true);
        st != VM_OK)
        return st;
    GaussArgs a;
    a.start = ctx->start.as<int32_t>();
    a.tstart = a.start;
    a.tparts = parts;
    int32_t *tperm = perm;
    if (y) {
        TreeGeom gt;
        void *tp = nullptr;
        if (vm_status st = build_tree(ctx, target_bufs(ctx), mi, y, y, level, opts, gt, tperm, tp, false);
            st != VM_OK)
            return st;
        a.tstart = ctx->t_start.as<int32_t>();
        a.tparts = tp;
    }
    a.n = mi;
    a.nleaf = 1 << (3 * level);
    a.level = level;
    a.periodic = opts->periodic > 0;
    a.w = g.w;
    a.sigma = sigma;
    a.out = ctx->rbf_b.as<double>();
    {
        Timed tm(ctx, VM_PH_GAUSS);
        VM_HIP(launch_gauss(s, a, parts, mixed), "gaussian sum");
    }
    Timed tm(ctx, VM_PH_KRYLOV);
    VM_HIP(launch_scatter3(s, mi, tperm, ctx->rbf_b.as<double>(), 1.0, omega), "scatter");
    return VM_OK;
}

// One Heun step of eqs. 7-8 with the core sigma1 at the start and sigma2 at
// the Euler prediction (sigma1 = sigma2 without diffusion).  u0, grad0: the
// initial state's velocity and gradient (may be NULL); diag (device [3] or
// NULL): E, Omega, Omega_p of the initial state for particle volume h3.
vm_status heun_impl(vm_ctx *ctx, int64_t n, double *x, double *alpha, double sigma1, double sigma2, int p,
                    int level, const vm_opts *opts, double dt, double *u0, double *grad0, double *diag, double h3) {
    const size_t bytes = sizeof(double) * 3 * size_t(n);
    VM_HIP(ctx->rk_u.reserve(bytes), "alloc rk");
    VM_HIP(ctx->rk_s.reserve(bytes), "alloc rk");
    VM_HIP(ctx->rk_x.reserve(bytes), "alloc rk");
    VM_HIP(ctx->rk_a.reserve(bytes), "alloc rk");
    double *u = u0 ? u0 : ctx->rk_u.as<double>();
    double *sv = ctx->rk_s.as<double>();
    double *J = grad0;
    if (diag && !J) {
        VM_HIP(ctx->run_J.reserve(sizeof(double) * 9 * size_t(n)), "alloc gradient");
        J = ctx->run_J.as<double>();
    }
    vm_status st = vm_fmm_eval(ctx, n, x, alpha, sigma1, p, level, opts, u, sv, J);
    if (st != VM_OK) return st;
    const int ni = int(n);
    if (diag) {
        VM_HIP(ctx->diag.reserve(sizeof(double) * 3 * 1024), "alloc diagnostics");
        VM_HIP(launch_diagnostics(ctx->stream, ni, u, J, alpha, h3, ctx->diag.as<double>(), diag), "diagnostics");
    }
    VM_HIP(launch_rk_stage1(ctx->stream, ni, x, alpha, u, sv, dt, ctx->rk_x.as<double>(), ctx->rk_a.as<double>()),
           "rk stage 1");
    u = ctx->rk_u.as<double>();
    st = vm_fmm_eval(ctx, n, ctx->rk_x.as<double>(), ctx->rk_a.as<double>(), sigma2, p, level, opts, u, sv, nullptr);
    if (st != VM_OK) return st;
    TreeGeom g;
    for (int d = 0; d < 3; ++d) g.lo[d] = opts->box_lo[d];
    g.box_len = opts->box_len;
    g.inv_len = 1.0 / opts->box_len;
    g.inv_w = 0.0;
    g.w = 0.0;
    g.level = level;
    g.periodic = opts->periodic > 0;
    VM_HIP(launch_rk_stage2(ctx->stream, ni, x, alpha, u, sv, dt, g), "rk stage 2");
    return VM_OK;
}

// One forward Euler step (the paper's integrator): x + dt u, alpha + dt
// dalpha/dt, positions wrapped when periodic.  diag as for heun_impl.
vm_status euler_impl(vm_ctx *ctx, int64_t n, double *x, double *alpha, double sigma, int p, int level,
                     const vm_opts *opts, double dt, double *diag, double h3) {
    const size_t bytes = sizeof(double) * 3 * size_t(n);
    VM_HIP(ctx->rk_u.reserve(bytes), "alloc rk");
    VM_HIP(ctx->rk_s.reserve(bytes), "alloc rk");
    double *u = ctx->rk_u.as<double>(), *sv = ctx->rk_s.as<double>(), *J = nullptr;
    if (diag) {
        VM_HIP(ctx->run_J.reserve(sizeof(double) * 9 * size_t(n)), "alloc gradient");
        J = ctx->run_J.as<double>();
    }
    vm_status st = vm_fmm_eval(ctx, n, x, alpha, sigma, p, level, opts, u, sv, J);
    if (st != VM_OK) return st;
    const int ni = int(n);
    if (diag) {
        VM_HIP(ctx->diag.reserve(sizeof(double) * 3 * 1024), "alloc diagnostics");
        VM_HIP(launch_diagnostics(ctx->stream, ni, u, J, alpha, h3, ctx->diag.as<double>(), diag), "diagnostics");
    }
    TreeGeom g;
    for (int d = 0; d < 3; ++d) g.lo[d] = opts->box_lo[d];
    g.box_len = opts->box_len;
    g.inv_len = 1.0 / opts->box_len;
    g.inv_w = 0.0;
    g.w = 0.0;
    g.level = level;
    g.periodic = opts->periodic > 0;
    // the second Heun stage with twice the step is x + dt u, alpha + dt s
    VM_HIP(launch_rk_stage2(ctx->stream, ni, x, alpha, u, sv, 2.0 * dt, g), "euler update");
    return VM_OK;
}

// Reinitialisation onto the ng^3 lattice: the vorticity the particles carry
// with core sigma at the lattice sites, interpolated with core sigma0 there
// (GMRES from h^3 omega); x <- sites, alpha <- the new strengths.
vm_status reinit_impl(vm_ctx *ctx, int64_t n, double *x, double *alpha, double sigma, int ng, double sigma0,
                      int level, const vm_opts *opts, double tol, int max_iter, int *iters, double *resid) {
    const size_t bytes = sizeof(double) * 3 * size_t(n);
    VM_HIP(ctx->rin_y.reserve(bytes), "alloc reinitialisation");
    VM_HIP(ctx->rin_w.reserve(bytes), "alloc reinitialisation");
    const double h = opts->box_len / ng;
    double *y = ctx->rin_y.as<double>(), *w = ctx->rin_w.as<double>();
    VM_HIP(launch_lattice_sites(ctx->stream, ng, opts->box_lo, h, y), "lattice sites");
    if (vm_status st = gauss_impl(ctx, int(n), x, alpha, int(n), y, sigma, level, opts, w); st != VM_OK) return st;
    if (vm_status st = check_flag(ctx, opts); st != VM_OK) return st;
    if (vm_status st = vm_rbf_solve(ctx, n, y, w, sigma0, h * h * h, level, opts, tol, max_iter, alpha, iters, resid);
        st != VM_OK)
        return st;
    VM_HIP(hipMemcpyAsync(x, y, bytes, hipMemcpyDeviceToDevice, ctx->stream), "copy sites");
    return VM_OK;
}

// One evaluation (the launch sequence of Sec. 3.1): tree, upward pass,
// lattice, downward pass, then L2P and P2P at the particles (y == nullptr)
// or at the m points y, which get a tree of their own (then no stretching).
vm_status fmm_impl(vm_ctx *ctx, int64_t n, const double *x, const double *alpha, int64_t m, const double *y,
                   double sigma, int p, int level, const vm_opts *opts, double *u, double *dalpha_dt, double *grad) {
    hipStream_t s = ctx->stream;
    const int mixed = opts->precision == VM_MIXED;
    const int K = opts->periodic;
    const int periodic = K > 0;
    const int ni = int(n);
    const int mi = y ? int(m) : ni;   // targets
    const int64_t nleaf = int64_t(1) << (3 * level);

    if (vm_status st = ensure_tables(ctx); st != VM_OK) return st;
    OpSet *ops = nullptr;
    if (vm_status st = ensure_ops(ctx, p, &ops); st != VM_OK) return st;
    if (opts->truncation == VM_TRIANGULAR)
        if (vm_status st = ensure_tri_ops(ctx, ops, 0); st != VM_OK) return st;
    // square-truncation M2L by reflection orbits where its kernel is built (from
    // level kSymMinLevel on; its source offsets are 32-bit byte offsets: levels
    // up to 7 in FP32, 6 in FP64)
    const bool use_sym = opts->truncation != VM_TRIANGULAR && m2l_sym_supported(p) && level >= kSymMinLevel &&
                         level <= (mixed ? 7 : 6);
    if (use_sym)
        if (vm_status st = ensure_sym_ops(ctx, ops, 0); st != VM_OK) return st;
    const double *tlat = nullptr;
    if (K >= 2)
        if (vm_status st = ensure_lattice(ctx, p, K, &tlat); st != VM_OK) return st;

    // workspace
    const int C = ncoef(p), kp = coef_stride(C);
    const size_t esz = mixed ? sizeof(float) : sizeof(double);
    const int64_t ncells = ((int64_t(1) << (3 * (level + 1))) - 1) / 7;
    VM_HIP(ctx->far.reserve(sizeof(double) * 12 * size_t(mi)), "alloc far field");
    VM_HIP(ctx->nearf.reserve(sizeof(double) * 15 * size_t(mi)), "alloc near field");
    VM_HIP(ctx->trpart.reserve(kTrPartBytes), "alloc split partials");
    if (ctx->zeros.bytes == 0) VM_HIP(ctx->zeros.reserve(tr_zero_elems(coef_stride(ncoef(VM_MAX_P))) * sizeof(double), true),
                                      "alloc zero cell");
    // slack after the last cell: the FP32 M2L reads up to a k block past a component
    const size_t cbytes = (size_t(ncells) * 3 * kp + tr_slack_elems(kp)) * esz;
    const bool relayout = ctx->layout_p != p || ctx->layout_prec != mixed;
    if (relayout || ctx->mbuf.bytes < cbytes) {
        // coefficient padding (rows C..kp-1) must stay zero: clear on any change of layout
        // (the class-major copy's padding too: P2M writes only its valid positions)
        ctx->mbuf.release();
        ctx->lbuf.release();
        ctx->mcbuf.release();
        VM_HIP(ctx->mbuf.reserve(cbytes, true), "alloc multipoles");
        VM_HIP(ctx->lbuf.reserve(cbytes, true), "alloc locals");
        ctx->layout_p = p;
        ctx->layout_prec = mixed;
    }

    if (use_sym)
        VM_HIP(ctx->mcbuf.reserve(esz * size_t(ncells + 1) * 3 * (16 * sym_layout(p).nblk), true),
               "alloc class-major multipoles");

    // --- tree ------------------------------------------------------------
    TreeGeom g;
    int32_t *vin = nullptr;
    void *pv = nullptr;
    if (vm_status st = clear_flag(ctx, opts); st != VM_OK) return st;
    if (vm_status st = build_tree(ctx, source_bufs(ctx), ni, x, alpha, level, opts, g, vin, pv, true); st != VM_OK)
        return st;
    int32_t *start = ctx->start.as<int32_t>();
    ctx->last_p = p;
    ctx->last_mixed = mixed;
    const void *parts = pv;
    // targets: the particles, or the points y in a second tree at the same level
    const void *tparts = parts;
    const int32_t *tstart = start;
    int32_t *tperm = vin;
    if (y) {
        TreeGeom gt;
        void *tp = nullptr;
        if (vm_status st = build_tree(ctx, target_bufs(ctx), mi, y, y, level, opts, gt, tperm, tp, false);
            st != VM_OK)
            return st;
        tparts = tp;
        tstart = ctx->t_start.as<int32_t>();
    }

    // --- near field (side stream) and far field (stream), then combine -------
    const int lmin = periodic ? 0 : 2;
    const bool far = level >= lmin && !(periodic && K < 2 && level == 0);
    ctx->last_far = far;
    P2PArgs a;
    a.n = mi;
    a.nleaf = int(nleaf);
    a.level = level;
    a.periodic = periodic;
    a.scheme = opts->scheme;
    a.have_far = far ? 1 : 0;
    a.w = g.w;
    a.sigma = sigma;
    a.start = start;
    a.tstart = tstart;
    a.tparts = tparts;
    a.perm = tperm;
    a.alpha = alpha;
    a.far = ctx->far.as<double>();
    a.u = u;
    a.dalpha = y ? nullptr : dalpha_dt;
    a.grad = grad;
    auto near_field = [&](hipStream_t st, const P2PArgs &args) -> vm_status {
        Timed tm(ctx, VM_PH_P2P, st);
        if (mixed) VM_HIP(launch_p2p32(st, args, ctx->p32.as<Part32>()), "P2P");
        else VM_HIP(launch_p2p64(st, args, ctx->p64.as<Part64>()), "P2P");
        return VM_OK;
    };
    if (far) {
        // the near field (VALU) alongside the far field's launches (MFMA,
        // latency-bound small levels), into the near buffer; L2P joins
        P2PArgs an = a;
        an.have_far = 0;
        an.near = ctx->nearf.as<double>();
        VM_HIP(hipEventRecord(ctx->ev_fork, s), "fork");
        VM_HIP(hipStreamWaitEvent(ctx->side, ctx->ev_fork, 0), "fork");
        if (vm_status st = near_field(ctx->side, an); st != VM_OK) return st;
        VM_HIP(hipEventRecord(ctx->ev_join, ctx->side), "join");
    }
    if (far) {
        DevTables tab;
        tab.c1_64 = ops->c1_64.as<double>(); tab.c2_64 = ops->c2_64.as<double>(); tab.diag_64 = ops->dg_64.as<double>();
        tab.c1_32 = ops->c1_32.as<float>(); tab.c2_32 = ops->c2_32.as<float>(); tab.diag_32 = ops->dg_32.as<float>();
        tab.l2p_idx = ops->l2p_idx.as<int32_t>();
        tab.l2p_w64 = ops->l2p_w64.as<double>();
        tab.l2p_w32 = ops->l2p_w32.as<float>();
        tab.l2p_width = ops->width;
        tab.nu = ops->nu;
        tab.ng = ops->ng;
        auto run = [&](auto tag) -> vm_status {
            using T = decltype(tag);
            const bool f32 = sizeof(T) == 4;
            T *M = ctx->mbuf.as<T>(), *L = ctx->lbuf.as<T>();
            auto lev = [&](T *b, int l) { return b + size_t(((int64_t(1) << (3 * l)) - 1) / 7) * 3 * kp; };
            const int tri = opts->truncation == VM_TRIANGULAR;
            const T *m2l = tri ? (f32 ? (const T *)ops->m2lt32.ptr : (const T *)ops->m2lt64.ptr)
                               : (f32 ? (const T *)ops->m2l32.ptr : (const T *)ops->m2l64.ptr);
            const T *m2m = f32 ? (const T *)ops->m2m32.ptr : (const T *)ops->m2m64.ptr;
            const T *l2l = f32 ? (const T *)ops->l2l32.ptr : (const T *)ops->l2l64.ptr;
            const int16_t *lists = ctx->octlists.as<int16_t>();
            const int8_t *offs = ctx->offsets.as<int8_t>();
            // with the orbit M2L, P2M also writes the finest level's class-major copy
            const int kc = use_sym ? 16 * sym_layout(p).nblk : 0;
            T *mc = use_sym ? ctx->mcbuf.as<T>() : nullptr;
            const int64_t base_fine = ((int64_t(1) << (3 * level)) - 1) / 7;
            {
                Timed tm(ctx, VM_PH_P2M);
                VM_HIP(launch_p2m<T>(s, int(nleaf), parts, start, p, kp, g.inv_w, tab, lev(M, level), LeafMap(),
                                     use_sym ? mc + size_t(base_fine) * 3 * kc : nullptr,
                                     ops->sym_mcpos.as<int16_t>(), kc),
                       "P2M");
            }
            for (int l = level - 1; l >= lmin; --l) {
                Timed tm(ctx, VM_PH_M2M);
                VM_HIP(launch_translate<T>(s, 2, l, periodic, p, kp, m2m, lists, offs, lev(M, l + 1), lev(M, l), 0),
                       "M2M");
            }
            const bool sym = use_sym;
            if (sym) {
                // the coarser levels' class-major copy (the finest came from P2M)
                Timed tm(ctx, VM_PH_M2L);
                VM_HIP(launch_sym_pack_range<T>(s, base_fine, ncells, kp, kc, M, ops->sym_mcsrc.as<int16_t>(), mc),
                       "M2L class-major multipoles");
            }
            bool have_parent = false;   // L at level l-1 holds something
            if (periodic && K >= 2) {
                Timed tm(ctx, VM_PH_LATTICE);
                VM_HIP(launch_lattice<T>(s, p, kp, tlat, lev(M, 0), lev(L, 0)), "lattice");
                have_parent = true;
            }
            for (int l = periodic ? 1 : 2; l <= level; ++l) {
                if (have_parent) {
                    Timed tm(ctx, VM_PH_L2L);
                    VM_HIP(launch_translate<T>(s, 1, l, periodic, p, kp, l2l, lists, offs, lev(L, l - 1), lev(L, l), 0),
                           "L2L");
                }
                Timed tm(ctx, VM_PH_M2L);
                // the orbit kernel from level 4 on; the few cells of the coarser
                // levels run the dense operators
                if (sym && l >= kSymMinLevel) {
                    const int64_t base = ((int64_t(1) << (3 * l)) - 1) / 7;
                    if constexpr (sizeof(T) == 4)
                        VM_HIP(launch_m2l_sym(s, l, periodic, p, kp, mc + size_t(base) * 3 * kc, ncells - base,
                                              ops->sym[0].ops.as<float>(), ops->sym[0].off.as<int32_t>(),
                                              ops->sym_orb.as<int32_t>(), ops->sym_row.as<int16_t>(), lev(L, l),
                                              have_parent ? 1 : 0, ctx->trpart.as<float>(),
                                              ctx->trpart.bytes / sizeof(float)),
                               "M2L");
                    else
                        VM_HIP(launch_m2l_sym64(s, l, periodic, p, kp, mc + size_t(base) * 3 * kc, ncells - base,
                                                ops->sym[0].ops64.as<double>(), ops->sym[0].sl64.as<int32_t>(),
                                                ops->sym_orb.as<int32_t>(), ops->sym_row.as<int16_t>(), lev(L, l),
                                                have_parent ? 1 : 0, ctx->trpart.as<double>(),
                                                ctx->trpart.bytes / sizeof(double)),
                               "M2L");
                } else {
                    VM_HIP(launch_translate<T>(s, 0, l, periodic, p, kp, m2l, lists, offs, lev(M, l), lev(L, l),
                                               have_parent ? 1 : 0, ctx->trpart.as<T>(), ctx->trpart.bytes / sizeof(T),
                                               ctx->zeros.as<T>(), tri),
                           "M2L");
                }
                have_parent = true;
            }
            // the near field first (side stream), then L2P adds the far field
            // and writes the outputs
            VM_HIP(hipStreamWaitEvent(s, ctx->ev_join, 0), "join");
            NearCombine nc;
            nc.near = ctx->nearf.as<double>();
            nc.perm = tperm;
            nc.alpha = alpha;
            nc.u = u;
            nc.dalpha = y ? nullptr : dalpha_dt;
            nc.grad = grad;
            nc.scheme = opts->scheme;
            auto &ll = ctx->last_l2p;
            ll = {true, int(nleaf), mi, p, kp, int(f32), g.inv_w, g.w, tparts, lev(L, level), tstart, tab};
            Timed tm(ctx, VM_PH_L2P);
            VM_HIP(launch_l2p<T>(s, int(nleaf), mi, tparts, tstart, p, kp, g.inv_w, g.w, tab, lev(L, level),
                                 ctx->far.as<double>(), LeafMap(), nc),
                   "L2P");
            return VM_OK;
        };
        vm_status st = mixed ? run(float()) : run(double());
        if (st != VM_OK) return st;
    }

    if (!far)
        if (vm_status st = near_field(s, a); st != VM_OK) return st;

    if (!y) {
        auto &le = ctx->last_eval;
        le.valid = true;
        le.x = x;
        le.alpha = alpha;
        le.n = n;
        le.sigma = sigma;
        le.p = p;
        le.level = level;
        le.opts = *opts;
        le.gen = ctx->tree_gen;
    }
    return check_flag(ctx, opts);
}

// ------------------------------------------------------------- adaptive tree ----

// Grows b to at least `want` bytes keeping its first `keep` bytes.
vm_status grow_keep(vm_ctx *ctx, DevBuf &b, size_t want, size_t keep) {
    if (want <= b.bytes && b.ptr) return VM_OK;
    void *np = nullptr;
    VM_HIP(hipMalloc(&np, want), "alloc adaptive tree");
    if (keep && b.ptr)
        VM_HIP(hipMemcpyAsync(np, b.ptr, std::min(keep, b.bytes), hipMemcpyDeviceToDevice, ctx->stream),
               "copy adaptive tree");
    VM_HIP(hipStreamSynchronize(ctx->stream), "synchronize");
    b.release();
    b.ptr = np;
    b.bytes = want;
    return VM_OK;
}

vm_status read_ints(vm_ctx *ctx, const void *dev, int *host, int count) {
    VM_HIP(hipMemcpyAsync(host, dev, sizeof(int) * size_t(count), hipMemcpyDeviceToHost, ctx->stream), "read counts");
    VM_HIP(hipStreamSynchronize(ctx->stream), "synchronize");
    return VM_OK;
}

// Cell arrays of capacity `cap` (the first `keep` cells kept).
vm_status ad_cells(vm_ctx *ctx, size_t cap, size_t keep) {
    auto &A = ctx->ad;
    if (cap <= A.cell_cap) return VM_OK;
    DevBuf *b4[] = {&A.key, &A.level, &A.start, &A.count, &A.parent};
    for (DevBuf *b : b4)
        if (vm_status st = grow_keep(ctx, *b, cap * 4, keep * 4); st != VM_OK) return st;
    if (vm_status st = grow_keep(ctx, A.child, cap * 32, keep * 32); st != VM_OK) return st;
    A.cell_cap = cap;
    return VM_OK;
}

AdTreeView ad_view(vm_ctx *ctx, const vm_opts *opts, int ncrit, int max_level) {
    auto &A = ctx->ad;
    AdTreeView t;
    t.key = A.key.as<uint32_t>();
    t.level = A.level.as<int32_t>();
    t.start = A.start.as<int32_t>();
    t.count = A.count.as<int32_t>();
    t.parent = A.parent.as<int32_t>();
    t.child = A.child.as<int32_t>();
    t.ncrit = ncrit;
    t.max_level = max_level;
    t.periodic = opts->periodic > 0;
    for (int d = 0; d < 3; ++d) t.lo[d] = opts->box_lo[d];
    t.box_len = opts->box_len;
    t.inv_len = 1.0 / opts->box_len;
    return t;
}

// Tables of the cell-particle kernels for degree p (recurrence of degree
// p + 2, the M2P table) and the slot of each M2L offset in its octant's list.
vm_status ensure_ad_tables(vm_ctx *ctx, int p) {
    auto &A = ctx->ad;
    if (A.rec_p != p) {
        const RecTable r = rec_table(p + 2);
        VM_HIP(upload(A.rec_c1, r.c1), "upload recurrence");
        VM_HIP(upload(A.rec_c2, r.c2), "upload recurrence");
        VM_HIP(upload(A.rec_dg, r.diag), "upload recurrence");
        A.rec_p = p;
    }
    if (A.m2p_p != p) {
        const M2PTable m = m2p_table(p);
        VM_HIP(upload(A.m2p_rowptr, m.rowptr), "upload M2P table");
        VM_HIP(upload(A.m2p_col, m.col), "upload M2P table");
        VM_HIP(upload(A.m2p_harm, m.harm), "upload M2P table");
        VM_HIP(upload(A.m2p_w, m.w), "upload M2P table");
        VM_HIP(upload(A.m2p_G, m.G), "upload M2P table");
        A.m2p_nrow = m.nrow;
        A.m2p_nharm = m.nharm;
        A.m2p_p = p;
    }
    if (A.vslot.bytes == 0) {
        const OffsetTable &t = offset_table();
        const std::vector<int16_t> lists = device_octant_lists();
        std::vector<int16_t> vs(8 * 343, int16_t(-1));
        for (int o = 0; o < 8; ++o)
            for (int i = 0; i < 189; ++i) {
                const int8_t *d = t.d[lists[o * 189 + i]];
                vs[o * 343 + (d[0] + 3) + 7 * (d[1] + 3) + 49 * (d[2] + 3)] = int16_t(i);
            }
        VM_HIP(upload(A.vslot, vs), "upload M2L slots");
    }
    return VM_OK;
}

// Adaptive hybrid treecode-FMM (Sec. 3.2), FP64: tree from the particles
// sorted at max_level, dual traversal into P2P / M2L / M2P / P2L lists, then
// P2M, M2M, lattice, L2L + M2L + P2L per level, L2P + M2P, P2P.
vm_status adaptive_impl(vm_ctx *ctx, int64_t n64, const double *x, const double *alpha, double sigma, int p,
                        int ncrit, int max_level, const vm_opts *opts, double *u, double *dalpha_dt, double *grad) {
    hipStream_t s = ctx->stream;
    auto &A = ctx->ad;
    const int n = int(n64);
    const int K = opts->periodic;
    if (vm_status st = ensure_tables(ctx); st != VM_OK) return st;
    OpSet *ops = nullptr;
    if (vm_status st = ensure_ops(ctx, p, &ops); st != VM_OK) return st;
    const double *tlat = nullptr;
    if (K >= 2)
        if (vm_status st = ensure_lattice(ctx, p, K, &tlat); st != VM_OK) return st;
    if (vm_status st = ensure_ad_tables(ctx, p); st != VM_OK) return st;
    // M2L by reflection orbits at the levels with enough cells (p = 10)
    const bool ad_sym = m2l_sym_supported(p);
    if (ad_sym)
        if (vm_status st = ensure_sym_ops(ctx, ops, 0); st != VM_OK) return st;
    const int C = ncoef(p), kp = coef_stride(C);
    A.valid = false;
    ++ctx->tree_gen;
    ctx->last_eval.valid = false;
    ctx->last_level = -1;   // the uniform debug views no longer describe the buffers
    ctx->last_p = -1;

    // --- particles sorted at the finest level ---------------------------------
    const TreeBufs b = source_bufs(ctx);
    const int nblk = (n + kRadixTile - 1) / kRadixTile;
    VM_HIP(b.keys_a->reserve(sizeof(uint32_t) * size_t(n)), "alloc keys");
    VM_HIP(b.keys_b->reserve(sizeof(uint32_t) * size_t(n)), "alloc keys");
    VM_HIP(b.vals_a->reserve(sizeof(int32_t) * size_t(n)), "alloc perm");
    VM_HIP(b.vals_b->reserve(sizeof(int32_t) * size_t(n)), "alloc perm");
    VM_HIP(ctx->hist.reserve(sizeof(uint32_t) * (size_t(nblk) * 256 + size_t(nblk) * 256 / 4096 + 256)),
           "alloc histogram");
    VM_HIP(A.ints.reserve(sizeof(int) * 320), "alloc counters");
    int *dints = A.ints.as<int>();
    if (vm_status st = clear_flag(ctx, opts); st != VM_OK) return st;
    TreeGeom g;
    uint32_t *kin = nullptr;
    int32_t *vin = nullptr;
    {
        Timed tm(ctx, VM_PH_TREE);
        if (vm_status st = sort_particles(ctx, b, n, x, max_level, opts, g, kin, vin); st != VM_OK) return st;
    }

    // --- cells, level by level (the host learns each level's size) -------------
    Timed tm_lists(ctx, VM_PH_LISTS);
    if (vm_status st = ad_cells(ctx, std::max<size_t>(1024, size_t(n) / size_t(std::max(ncrit, 1)) * 2 + 64), 0);
        st != VM_OK)
        return st;
    AdTreeView t = ad_view(ctx, opts, ncrit, max_level);
    VM_HIP(launch_ad_root(s, t, n), "adaptive root");
    std::vector<int> lo{0, 1};
    int off = 0, ncl = 1;
    for (int l = 0; l < max_level && ncl > 0; ++l) {
        const size_t need = size_t(off) + ncl + 8 * size_t(ncl);
        if (need > A.cell_cap) {
            if (vm_status st = ad_cells(ctx, std::max(need, 2 * A.cell_cap), size_t(off) + ncl); st != VM_OK) return st;
            t = ad_view(ctx, opts, ncrit, max_level);
        }
        const int slots = 8 * ncl;
        VM_HIP(A.sstart.reserve(sizeof(int32_t) * slots), "alloc slots");
        VM_HIP(A.scount.reserve(sizeof(int32_t) * slots), "alloc slots");
        VM_HIP(A.rank.reserve(sizeof(uint32_t) * std::max(slots, n)), "alloc ranks");
        VM_HIP(A.tsum.reserve(sizeof(uint32_t) * scan_tile_sums(std::max(slots, 3 * n + 3))), "alloc scan sums");
        VM_HIP(launch_ad_level(s, t, off, ncl, kin, A.sstart.as<int32_t>(), A.scount.as<int32_t>(),
                               A.rank.as<uint32_t>(), A.tsum.as<uint32_t>(), dints), "adaptive level");
        int nn = 0;
        if (vm_status st = read_ints(ctx, dints, &nn, 1); st != VM_OK) return st;
        off += ncl;
        ncl = nn;
        if (ncl > 0) lo.push_back(off + ncl);
    }
    if (ncl > 0) VM_HIP(launch_ad_no_children(s, t, off, ncl), "adaptive last level");
    const int ncell = lo.back();
    const int nlev = int(lo.size()) - 1;

    // --- leaves in particle order and the sorted records -----------------------
    VM_HIP(A.leaf_at.reserve(sizeof(int32_t) * size_t(n)), "alloc leaves");
    VM_HIP(A.rank.reserve(sizeof(uint32_t) * size_t(std::max(n, 3 * ncell))), "alloc ranks");
    VM_HIP(A.tsum.reserve(sizeof(uint32_t) * scan_tile_sums(std::max(n, 3 * ncell))), "alloc scan sums");
    VM_HIP(A.lcell.reserve(sizeof(int32_t) * size_t(ncell)), "alloc leaves");
    VM_HIP(A.lstart.reserve(sizeof(int32_t) * (size_t(ncell) + 1)), "alloc leaves");
    VM_HIP(A.llev.reserve(sizeof(int32_t) * size_t(ncell)), "alloc leaves");
    VM_HIP(launch_ad_leaves(s, t, ncell, n, A.leaf_at.as<int32_t>(), A.rank.as<uint32_t>(), A.tsum.as<uint32_t>(),
                            A.lcell.as<int32_t>(), A.lstart.as<int32_t>(), A.llev.as<int32_t>(), dints + 1),
           "adaptive leaves");
    int nleaf = 0;
    if (vm_status st = read_ints(ctx, dints + 1, &nleaf, 1); st != VM_OK) return st;
    // target blocks of 64 (the near field and M2P work items)
    VM_HIP(A.items.reserve(sizeof(int2) * (size_t(nleaf) + size_t(n) / 64 + 1)), "alloc work items");
    VM_HIP(launch_ad_blocks(s, nleaf, A.lstart.as<int32_t>(), nullptr, nullptr, 64, A.rank.as<uint32_t>(),
                            A.tsum.as<uint32_t>(), A.items.as<int2>(), dints + 3), "adaptive work items");
    int nitem = 0;
    if (vm_status st = read_ints(ctx, dints + 3, &nitem, 1); st != VM_OK) return st;
    VM_HIP(A.parts.reserve(sizeof(Part64) * size_t(n)), "alloc particles");
    Part64 *parts = A.parts.as<Part64>();
    VM_HIP(A.ctr.reserve(sizeof(double) * 4 * size_t(ncell)), "alloc cell centres");
    VM_HIP(launch_ad_centres(s, t, ncell, A.ctr.as<double>()), "cell centres");
    t.ctr = A.ctr.as<double>();
    VM_HIP(launch_ad_permute(s, t, n, x, alpha, vin, nleaf, A.lcell.as<int32_t>(), parts), "adaptive permute");

    // --- dual traversal: counting pass (partners), offsets, filling pass --------
    VM_HIP(A.part.reserve(sizeof(int32_t) * 27 * size_t(ncell)), "alloc partners");
    VM_HIP(A.pcode.reserve(27 * size_t(ncell)), "alloc partners");
    VM_HIP(A.npart.reserve(sizeof(int32_t) * size_t(ncell)), "alloc partners");
    VM_HIP(A.cnt.reserve(sizeof(uint32_t) * 3 * size_t(ncell)), "alloc list counts");
    VM_HIP(A.off.reserve(sizeof(uint32_t) * 3 * size_t(ncell)), "alloc list offsets");
    VM_HIP(A.vtab.reserve(sizeof(int32_t) * 189 * size_t(ncell)), "alloc M2L table");
    VM_HIP(hipMemsetAsync(dints + 2, 0, sizeof(int), s), "clear error flag");
    AdLists ls{};
    ls.part = A.part.as<int32_t>();
    ls.pcode = A.pcode.as<int8_t>();
    ls.npart = A.npart.as<int32_t>();
    ls.vtab = A.vtab.as<int32_t>();
    ls.vslot = A.vslot.as<int16_t>();
    ls.cnt = A.cnt.as<uint32_t>();
    ls.off = A.off.as<uint32_t>();
    ls.err = dints + 2;
    for (int l = 0; l < nlev; ++l)
        VM_HIP(launch_ad_traverse(s, t, ls, l, lo[l], lo[l + 1] - lo[l], 0, 0, ncell), "adaptive traversal");
    VM_HIP(hipMemcpyAsync(A.off.ptr, A.cnt.ptr, sizeof(uint32_t) * 3 * size_t(ncell), hipMemcpyDeviceToDevice, s),
           "copy list counts");
    VM_HIP(launch_exclusive_scan(s, 3 * ncell, A.off.as<uint32_t>(), A.tsum.as<uint32_t>()), "list offsets");
    uint32_t tail[2] = {0, 0};
    VM_HIP(hipMemcpyAsync(&tail[0], A.off.as<uint32_t>() + 3 * size_t(ncell) - 1, 4, hipMemcpyDeviceToHost, s),
           "read list size");
    VM_HIP(hipMemcpyAsync(&tail[1], A.cnt.as<uint32_t>() + 3 * size_t(ncell) - 1, 4, hipMemcpyDeviceToHost, s),
           "read list size");
    VM_HIP(hipStreamSynchronize(s), "synchronize");
    const size_t nentry = size_t(tail[0]) + tail[1];
    VM_HIP(A.src.reserve(sizeof(int32_t) * std::max<size_t>(nentry, 1)), "alloc lists");
    VM_HIP(A.p2p_meta.reserve(sizeof(P2PMeta) * std::max<size_t>(nentry, 1)), "alloc lists");
    VM_HIP(A.code.reserve(std::max<size_t>(nentry, 1)), "alloc lists");
    for (int k = 0; k < 3; ++k) {
        ls.src[k] = A.src.as<int32_t>();
        ls.code[k] = A.code.as<int8_t>();
    }
    VM_HIP(hipMemsetAsync(A.vtab.ptr, 0xff, sizeof(int32_t) * 189 * size_t(ncell), s), "clear M2L table");
    // the filling pass over every cell in one launch (the partners are final)
    VM_HIP(launch_ad_traverse(s, t, ls, -1, 0, ncell, 1, 0, ncell), "adaptive traversal");
    // M2P work items: blocks of 16 targets of the leaves with an M2P list, times
    // chunks of their entries (counted here, written once their number is known)
    VM_HIP(A.m2p_off.reserve(sizeof(uint32_t) * (size_t(nleaf) + 1)), "alloc work items");
    VM_HIP(launch_ad_m2p_count(s, nleaf, A.lstart.as<int32_t>(), A.lcell.as<int32_t>(), A.cnt.as<uint32_t>() + ncell,
                               A.m2p_off.as<uint32_t>(), A.tsum.as<uint32_t>(), dints + 4),
           "M2P work items");
    int err_m2p[3] = {0, 0, 0};   // error flag, (target blocks of 64), M2P items
    if (vm_status st = read_ints(ctx, dints + 2, err_m2p, 3); st != VM_OK) return st;
    const int err = err_m2p[0], nitem16 = err_m2p[2];
    if (err) return fail(ctx, VM_EDEVICE, "adaptive traversal: partner or stack overflow, or an M2L offset outside its list");
    VM_HIP(A.items16.reserve(sizeof(int4) * (size_t(nitem16) + 1)), "alloc work items");
    VM_HIP(A.m2p_part.reserve(sizeof(double) * 12 * 16 * (size_t(nitem16) + 1)), "alloc M2P partial sums");
    VM_HIP(launch_ad_m2p_fill(s, nleaf, A.lstart.as<int32_t>(), A.lcell.as<int32_t>(), A.cnt.as<uint32_t>() + ncell,
                              A.m2p_off.as<uint32_t>(), A.items16.as<int4>()),
           "M2P work items");
    tm_lists.stop();

    // --- expansions -------------------------------------------------------------
    const size_t cbytes = (size_t(ncell) * 3 * kp + tr_slack_elems(kp)) * sizeof(double);
    VM_HIP(A.M.reserve(cbytes), "alloc multipoles");
    VM_HIP(A.L.reserve(cbytes), "alloc locals");
    VM_HIP(hipMemsetAsync(A.M.ptr, 0, cbytes, s), "clear multipoles");
    VM_HIP(hipMemsetAsync(A.L.ptr, 0, cbytes, s), "clear locals");
    VM_HIP(ctx->far.reserve(sizeof(double) * 12 * size_t(n)), "alloc far field");
    VM_HIP(A.iota.reserve(sizeof(int32_t) * size_t(ncell)), "alloc cell list");
    VM_HIP(A.tcell.reserve(sizeof(int32_t) * size_t(ncell)), "alloc octant groups");
    VM_HIP(A.tpart.reserve(sizeof(double) * kAdSplitElems), "alloc M2L partial sums");
    const int ad_kc = 16 * sym_layout(p).nblk;
    if (ad_sym) VM_HIP(A.mc.reserve(sizeof(double) * (size_t(ncell) + 1) * 3 * ad_kc), "alloc class-major multipoles");
    VM_HIP(launch_iota(s, ncell, A.iota.as<int32_t>(), A.rank.as<uint32_t>()), "cell list");
    double *M = A.M.as<double>(), *L = A.L.as<double>();
    DevTables tab;
    tab.c1_64 = ops->c1_64.as<double>(); tab.c2_64 = ops->c2_64.as<double>(); tab.diag_64 = ops->dg_64.as<double>();
    tab.c1_32 = ops->c1_32.as<float>(); tab.c2_32 = ops->c2_32.as<float>(); tab.diag_32 = ops->dg_32.as<float>();
    tab.l2p_idx = ops->l2p_idx.as<int32_t>();
    tab.l2p_w64 = ops->l2p_w64.as<double>();
    tab.l2p_w32 = ops->l2p_w32.as<float>();
    tab.l2p_width = ops->width;
    tab.nu = ops->nu;
    tab.ng = ops->ng;
    DevTables tabI = tab;   // recurrence of degree p + 2 for the irregular harmonics
    tabI.c1_64 = A.rec_c1.as<double>();
    tabI.c2_64 = A.rec_c2.as<double>();
    tabI.diag_64 = A.rec_dg.as<double>();
    LeafMap lm;
    lm.cell = A.lcell.as<int32_t>();
    lm.lev = A.llev.as<int32_t>();
    lm.box_len = opts->box_len;
    lm.inv_len = 1.0 / opts->box_len;
    const int32_t *lcell = A.lcell.as<int32_t>(), *lstart = A.lstart.as<int32_t>();
    const int16_t *lists = ctx->octlists.as<int16_t>();
    {
        Timed tm(ctx, VM_PH_P2M);
        VM_HIP(launch_p2m<double>(s, nleaf, parts, lstart, p, kp, 0.0, tab, M, lm), "adaptive P2M");
    }
    for (int l = nlev - 2; l >= 0; --l) {
        AdaptTr ad;
        ad.tcell = A.iota.as<int32_t>() + lo[l];
        ad.ntarget = lo[l + 1] - lo[l];
        ad.child = t.child;
        Timed tm(ctx, VM_PH_M2M);
        VM_HIP(launch_translate_adaptive<double>(s, 2, p, kp, ops->m2m64.as<double>(), lists, M, M, 0, ad),
               "adaptive M2M");
    }
    if (ad_sym) {
        Timed tm(ctx, VM_PH_M2L);
        VM_HIP(launch_sym_pack<double>(s, ncell, kp, ad_kc, M, ops->sym_mcsrc.as<int16_t>(), A.mc.as<double>()),
               "M2L class-major multipoles");
    }
    if (K >= 2) {
        Timed tm(ctx, VM_PH_LATTICE);
        VM_HIP(launch_lattice<double>(s, p, kp, tlat, M, L), "lattice");
    }
    // octant groups of every level: one stable sort of the cells by (level,
    // octant), the groups' starts read once
    std::vector<int> gstart(size_t(8) * nlev + 1, 0);
    {
        const size_t gblk = (std::max<size_t>(size_t(n), size_t(ncell)) + kRadixTile - 1) / kRadixTile;
        VM_HIP(ctx->hist.reserve(sizeof(uint32_t) * (gblk * 256 + gblk * 256 / 4096 + 256)), "alloc histogram");
        VM_HIP(A.gk.reserve(sizeof(uint32_t) * 2 * size_t(ncell)), "alloc octant groups");
        VM_HIP(A.gv.reserve(sizeof(int32_t) * size_t(ncell)), "alloc octant groups");
        uint32_t *gk = A.gk.as<uint32_t>();
        VM_HIP(launch_ad_groups(s, t, ncell, nlev, gk, A.gv.as<int32_t>(), gk + ncell, A.tcell.as<int32_t>(),
                                ctx->hist.as<uint32_t>(), dints + 16),
               "octant groups");
        if (vm_status st = read_ints(ctx, dints + 16, gstart.data(), int(gstart.size())); st != VM_OK) return st;
    }
    for (int l = 1; l < nlev; ++l) {
        const int nl = lo[l + 1] - lo[l];
        int oc[8];
        AdaptTr ad;
        ad.tcell = A.tcell.as<int32_t>();
        for (int o = 0; o < 8; ++o) {
            ad.oct_base[o] = gstart[8 * l + o];
            ad.oct_n[o] = oc[o] = gstart[8 * l + o + 1] - gstart[8 * l + o];
        }
        ad.parent = t.parent;
        ad.stab = A.vtab.as<int32_t>();
        ad.cell0 = 0;
        ad.part_cell0 = lo[l];
        ad.part_cells = nl;
        {
            Timed tm(ctx, VM_PH_L2L);
            VM_HIP(launch_translate_adaptive<double>(s, 1, p, kp, ops->l2l64.as<double>(), lists, L, L, 1, ad),
                   "adaptive L2L");
        }
        {
            Timed tm(ctx, VM_PH_M2L);
            if (ad_sym && nl >= kAdSymMinCells) {
                SymAdapt sa;
                sa.tcell = A.tcell.as<int32_t>();
                sa.vtab = A.vtab.as<int32_t>();
                sa.vslot = A.vslot.as<int16_t>();
                for (int o = 0; o < 8; ++o) {
                    sa.oct_base[o] = ad.oct_base[o];
                    sa.oct_n[o] = oc[o];
                }
                sa.cell0 = 0;
                sa.part_cell0 = lo[l];
                sa.part_cells = nl;
                VM_HIP(launch_m2l_sym64_adaptive(s, p, kp, A.mc.as<double>(), ncell, ops->sym[0].ops64.as<double>(),
                                                 ops->sym[0].sl64.as<int32_t>(), ops->sym_orb.as<int32_t>(),
                                                 ops->sym_row.as<int16_t>(), L, 1, sa, A.tpart.as<double>(),
                                                 kAdSplitElems),
                       "adaptive M2L");
            } else {
                VM_HIP(launch_translate_adaptive<double>(s, 0, p, kp, ops->m2l64.as<double>(), lists, M, L, 1, ad,
                                                         A.tpart.as<double>(), kAdSplitElems),
                       "adaptive M2L");
            }
        }
        Timed tm(ctx, VM_PH_P2L);
        VM_HIP(launch_ad_p2l(s, t, ls, lo[l], nl, ncell, p, kp, tabI, parts, L), "adaptive P2L");
    }
    {
        Timed tm(ctx, VM_PH_L2P);
        VM_HIP(launch_l2p<double>(s, nleaf, n, parts, lstart, p, kp, 0.0, 1.0, tab, L, ctx->far.as<double>(), lm),
               "adaptive L2P");
    }
    {
        Timed tm(ctx, VM_PH_M2P);
        VM_HIP(launch_ad_m2p(s, t, ls, nitem16, A.items16.as<int4>(), lcell, lstart, n, ncell, p, kp, A.m2p_nrow,
                             A.m2p_nharm, tabI,
                             A.m2p_rowptr.as<int32_t>(), A.m2p_col.as<int32_t>(), A.m2p_harm.as<int32_t>(),
                             A.m2p_w.as<double>(), A.m2p_G.as<double>(), parts, M, ctx->far.as<double>(),
                             A.m2p_part.as<double>()),
               "adaptive M2P");
    }
    P2PArgs a{};
    a.n = n;
    a.scheme = opts->scheme;
    a.have_far = 1;
    a.sigma = sigma;
    a.perm = vin;
    a.alpha = alpha;
    a.far = ctx->far.as<double>();
    a.u = u;
    a.dalpha = dalpha_dt;
    a.grad = grad;
    {
        Timed tm(ctx, VM_PH_P2P);
        VM_HIP(launch_ad_p2p_meta(s, t, ncell, A.off.as<uint32_t>(), A.cnt.as<uint32_t>(), A.src.as<int32_t>(),
                                  A.code.as<int8_t>(), A.p2p_meta.as<P2PMeta>()),
               "adaptive P2P entries");
        VM_HIP(launch_p2p64_list(s, a, nitem, A.items.as<int2>(), lcell, lstart, A.off.as<uint32_t>(),
                                 A.cnt.as<uint32_t>(), A.p2p_meta.as<P2PMeta>(), parts),
               "adaptive P2P");
    }
    A.valid = true;
    A.n = n;
    A.ncell = ncell;
    A.nleaf = nleaf;
    A.max_level = max_level;
    A.ncrit = ncrit;
    A.periodic = K > 0;
    A.level_off = lo;
    ctx->last_keys = kin;
    ctx->last_perm = vin;
    return check_flag(ctx, opts);
}

// Solution of the (j+1) x (j+1) upper triangular system R y = g of one
// component's rotated Hessenberg matrix (column-major, leading dimension ld).
void back_substitute(const std::vector<double> &R, int ld, const std::vector<double> &g, int cols, double *y) {
    for (int i = cols - 1; i >= 0; --i) {
        double t = g[i];
        for (int l = i + 1; l < cols; ++l) t -= R[size_t(l) * ld + i] * y[l];
        const double d = R[size_t(i) * ld + i];
        y[i] = d != 0.0 ? t / d : 0.0;
    }
}


}  // namespace

extern "C" {

vm_status vm_create(vm_ctx **out, int device, void *hip_stream) {
    if (!out) return VM_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return VM_EDEVICE;
    auto *c = new (std::nothrow) vm_ctx();
    if (!c) return VM_ENOMEM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    int prev = 0;
    (void)hipGetDevice(&prev);
    bool ok = hipSetDevice(device) == hipSuccess &&
              hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) == hipSuccess &&
              hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) == hipSuccess;
    (void)hipSetDevice(prev);
    if (!ok) {
        vm_destroy(c);
        return VM_EDEVICE;
    }
    *out = c;
    return VM_OK;
}

void vm_destroy(vm_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->side) {
        (void)hipStreamSynchronize(ctx->side);
        (void)hipStreamDestroy(ctx->side);
    }
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
    for (hipEvent_t e : ctx->events) (void)hipEventDestroy(e);
    if (ctx->fft_ng > 0) (void)hipfftDestroy(ctx->fft_plan);
    delete ctx;
}

vm_status vm_set_stream(vm_ctx *ctx, void *hip_stream) {
    if (!ctx) return VM_EINVAL;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return VM_OK;
}

const char *vm_last_error(const vm_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

vm_status vm_fmm_eval(vm_ctx *ctx, int64_t n, const double *x, const double *alpha, double sigma, int p,
                      int level, const vm_opts *opts, double *u, double *dalpha_dt, double *grad) {
    if (!ctx) return VM_EINVAL;
    if (vm_status st = check_common(ctx, n, sigma, level, opts); st != VM_OK) return st;
    if (!x || !alpha || !u) return fail(ctx, VM_EINVAL, "x, alpha and u must be non-NULL");
    if (misaligned(x) || misaligned(alpha) || misaligned(u) || misaligned(dalpha_dt) || misaligned(grad))
        return fail(ctx, VM_EINVAL, "arrays must be 8-byte aligned");
    if (p < 1 || p > VM_MAX_P) return fail(ctx, VM_EINVAL, "p out of range [1, VM_MAX_P = 18]");
    if (opts->scheme != VM_CLASSIC && opts->scheme != VM_TRANSPOSE) return fail(ctx, VM_EINVAL, "unknown scheme");

    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    return fmm_impl(ctx, n, x, alpha, 0, nullptr, sigma, p, level, opts, u, dalpha_dt, grad);
}

vm_status vm_fmm_eval_at(vm_ctx *ctx, int64_t n, const double *x, const double *alpha, int64_t m, const double *y,
                         double sigma, int p, int level, const vm_opts *opts, double *u, double *grad) {
    if (!ctx) return VM_EINVAL;
    if (vm_status st = check_common(ctx, n, sigma, level, opts); st != VM_OK) return st;
    if (m < 1 || m >= (int64_t(1) << 31)) return fail(ctx, VM_EINVAL, "m out of range [1, 2^31)");
    if (!x || !alpha || !y || !u) return fail(ctx, VM_EINVAL, "x, alpha, y and u must be non-NULL");
    if (misaligned(x) || misaligned(alpha) || misaligned(y) || misaligned(u) || misaligned(grad))
        return fail(ctx, VM_EINVAL, "arrays must be 8-byte aligned");
    if (p < 1 || p > VM_MAX_P) return fail(ctx, VM_EINVAL, "p out of range [1, VM_MAX_P = 18]");
    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    return fmm_impl(ctx, n, x, alpha, m, y, sigma, p, level, opts, u, nullptr, grad);
}

vm_status vm_fmm_eval_adaptive(vm_ctx *ctx, int64_t n, const double *x, const double *alpha, double sigma, int p,
                               int ncrit, int max_level, const vm_opts *opts, double *u, double *dalpha_dt,
                               double *grad) {
    if (!ctx) return VM_EINVAL;
    if (vm_status st = check_common(ctx, n, sigma, max_level, opts); st != VM_OK) return st;
    if (p < 1 || p > VM_ADAPTIVE_MAX_P) return fail(ctx, VM_EINVAL, "p out of range [1, 14] for the adaptive tree");
    if (ncrit < 1) return fail(ctx, VM_EINVAL, "ncrit must be positive");
    if (opts->precision != VM_FP64) return fail(ctx, VM_EINVAL, "the adaptive tree computes in FP64 only");
    if (opts->truncation != VM_SQUARE) return fail(ctx, VM_EINVAL, "the adaptive tree takes the square truncation only");
    if (opts->scheme != VM_CLASSIC && opts->scheme != VM_TRANSPOSE) return fail(ctx, VM_EINVAL, "unknown scheme");
    if (!x || !alpha || !u) return fail(ctx, VM_EINVAL, "x, alpha and u must be non-NULL");
    if (misaligned(x) || misaligned(alpha) || misaligned(u) || misaligned(dalpha_dt) || misaligned(grad))
        return fail(ctx, VM_EINVAL, "arrays must be 8-byte aligned");
    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    return adaptive_impl(ctx, n, x, alpha, sigma, p, ncrit, max_level, opts, u, dalpha_dt, grad);
}

}  // extern "C"

namespace {

// The transposed FMM (vm_fmm_adjoint).  J_in: the total gradient of the
// evaluation whose tree the context still holds (the forward state is then
// not recomputed), or nullptr.
vm_status adjoint_impl(vm_ctx *ctx, int64_t n, const double *x, const double *alpha, double sigma, int p,
                       int level, const vm_opts *opts, const double *u_bar, double *x_bar, double *alpha_bar,
                       const double *J_in) {
    if (!ctx) return VM_EINVAL;
    if (!u_bar) return fail(ctx, VM_EINVAL, "u_bar must be non-NULL");
    if (reinterpret_cast<uintptr_t>(u_bar) & 7u) return fail(ctx, VM_EINVAL, "arrays must be 8-byte aligned");
    if ((x_bar && (reinterpret_cast<uintptr_t>(x_bar) & 7u)) || (alpha_bar && (reinterpret_cast<uintptr_t>(alpha_bar) & 7u)))
        return fail(ctx, VM_EINVAL, "arrays must be 8-byte aligned");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(ctx, VM_EINVAL, "n out of range [1, 2^31)");
    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    const size_t v3 = sizeof(double) * 3 * size_t(n), v9 = sizeof(double) * 9 * size_t(n);
    // 1. forward state: tree, expansions, far field and the total gradient J
    vm_status st = VM_OK;
    const double *Jf = J_in;
    if (!Jf) {
        VM_HIP(ctx->adj_u.reserve(v3), "alloc adjoint");
        VM_HIP(ctx->adj_J.reserve(v9), "alloc adjoint");
        st = vm_fmm_eval(ctx, n, x, alpha, sigma, p, level, opts, ctx->adj_u.as<double>(), nullptr,
                         ctx->adj_J.as<double>());
        if (st != VM_OK) return st;
        Jf = ctx->adj_J.as<double>();
    }
    hipStream_t s = ctx->stream;
    const int mixed = opts->precision == VM_MIXED;
    const int K = opts->periodic, periodic = K > 0;
    const int ni = int(n);
    const int64_t nleaf = int64_t(1) << (3 * level);
    const int C = ncoef(p), kp = coef_stride(C);
    OpSet *ops = ctx->ops[p].get();
    if (vm_status e = ensure_adj_ops(ctx, ops); e != VM_OK) return e;
    if (opts->truncation == VM_TRIANGULAR)
        if (vm_status e = ensure_tri_ops(ctx, ops, 1); e != VM_OK) return e;
    const double *tlat_t = nullptr;
    if (K >= 2)
        if (vm_status e = ensure_lattice_t(ctx, p, K, &tlat_t); e != VM_OK) return e;
    // the adjoint M2L by reflection orbits where the forward one runs so
    const bool use_sym = opts->truncation != VM_TRIANGULAR && m2l_sym_supported(p) && level >= kSymMinLevel &&
                         level <= (mixed ? 7 : 6);
    const int64_t ncells = ((int64_t(1) << (3 * (level + 1))) - 1) / 7;
    if (use_sym) {
        if (vm_status e = ensure_sym_ops(ctx, ops, 1); e != VM_OK) return e;
        VM_HIP(ctx->mcbuf.reserve((mixed ? sizeof(float) : sizeof(double)) * size_t(ncells + 1) * 3 *
                                  (16 * sym_layout(p).nblk)),
               "alloc class-major multipoles");
    }
    VM_HIP(ctx->adj_v.reserve(v3), "alloc adjoint");
    VM_HIP(ctx->adj_Jv.reserve(v9), "alloc adjoint");
    VM_HIP(ctx->adj_far.reserve(2 * v3), "alloc adjoint");
    if (mixed) VM_HIP(ctx->adj_p32.reserve(sizeof(Part32) * (size_t(n) + 1)), "alloc adjoint");
    else VM_HIP(ctx->adj_p64.reserve(sizeof(Part64) * n), "alloc adjoint");
    const int32_t *start = ctx->start.as<int32_t>();
    const int32_t *perm = ctx->last_perm;
    const double w = std::ldexp(opts->box_len, -level), inv_w = std::ldexp(1.0 / opts->box_len, level);
    const void *parts = mixed ? (const void *)ctx->p32.ptr : (const void *)ctx->p64.ptr;

    // 2. far field, transposed: L2P^T -> L2L^T (up) -> lattice^T -> M2M^T + M2L^T (down) -> P2M^T
    const int lmin = periodic ? 0 : 2;
    const bool far = ctx->last_far;
    if (far) {
        DevTables tab;
        tab.c1_64 = ops->c1_64.as<double>(); tab.c2_64 = ops->c2_64.as<double>(); tab.diag_64 = ops->dg_64.as<double>();
        tab.c1_32 = ops->c1_32.as<float>(); tab.c2_32 = ops->c2_32.as<float>(); tab.diag_32 = ops->dg_32.as<float>();
        tab.l2p_idx = nullptr; tab.l2p_w64 = nullptr; tab.l2p_w32 = nullptr;
        tab.l2p_width = 0; tab.nu = p * p; tab.ng = (p - 1) * (p - 1);
        auto run = [&](auto tag) -> vm_status {
            using T = decltype(tag);
            const bool f32 = sizeof(T) == 4;
            T *Mb = ctx->mbuf.as<T>(), *Lb = ctx->lbuf.as<T>();   // adjoints overwrite the forward state
            auto lev = [&](T *b, int l) { return b + size_t(((int64_t(1) << (3 * l)) - 1) / 7) * 3 * kp; };
            const int tri = opts->truncation == VM_TRIANGULAR;
            const T *m2lT = tri ? (f32 ? (const T *)ops->m2lTt32.ptr : (const T *)ops->m2lTt64.ptr)
                                : (f32 ? (const T *)ops->m2lT32.ptr : (const T *)ops->m2lT64.ptr);
            const T *m2mT = f32 ? (const T *)ops->m2mT32.ptr : (const T *)ops->m2mT64.ptr;
            const T *l2lT = f32 ? (const T *)ops->l2lT32.ptr : (const T *)ops->l2lT64.ptr;
            const T *tw = f32 ? (const T *)ops->t_w32.ptr : (const T *)ops->t_w64.ptr;
            const T *gw = f32 ? (const T *)ops->g_w32.ptr : (const T *)ops->g_w64.ptr;
            const int16_t *lists = ctx->octlists.as<int16_t>();
            const int8_t *offs = ctx->offsets.as<int8_t>();
            VM_HIP(launch_l2p_adj<T>(s, int(nleaf), ni, parts, start, perm, u_bar, p, kp, inv_w, w, tab,
                                     ops->t_idx.as<int32_t>(), tw, ops->width_t, lev(Lb, level)),
                   "L2P^T");
            const int lstart = periodic ? 1 : 2;
            auto had_l2l = [&](int l) { return l > lstart || (periodic && K >= 2 && l == 1); };
            for (int l = level; l >= lstart; --l)
                if (had_l2l(l))
                    VM_HIP(launch_translate<T>(s, 2, l - 1, periodic, p, kp, l2lT, lists, offs, lev(Lb, l),
                                               lev(Lb, l - 1), 0),
                           "L2L^T");
            bool parent = false;
            if (periodic && K >= 2) {
                VM_HIP(launch_lattice<T>(s, p, kp, tlat_t, lev(Lb, 0), lev(Mb, 0)), "lattice^T");
                parent = true;
            }
            // the local adjoints of every level are final here: class-major copy for the orbit kernel
            const int kc = 16 * sym_layout(p).nblk;
            T *mc = ctx->mcbuf.as<T>();
            if (use_sym)
                VM_HIP(launch_sym_pack<T>(s, ncells, kp, kc, Lb, ops->sym_mcsrc.as<int16_t>(), mc),
                       "M2L^T class-major local adjoints");
            for (int l = periodic ? 1 : lmin; l <= level; ++l) {
                if (parent)
                    VM_HIP(launch_translate<T>(s, 1, l, periodic, p, kp, m2mT, lists, offs, lev(Mb, l - 1),
                                               lev(Mb, l), 0),
                           "M2M^T");
                if (use_sym && l >= kSymMinLevel) {
                    const int64_t base = ((int64_t(1) << (3 * l)) - 1) / 7;
                    if constexpr (sizeof(T) == 4)
                        VM_HIP(launch_m2l_sym(s, l, periodic, p, kp, mc + size_t(base) * 3 * kc, ncells - base,
                                              ops->sym[1].ops.as<float>(), ops->sym[1].off.as<int32_t>(),
                                              ops->sym_orb.as<int32_t>(), ops->sym_row.as<int16_t>(), lev(Mb, l),
                                              parent ? 1 : 0, ctx->trpart.as<float>(),
                                              ctx->trpart.bytes / sizeof(float)),
                               "M2L^T");
                    else
                        VM_HIP(launch_m2l_sym64(s, l, periodic, p, kp, mc + size_t(base) * 3 * kc, ncells - base,
                                                ops->sym[1].ops64.as<double>(), ops->sym[1].sl64.as<int32_t>(),
                                                ops->sym_orb.as<int32_t>(), ops->sym_row.as<int16_t>(), lev(Mb, l),
                                                parent ? 1 : 0, ctx->trpart.as<double>(),
                                                ctx->trpart.bytes / sizeof(double)),
                               "M2L^T");
                } else {
                    VM_HIP(launch_translate<T>(s, 0, l, periodic, p, kp, m2lT, lists, offs, lev(Lb, l), lev(Mb, l),
                                               parent ? 1 : 0, ctx->trpart.as<T>(), ctx->trpart.bytes / sizeof(T),
                                               ctx->zeros.as<T>(), tri),
                           "M2L^T");
                }
                parent = true;
            }
            VM_HIP(launch_p2m_adj<T>(s, int(nleaf), ni, parts, start, p, kp, inv_w, tab, ops->g_idx.as<int32_t>(), gw,
                                     ops->width_g, lev(Mb, level), ctx->adj_far.as<double>()),
                   "P2M^T");
            return VM_OK;
        };
        st = mixed ? run(float()) : run(double());
        if (st != VM_OK) return st;
    }

    // 3. near field with u_bar as strengths: v and its gradient Jv (caller order)
    P2PArgs a;
    a.n = ni;
    a.nleaf = int(nleaf);
    a.level = level;
    a.periodic = periodic;
    a.scheme = 0;
    a.have_far = 0;
    a.w = w;
    a.sigma = sigma;
    a.start = start;
    a.tstart = start;
    a.tparts = mixed ? ctx->adj_p32.ptr : ctx->adj_p64.ptr;
    a.perm = perm;
    a.alpha = nullptr;
    a.far = nullptr;
    a.u = ctx->adj_v.as<double>();
    a.dalpha = nullptr;
    a.grad = ctx->adj_Jv.as<double>();
    if (mixed) {
        VM_HIP(launch_parts_with32(s, ni, ctx->p32.as<Part32>(), perm, u_bar, ctx->adj_p32.as<Part32>()), "adjoint");
        VM_HIP(launch_p2p32(s, a, ctx->adj_p32.as<Part32>()), "P2P^T");
    } else {
        VM_HIP(launch_parts_with64(s, ni, ctx->p64.as<Part64>(), perm, u_bar, ctx->adj_p64.as<Part64>()), "adjoint");
        VM_HIP(launch_p2p64(s, a, ctx->adj_p64.as<Part64>()), "P2P^T");
    }
    // 4. combine
    VM_HIP(launch_adj_combine(s, ni, perm, u_bar, alpha, Jf, ctx->adj_v.as<double>(),
                              ctx->adj_Jv.as<double>(), far ? ctx->adj_far.as<double>() : nullptr, x_bar, alpha_bar),
           "adjoint combine");
    return VM_OK;
}

}  // namespace

extern "C" {

vm_status vm_fmm_adjoint(vm_ctx *ctx, int64_t n, const double *x, const double *alpha, double sigma, int p,
                         int level, const vm_opts *opts, const double *u_bar, double *x_bar, double *alpha_bar) {
    return adjoint_impl(ctx, n, x, alpha, sigma, p, level, opts, u_bar, x_bar, alpha_bar, nullptr);
}

vm_status vm_fmm_adjoint_reuse(vm_ctx *ctx, int64_t n, const double *x, const double *alpha, double sigma, int p,
                               int level, const vm_opts *opts, const double *grad, const double *u_bar,
                               double *x_bar, double *alpha_bar) {
    if (!ctx) return VM_EINVAL;
    if (!opts || !grad) return fail(ctx, VM_EINVAL, "opts and grad must be non-NULL");
    if (misaligned(grad)) return fail(ctx, VM_EINVAL, "arrays must be 8-byte aligned");
    const auto &le = ctx->last_eval;
    const vm_opts &o = le.opts;
    const bool same = le.valid && le.gen == ctx->tree_gen && le.x == x && le.alpha == alpha && le.n == n &&
                      le.sigma == sigma && le.p == p && le.level == level && o.box_lo[0] == opts->box_lo[0] &&
                      o.box_lo[1] == opts->box_lo[1] && o.box_lo[2] == opts->box_lo[2] &&
                      o.box_len == opts->box_len && o.periodic == opts->periodic &&
                      o.precision == opts->precision && o.truncation == opts->truncation;
    if (!same) return fail(ctx, VM_EINVAL, "the context's last evaluation is not this one");
    return adjoint_impl(ctx, n, x, alpha, sigma, p, level, opts, u_bar, x_bar, alpha_bar, grad);
}

vm_status vm_rk2_step(vm_ctx *ctx, int64_t n, double *x, double *alpha, double sigma, int p, int level,
                      const vm_opts *opts, double dt, double *u0, double *grad0) {
    if (!ctx) return VM_EINVAL;
    if (!opts || !x || !alpha) return fail(ctx, VM_EINVAL, "opts, x and alpha must be non-NULL");
    if (!std::isfinite(dt)) return fail(ctx, VM_EINVAL, "dt must be finite");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(ctx, VM_EINVAL, "n out of range [1, 2^31)");
    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    return heun_impl(ctx, n, x, alpha, sigma, sigma, p, level, opts, dt, u0, grad0, nullptr, 0.0);
}

vm_status vm_reinit(vm_ctx *ctx, int64_t n, double *x, double *alpha, double sigma, int ng, double sigma0,
                    int level, const vm_opts *opts, double tol, int max_iter, int *iters, double *resid) {
    if (!ctx) return VM_EINVAL;
    if (vm_status st = check_common(ctx, n, sigma, level, opts); st != VM_OK) return st;
    if (!x || !alpha) return fail(ctx, VM_EINVAL, "x and alpha must be non-NULL");
    if (misaligned(x) || misaligned(alpha)) return fail(ctx, VM_EINVAL, "arrays must be 8-byte aligned");
    if (!(sigma0 > 0.0) || !std::isfinite(sigma0)) return fail(ctx, VM_EINVAL, "sigma0 must be positive");
    if (ng < 1 || int64_t(ng) * ng * ng != n) return fail(ctx, VM_EINVAL, "n must equal ng^3");
    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    return reinit_impl(ctx, n, x, alpha, sigma, ng, sigma0, level, opts, tol, max_iter, iters, resid);
}

vm_status vm_run(vm_ctx *ctx, int64_t n, double *x, double *alpha, double *sigma, int p, int level,
                 const vm_opts *opts, const vm_loop *lp, double *diag, int *products, double *resid) {
    if (!ctx) return VM_EINVAL;
    if (!lp || !sigma) return fail(ctx, VM_EINVAL, "loop and sigma must be non-NULL");
    if (vm_status st = check_common(ctx, n, *sigma, level, opts); st != VM_OK) return st;
    if (!x || !alpha) return fail(ctx, VM_EINVAL, "x and alpha must be non-NULL");
    if (misaligned(x) || misaligned(alpha) || misaligned(diag))
        return fail(ctx, VM_EINVAL, "arrays must be 8-byte aligned");
    if (p < 1 || p > VM_MAX_P) return fail(ctx, VM_EINVAL, "p out of range [1, VM_MAX_P = 18]");
    if (opts->scheme != VM_CLASSIC && opts->scheme != VM_TRANSPOSE) return fail(ctx, VM_EINVAL, "unknown scheme");
    if (lp->integrator != VM_EULER && lp->integrator != VM_HEUN) return fail(ctx, VM_EINVAL, "unknown integrator");
    if (!std::isfinite(lp->dt) || !(lp->dt >= 0.0)) return fail(ctx, VM_EINVAL, "dt must be finite and >= 0");
    if (!std::isfinite(lp->nu) || !(lp->nu >= 0.0)) return fail(ctx, VM_EINVAL, "nu must be finite and >= 0");
    if (lp->steps < 0 || lp->reinit_every < 0) return fail(ctx, VM_EINVAL, "steps and reinit_every must be >= 0");
    if (lp->reinit_every > 0) {
        if (lp->ng < 1 || int64_t(lp->ng) * lp->ng * lp->ng != n) return fail(ctx, VM_EINVAL, "n must equal ng^3");
        if (!(lp->tol >= 0.0) || !(lp->tol < 1.0)) return fail(ctx, VM_EINVAL, "tol out of range [0, 1)");
        if (lp->max_iter < 0 || lp->max_iter > VM_RBF_MAX_ITER) return fail(ctx, VM_EINVAL, "max_iter out of range");
    }
    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    const double sigma0 = *sigma;
    const double h3 = opts->box_len * opts->box_len * opts->box_len / double(n);
    double sg = sigma0, worst = 0.0;
    int total = 0;
    for (int step = 0; step < lp->steps; ++step) {
        // core spreading: d sigma^2 / dt = 2 nu, advanced with the step
        const double sg_next = std::sqrt(sg * sg + 2.0 * lp->nu * lp->dt);
        double *d = diag ? diag + 3 * size_t(step) : nullptr;
        vm_status st = lp->integrator == VM_EULER
                           ? euler_impl(ctx, n, x, alpha, sg, p, level, opts, lp->dt, d, h3)
                           : heun_impl(ctx, n, x, alpha, sg, sg_next, p, level, opts, lp->dt, nullptr, nullptr, d, h3);
        if (st != VM_OK) return st;
        sg = sg_next;
        if (lp->reinit_every > 0 && (step + 1) % lp->reinit_every == 0) {
            int it = 0;
            double r = 0.0;
            st = reinit_impl(ctx, n, x, alpha, sg, lp->ng, sigma0, level, opts, lp->tol, lp->max_iter, &it, &r);
            if (st != VM_OK) return st;
            total += it;
            worst = std::max(worst, r);
            sg = sigma0;
        }
    }
    *sigma = sg;
    if (products) *products = total;
    if (resid) *resid = worst;
    return VM_OK;
}

vm_status vm_diagnostics(vm_ctx *ctx, int64_t n, const double *u, const double *grad, const double *alpha,
                         double h3, double *out) {
    if (!ctx) return VM_EINVAL;
    if (!u || !out) return fail(ctx, VM_EINVAL, "u and out must be non-NULL");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(ctx, VM_EINVAL, "n out of range [1, 2^31)");
    if (!(h3 > 0.0)) return fail(ctx, VM_EINVAL, "h3 must be positive");
    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    VM_HIP(ctx->diag.reserve(sizeof(double) * 3 * 1024), "alloc diagnostics");
    VM_HIP(launch_diagnostics(ctx->stream, int(n), u, grad, alpha, h3, ctx->diag.as<double>(), out), "diagnostics");
    return VM_OK;
}

vm_status vm_diagnostics_noalloc(vm_ctx *ctx, int64_t n, const double *u, const double *grad,
                                 const double *alpha, double h3, double *out) {
    if (!ctx) return VM_EINVAL;
    if (!u || !out) return fail(ctx, VM_EINVAL, "u and out must be non-NULL");
    if (n < 1 || n >= (int64_t(1) << 31)) return fail(ctx, VM_EINVAL, "n out of range [1, 2^31)");
    if (!(h3 > 0.0)) return fail(ctx, VM_EINVAL, "h3 must be positive");
    if (size_t(3) * sizeof(double) * diag_blocks(int(n)) > diag_scratch_bytes())
        return fail(ctx, VM_EINVAL, "partial sums exceed the static scratch array");
    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    double *part = nullptr;
    VM_HIP(diag_scratch(ctx->device, &part), "hipGetSymbolAddress(scratch)");
    VM_HIP(launch_diagnostics(ctx->stream, int(n), u, grad, alpha, h3, part, out), "diagnostics");
    return VM_OK;
}

vm_status vm_gauss_sum(vm_ctx *ctx, int64_t n, const double *x, const double *gamma, double sigma, int level,
                       const vm_opts *opts, double *omega) {
    if (!ctx) return VM_EINVAL;
    if (vm_status st = check_common(ctx, n, sigma, level, opts); st != VM_OK) return st;
    if (!x || !gamma || !omega) return fail(ctx, VM_EINVAL, "x, gamma and omega must be non-NULL");
    if (misaligned(x) || misaligned(gamma) || misaligned(omega))
        return fail(ctx, VM_EINVAL, "arrays must be 8-byte aligned");
    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    if (vm_status st = gauss_impl(ctx, int(n), x, gamma, int(n), nullptr, sigma, level, opts, omega); st != VM_OK)
        return st;
    return check_flag(ctx, opts);
}

vm_status vm_gauss_eval(vm_ctx *ctx, int64_t n, const double *x, const double *gamma, int64_t m, const double *y,
                        double sigma, int level, const vm_opts *opts, double *omega) {
    if (!ctx) return VM_EINVAL;
    if (vm_status st = check_common(ctx, n, sigma, level, opts); st != VM_OK) return st;
    if (m < 1 || m >= (int64_t(1) << 31)) return fail(ctx, VM_EINVAL, "m out of range [1, 2^31)");
    if (!x || !gamma || !y || !omega) return fail(ctx, VM_EINVAL, "x, gamma, y and omega must be non-NULL");
    if (misaligned(x) || misaligned(gamma) || misaligned(y) || misaligned(omega))
        return fail(ctx, VM_EINVAL, "arrays must be 8-byte aligned");
    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    if (vm_status st = gauss_impl(ctx, int(n), x, gamma, int(m), y, sigma, level, opts, omega); st != VM_OK)
        return st;
    return check_flag(ctx, opts);
}

static_assert(VM_RBF_RESTART + 1 <= kRbfMaxVecs, "Krylov basis exceeds the multi-vector kernels");

vm_status vm_rbf_solve(vm_ctx *ctx, int64_t n, const double *x, const double *omega, double sigma, double h3,
                       int level, const vm_opts *opts, double tol, int max_iter, double *gamma, int *iters,
                       double *resid) {
    if (!ctx) return VM_EINVAL;
    if (vm_status st = check_common(ctx, n, sigma, level, opts); st != VM_OK) return st;
    if (!x || !omega || !gamma) return fail(ctx, VM_EINVAL, "x, omega and gamma must be non-NULL");
    if (misaligned(x) || misaligned(omega) || misaligned(gamma))
        return fail(ctx, VM_EINVAL, "arrays must be 8-byte aligned");
    if (!(h3 > 0.0) || !std::isfinite(h3)) return fail(ctx, VM_EINVAL, "h3 must be positive");
    if (!(tol >= 0.0) || !(tol < 1.0)) return fail(ctx, VM_EINVAL, "tol out of range [0, 1)");
    if (max_iter < 0 || max_iter > VM_RBF_MAX_ITER) return fail(ctx, VM_EINVAL, "max_iter out of range");
    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = ctx->stream;
    const int ni = int(n), mixed = opts->precision == VM_MIXED;
    const int m = VM_RBF_RESTART;
    const size_t vlen = 3 * size_t(n);
    const int64_t ldv = int64_t(vlen);
    VM_HIP(ctx->rbf_b.reserve(sizeof(double) * vlen), "alloc rbf");
    VM_HIP(ctx->rbf_x.reserve(sizeof(double) * vlen), "alloc rbf");
    VM_HIP(ctx->rbf_V.reserve(sizeof(double) * vlen * (m + 1)), "alloc rbf basis");
    VM_HIP(ctx->rbf_part.reserve(sizeof(double) * 3 * kRbfMaxVecs * kRbfDotBlocks), "alloc rbf");
    VM_HIP(ctx->rbf_dots.reserve(sizeof(double) * 3 * kRbfMaxVecs), "alloc rbf");
    TreeGeom g;
    int32_t *perm = nullptr;
    void *parts = nullptr;
    // the records' strength fields are rewritten before every product
    if (vm_status st = clear_flag(ctx, opts); st != VM_OK) return st;
    if (vm_status st = build_tree(ctx, source_bufs(ctx), ni, x, omega, level, opts, g, perm, parts, true);
        st != VM_OK)
        return st;
    if (vm_status st = check_flag(ctx, opts); st != VM_OK) return st;

    double *b = ctx->rbf_b.as<double>(), *xs = ctx->rbf_x.as<double>(), *V = ctx->rbf_V.as<double>();
    auto vec = [&](int j) { return V + size_t(j) * vlen; };
    GaussArgs ga;
    ga.n = ni;
    ga.nleaf = 1 << (3 * level);
    ga.level = level;
    ga.periodic = opts->periodic > 0;
    ga.w = g.w;
    ga.sigma = sigma;
    ga.start = ctx->start.as<int32_t>();
    ga.tstart = ga.start;
    ga.tparts = parts;
    auto matvec = [&](const double *v, double *out) -> vm_status {
        Timed tm(ctx, VM_PH_GAUSS);
        VM_HIP(launch_pack(s, ni, v, parts, mixed), "pack strengths");
        ga.out = out;
        VM_HIP(launch_gauss(s, ga, parts, mixed), "gaussian sum");
        return VM_OK;
    };
    std::vector<double> dots(3 * kRbfMaxVecs);
    // dots[3 j + c] = <w_c, v_{j,c}>, j < k (synchronises)
    auto multidot = [&](const double *w, const double *Vb, int k) -> vm_status {
        {
            Timed tm(ctx, VM_PH_KRYLOV);
            VM_HIP(launch_multidot(s, ni, w, Vb, ldv, k, ctx->rbf_part.as<double>(), ctx->rbf_dots.as<double>()),
                   "dot products");
        }
        VM_HIP(hipMemcpyAsync(dots.data(), ctx->rbf_dots.ptr, sizeof(double) * 3 * k, hipMemcpyDeviceToHost, s),
               "read dot products");
        VM_HIP(hipStreamSynchronize(s), "synchronize");
        return VM_OK;
    };
    auto axpy = [&](double *w, const double *Vb, int k, const RbfCoefs &cf) -> vm_status {
        Timed tm(ctx, VM_PH_KRYLOV);
        VM_HIP(launch_multiaxpy(s, ni, w, Vb, ldv, k, cf), "vector update");
        return VM_OK;
    };
    RbfCoefs cf;
    auto clear = [&]() { std::memset(&cf, 0, sizeof(cf)); };
    vm_status st;

    // right-hand side in sorted order; initial guess gamma_0 = h^3 omega
    {
        Timed tm(ctx, VM_PH_KRYLOV);
        VM_HIP(launch_gather3(s, ni, perm, omega, b), "gather");
        VM_HIP(hipMemcpyAsync(xs, b, sizeof(double) * vlen, hipMemcpyDeviceToDevice, s), "copy");
    }
    clear();
    for (int c = 0; c < 3; ++c) cf.alpha[c] = h3;
    if ((st = axpy(xs, V, 0, cf)) != VM_OK) return st;

    // GMRES(m) on each component's system A gamma_c = omega_c, the three run
    // in lockstep so that every product serves all of them
    const int ld = m + 1;
    std::vector<double> H[3], gv[3], cs[3], sn[3];
    for (int c = 0; c < 3; ++c) {
        H[c].assign(size_t(ld) * m, 0.0);
        gv[c].assign(ld, 0.0);
        cs[c].assign(m, 0.0);
        sn[c].assign(m, 0.0);
    }
    double beta0[3] = {0, 0, 0}, rel[3] = {0, 0, 0};
    bool done[3] = {false, false, false};
    int total = 0;
    for (int cycle = 0;; ++cycle) {
        // r = omega - A gamma into v_0
        if ((st = matvec(xs, vec(0))) != VM_OK) return st;
        clear();
        for (int c = 0; c < 3; ++c) {
            cf.alpha[c] = -1.0;
            cf.c[c] = 1.0;
        }
        if ((st = axpy(vec(0), b, 1, cf)) != VM_OK) return st;
        if ((st = multidot(vec(0), vec(0), 1)) != VM_OK) return st;
        double beta[3];
        for (int c = 0; c < 3; ++c) {
            beta[c] = std::sqrt(dots[c]);
            if (cycle == 0) {
                beta0[c] = beta[c];
                done[c] = !(beta[c] > 0.0);
            }
            rel[c] = beta0[c] > 0.0 ? beta[c] / beta0[c] : 0.0;
            if (rel[c] <= tol) done[c] = true;
        }
        if ((done[0] && done[1] && done[2]) || total >= max_iter) break;
        bool active[3];
        int cols[3] = {0, 0, 0};
        clear();
        for (int c = 0; c < 3; ++c) {
            active[c] = !done[c];
            cf.alpha[c] = active[c] ? 1.0 / beta[c] : 0.0;
            std::fill(gv[c].begin(), gv[c].end(), 0.0);
            gv[c][0] = beta[c];
        }
        if ((st = axpy(vec(0), V, 0, cf)) != VM_OK) return st;
        for (int j = 0; j < m && total < max_iter && (active[0] || active[1] || active[2]); ++j) {
            double *w = vec(j + 1);
            if ((st = matvec(vec(j), w)) != VM_OK) return st;
            ++total;
            // classical Gram-Schmidt, twice
            std::vector<double> h(3 * size_t(j + 1), 0.0);
            for (int pass = 0; pass < 2; ++pass) {
                if ((st = multidot(w, V, j + 1)) != VM_OK) return st;
                clear();
                for (int c = 0; c < 3; ++c) cf.alpha[c] = 1.0;
                for (int i = 0; i <= j; ++i)
                    for (int c = 0; c < 3; ++c)
                        if (active[c]) {
                            h[3 * i + c] += dots[3 * i + c];
                            cf.c[3 * i + c] = -dots[3 * i + c];
                        }
                if ((st = axpy(w, V, j + 1, cf)) != VM_OK) return st;
            }
            if ((st = multidot(w, w, 1)) != VM_OK) return st;
            clear();
            for (int c = 0; c < 3; ++c) {
                if (!active[c]) continue;
                const double nrm = std::sqrt(dots[c]);
                double *col = &H[c][size_t(j) * ld];
                for (int i = 0; i <= j; ++i) col[i] = h[3 * i + c];
                col[j + 1] = nrm;
                for (int i = 0; i < j; ++i) {
                    const double t = cs[c][i] * col[i] + sn[c][i] * col[i + 1];
                    col[i + 1] = -sn[c][i] * col[i] + cs[c][i] * col[i + 1];
                    col[i] = t;
                }
                const double r = std::hypot(col[j], col[j + 1]);
                cs[c][j] = r > 0.0 ? col[j] / r : 1.0;
                sn[c][j] = r > 0.0 ? col[j + 1] / r : 0.0;
                col[j] = r;
                col[j + 1] = 0.0;
                gv[c][j + 1] = -sn[c][j] * gv[c][j];
                gv[c][j] = cs[c][j] * gv[c][j];
                cols[c] = j + 1;
                rel[c] = std::fabs(gv[c][j + 1]) / beta0[c];
                if (rel[c] <= tol) done[c] = true;
                if (done[c] || !(nrm > 0.0)) active[c] = false;
                cf.alpha[c] = active[c] ? 1.0 / nrm : 0.0;
            }
            if ((st = axpy(w, V, 0, cf)) != VM_OK) return st;
        }
        // gamma += V y for each component
        clear();
        int kmax = 0;
        for (int c = 0; c < 3; ++c) {
            cf.alpha[c] = 1.0;
            if (cols[c] == 0) continue;
            double y[VM_RBF_RESTART];
            back_substitute(H[c], ld, gv[c], cols[c], y);
            for (int i = 0; i < cols[c]; ++i) cf.c[3 * i + c] = y[i];
            kmax = std::max(kmax, cols[c]);
        }
        if ((st = axpy(xs, V, kmax, cf)) != VM_OK) return st;
        if ((done[0] && done[1] && done[2]) || total >= max_iter) break;
    }
    {
        Timed tm(ctx, VM_PH_KRYLOV);
        VM_HIP(launch_scatter3(s, ni, perm, xs, 1.0, gamma), "scatter");
    }
    if (iters) *iters = total;
    if (resid) *resid = std::max(rel[0], std::max(rel[1], rel[2]));
    return VM_OK;
}

vm_status vm_energy_spectrum(vm_ctx *ctx, int ng, const double *u, int kmax, double *E) {
    if (!ctx) return VM_EINVAL;
    if (ng < 2 || ng > 1290) return fail(ctx, VM_EINVAL, "ng out of range [2, 1290]");
    if (kmax < 0 || kmax > VM_SPECTRUM_MAX_K) return fail(ctx, VM_EINVAL, "kmax out of range");
    if (!u || !E) return fail(ctx, VM_EINVAL, "u and E must be non-NULL");
    if (misaligned(u) || misaligned(E)) return fail(ctx, VM_EINVAL, "arrays must be 8-byte aligned");
    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    hipStream_t s = ctx->stream;
    const int nzc = ng / 2 + 1;
    const size_t n3 = size_t(ng) * ng * ng, total = size_t(ng) * ng * nzc;
    if (ctx->fft_ng != ng) {
        if (ctx->fft_ng > 0) (void)hipfftDestroy(ctx->fft_plan);
        ctx->fft_ng = -1;
        if (hipfftPlan3d(&ctx->fft_plan, ng, ng, ng, HIPFFT_D2Z) != HIPFFT_SUCCESS)
            return fail(ctx, VM_EDEVICE, "hipfftPlan3d failed");
        ctx->fft_ng = ng;
    }
    if (hipfftSetStream(ctx->fft_plan, s) != HIPFFT_SUCCESS) return fail(ctx, VM_EDEVICE, "hipfftSetStream failed");
    if (ctx->spec_ng != ng || ctx->spec_kmax != kmax) {
        // entries of the half spectrum by shell rint(|m|), m the signed integer wavevector
        std::vector<int32_t> shell(total), start(size_t(kmax) + 2, 0), list;
        auto sgn = [ng](int i) { return i <= ng / 2 ? i : i - ng; };
        for (int ix = 0; ix < ng; ++ix)
            for (int iy = 0; iy < ng; ++iy)
                for (int kz = 0; kz < nzc; ++kz) {
                    const double mx = sgn(ix), my = sgn(iy), mz = kz;
                    const double r = std::nearbyint(std::sqrt(mx * mx + my * my + mz * mz));
                    const size_t e = (size_t(ix) * ng + iy) * nzc + kz;
                    shell[e] = r <= kmax ? int32_t(r) : -1;
                    if (shell[e] >= 0) ++start[size_t(shell[e]) + 1];
                }
        for (int k = 0; k <= kmax; ++k) start[size_t(k) + 1] += start[size_t(k)];
        list.resize(size_t(start[size_t(kmax) + 1]));
        std::vector<int32_t> fill(start.begin(), start.end() - 1);
        for (size_t e = 0; e < total; ++e)
            if (shell[e] >= 0) list[size_t(fill[size_t(shell[e])]++)] = int32_t(e);
        ctx->spec_ng = -1;
        VM_HIP(upload(ctx->spec_start, start), "upload shells");
        if (list.empty()) list.push_back(0);
        VM_HIP(upload(ctx->spec_list, list), "upload shells");
        ctx->spec_ng = ng;
        ctx->spec_kmax = kmax;
    }
    VM_HIP(ctx->spec_in.reserve(sizeof(double) * n3), "alloc spectrum");
    VM_HIP(ctx->spec_U.reserve(2 * sizeof(double) * total), "alloc spectrum");
    VM_HIP(ctx->spec_power.reserve(sizeof(double) * total), "alloc spectrum");
    const double inv = 1.0 / double(n3);
    for (int c = 0; c < 3; ++c) {
        // the transform may use its input as scratch: it works on a copy
        VM_HIP(hipMemcpyAsync(ctx->spec_in.ptr, u + size_t(c) * n3, sizeof(double) * n3, hipMemcpyDeviceToDevice, s),
               "copy component");
        if (hipfftExecD2Z(ctx->fft_plan, ctx->spec_in.as<hipfftDoubleReal>(), ctx->spec_U.as<hipfftDoubleComplex>()) !=
            HIPFFT_SUCCESS)
            return fail(ctx, VM_EDEVICE, "hipfftExecD2Z failed");
        VM_HIP(launch_spec_power(s, ng, ctx->spec_U.ptr, 0.5 * inv * inv, c == 0, ctx->spec_power.as<double>()),
               "spectrum power");
    }
    VM_HIP(launch_shell_sum(s, kmax + 1, ctx->spec_start.as<int32_t>(), ctx->spec_list.as<int32_t>(),
                            ctx->spec_power.as<double>(), E),
           "shell sums");
    return VM_OK;
}

vm_status vm_tune_level(vm_ctx *ctx, int64_t n, const double *x, const double *alpha, double sigma, int p,
                        const vm_opts *opts, double min_leaf_sigmas, int reps, int *level, double *ms) {
    if (!ctx) return VM_EINVAL;
    if (!level) return fail(ctx, VM_EINVAL, "level must be non-NULL");
    if (vm_status st = check_common(ctx, n, sigma, 0, opts); st != VM_OK) return st;
    if (!(min_leaf_sigmas > 0.0) || !std::isfinite(min_leaf_sigmas))
        return fail(ctx, VM_EINVAL, "min_leaf_sigmas must be positive");
    if (reps < 1 || reps > 100) return fail(ctx, VM_EINVAL, "reps out of range [1, 100]");
    if (ms)
        for (int l = 0; l <= VM_MAX_LEVEL; ++l) ms[l] = -1.0;
    // the finest level whose leaves are at least min_leaf_sigmas sigma wide and
    // not more numerous than the particles
    int lmax = 0;
    while (lmax < VM_MAX_LEVEL && std::ldexp(opts->box_len, -(lmax + 1)) >= min_leaf_sigmas * sigma &&
           (int64_t(1) << (3 * (lmax + 1))) <= n)
        ++lmax;
    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    const size_t bytes = sizeof(double) * 3 * size_t(n);
    VM_HIP(ctx->rk_u.reserve(bytes), "alloc tuning");
    VM_HIP(ctx->rk_s.reserve(bytes), "alloc tuning");
    hipEvent_t e0, e1;
    VM_HIP(hipEventCreate(&e0), "event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, VM_EDEVICE, "event");
    }
    // from the finest admissible level towards coarser ones while the time falls
    // (each coarser level has 8x the near-field pairs per leaf)
    double best = -1.0, prev = -1.0;
    int arg = lmax;
    vm_status st = VM_OK;
    for (int l = lmax; l >= 0; --l) {
        // one untimed call grows the workspace and builds the caches for this level
        st = vm_fmm_eval(ctx, n, x, alpha, sigma, p, l, opts, ctx->rk_u.as<double>(), ctx->rk_s.as<double>(), nullptr);
        if (st != VM_OK) break;
        if (hipEventRecord(e0, ctx->stream) != hipSuccess) { st = fail(ctx, VM_EDEVICE, "event"); break; }
        for (int r = 0; r < reps && st == VM_OK; ++r)
            st = vm_fmm_eval(ctx, n, x, alpha, sigma, p, l, opts, ctx->rk_u.as<double>(), ctx->rk_s.as<double>(),
                             nullptr);
        if (st != VM_OK) break;
        float t = 0.0f;
        if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t, e0, e1) != hipSuccess) {
            st = fail(ctx, VM_EDEVICE, "event timing");
            break;
        }
        const double avg = double(t) / reps;
        if (ms) ms[l] = avg;
        if (best < 0.0 || avg < best) {
            best = avg;
            arg = l;
        }
        if (prev >= 0.0 && avg > prev) break;
        prev = avg;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != VM_OK) return st;
    *level = arg;
    return VM_OK;
}

vm_status vm_tune_ncrit(vm_ctx *ctx, int64_t n, const double *x, const double *alpha, double sigma, int p,
                        int max_level, const vm_opts *opts, int reps, int *ncrit, double *ms) {
    if (!ctx) return VM_EINVAL;
    if (!ncrit) return fail(ctx, VM_EINVAL, "ncrit must be non-NULL");
    if (vm_status st = check_common(ctx, n, sigma, max_level, opts); st != VM_OK) return st;
    if (reps < 1 || reps > 100) return fail(ctx, VM_EINVAL, "reps out of range [1, 100]");
    if (ms)
        for (int i = 0; i < VM_NCRIT_CANDIDATES; ++i) ms[i] = -1.0;
    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    const size_t bytes = sizeof(double) * 3 * size_t(n);
    VM_HIP(ctx->rk_u.reserve(bytes), "alloc tuning");
    VM_HIP(ctx->rk_s.reserve(bytes), "alloc tuning");
    hipEvent_t e0, e1;
    VM_HIP(hipEventCreate(&e0), "event");
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, VM_EDEVICE, "event");
    }
    // leaf sizes 8, 16, ..., 1024 in increasing order while the time falls: a
    // larger bound trades expansion work (fewer, coarser cells) for near-field
    // pairs, so the time has one valley
    double best = -1.0, prev = -1.0;
    int arg = 8, rises = 0;
    vm_status st = VM_OK;
    for (int i = 0; i < VM_NCRIT_CANDIDATES; ++i) {
        const int nc = 8 << i;
        auto run = [&]() {
            return vm_fmm_eval_adaptive(ctx, n, x, alpha, sigma, p, nc, max_level, opts, ctx->rk_u.as<double>(),
                                        ctx->rk_s.as<double>(), nullptr);
        };
        st = run();   // untimed: workspace
        if (st != VM_OK) break;
        if (hipEventRecord(e0, ctx->stream) != hipSuccess) { st = fail(ctx, VM_EDEVICE, "event"); break; }
        for (int r = 0; r < reps && st == VM_OK; ++r) st = run();
        if (st != VM_OK) break;
        float tms = 0.0f;
        if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&tms, e0, e1) != hipSuccess) {
            st = fail(ctx, VM_EDEVICE, "event timing");
            break;
        }
        const double avg = double(tms) / reps;
        if (ms) ms[i] = avg;
        if (best < 0.0 || avg < best) {
            best = avg;
            arg = nc;
        }
        rises = (prev >= 0.0 && avg > prev) ? rises + 1 : 0;
        if (rises == 2) break;
        prev = avg;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != VM_OK) return st;
    *ncrit = arg;
    return VM_OK;
}

vm_status vm_debug_adaptive(vm_ctx *ctx, int what, int32_t *out, int64_t *rows) {
    if (!ctx || !rows) return VM_EINVAL;
    auto &A = ctx->ad;
    if (!A.valid) return fail(ctx, VM_EINVAL, "no adaptive evaluation yet");
    if (what < 0 || what > 5) return fail(ctx, VM_EINVAL, "what out of range [0, 5]");
    hipStream_t s = ctx->stream;
    const int nc = A.ncell;
    auto fetch = [&](const DevBuf &b, size_t count, auto *host) -> vm_status {
        VM_HIP(hipMemcpyAsync(host, b.ptr, count * sizeof(*host), hipMemcpyDeviceToHost, s), "copy debug view");
        return VM_OK;
    };
    if (what == 5) {
        *rows = A.n;
        if (!out) return VM_OK;
        VM_HIP(hipMemcpyAsync(out, ctx->last_perm, sizeof(int32_t) * size_t(A.n), hipMemcpyDeviceToHost, s),
               "copy debug view");
        VM_HIP(hipStreamSynchronize(s), "synchronize");
        return VM_OK;
    }
    std::vector<uint32_t> key(nc);
    std::vector<int32_t> lev(nc), st(nc), cnt(nc), par(nc);
    vm_status r = VM_OK;
    if ((r = fetch(A.key, nc, key.data())) != VM_OK || (r = fetch(A.level, nc, lev.data())) != VM_OK ||
        (r = fetch(A.start, nc, st.data())) != VM_OK || (r = fetch(A.count, nc, cnt.data())) != VM_OK ||
        (r = fetch(A.parent, nc, par.data())) != VM_OK)
        return r;
    std::vector<int32_t> rowsv;
    if (what == 0) {
        VM_HIP(hipStreamSynchronize(s), "synchronize");
        for (int c = 0; c < nc; ++c) {
            const int leaf = cnt[c] <= A.ncrit || lev[c] >= A.max_level;
            const int32_t row[6] = {int32_t(key[c]), lev[c], st[c], cnt[c], par[c], leaf};
            rowsv.insert(rowsv.end(), row, row + 6);
        }
    } else if (what == 2) {
        std::vector<int32_t> vt(size_t(nc) * 189);
        if ((r = fetch(A.vtab, vt.size(), vt.data())) != VM_OK) return r;
        VM_HIP(hipStreamSynchronize(s), "synchronize");
        const OffsetTable &t = offset_table();
        const std::vector<int16_t> lists = device_octant_lists();
        for (int c = 0; c < nc; ++c)
            for (int i = 0; i < 189; ++i) {
                const int b = vt[size_t(c) * 189 + i];
                if (b < 0) continue;
                const int l = lev[c], o = int(key[c] & 7u), side = 1 << l;
                const int8_t *d = t.d[lists[o * 189 + i]];
                int code = 0, mul = 1;
                for (int k = 0; k < 3; ++k) {
                    int cc = 0;
                    for (int bit = 0; bit < l; ++bit) cc |= int((key[c] >> (3 * bit + k)) & 1u) << bit;
                    const int pos = cc + d[k];
                    const int sh = pos < 0 ? -1 : (pos >= side ? 1 : 0);
                    code += (sh + 1) * mul;
                    mul *= 3;
                }
                const int32_t row[3] = {c, b, code};
                rowsv.insert(rowsv.end(), row, row + 3);
            }
    } else {
        const int k = what == 1 ? 0 : (what == 3 ? 1 : 2);   // P2P, M2P, P2L
        std::vector<uint32_t> lc(3 * size_t(nc)), lo(3 * size_t(nc));
        if ((r = fetch(A.cnt, lc.size(), lc.data())) != VM_OK || (r = fetch(A.off, lo.size(), lo.data())) != VM_OK)
            return r;
        VM_HIP(hipStreamSynchronize(s), "synchronize");
        const size_t total = size_t(lo.back()) + lc.back();
        std::vector<int32_t> src(total);
        std::vector<int8_t> code(total);
        if (total) {
            if ((r = fetch(A.src, total, src.data())) != VM_OK || (r = fetch(A.code, total, code.data())) != VM_OK)
                return r;
            VM_HIP(hipStreamSynchronize(s), "synchronize");
        }
        for (int c = 0; c < nc; ++c)
            for (uint32_t e = 0; e < lc[size_t(k) * nc + c]; ++e) {
                const size_t pos = size_t(lo[size_t(k) * nc + c]) + e;
                const int32_t row[3] = {c, src[pos], code[pos]};
                rowsv.insert(rowsv.end(), row, row + 3);
            }
    }
    const int width = what == 0 ? 6 : 3;
    *rows = int64_t(rowsv.size() / width);
    if (out) std::memcpy(out, rowsv.data(), rowsv.size() * sizeof(int32_t));
    return VM_OK;
}

vm_status vm_set_timing(vm_ctx *ctx, int enable) {
    if (!ctx) return VM_EINVAL;
    ctx->timing = enable != 0;
    ctx->timed.clear();
    return VM_OK;
}

vm_status vm_get_timing(vm_ctx *ctx, double *ms, int *launches) {
    if (!ctx || !ms || !launches) return VM_EINVAL;
    for (int i = 0; i < VM_NPHASE; ++i) {
        ms[i] = 0.0;
        launches[i] = 0;
    }
    VM_HIP(hipStreamSynchronize(ctx->stream), "synchronize");
    for (const auto &t : ctx->timed) {
        float e = 0.0f;
        VM_HIP(hipEventElapsedTime(&e, ctx->events[t.second], ctx->events[t.second + 1]), "event time");
        ms[t.first] += double(e);
        launches[t.first] += 1;
    }
    return VM_OK;
}

vm_status vm_debug_tree(vm_ctx *ctx, uint32_t *keys, int32_t *perm, int32_t *leaf_start) {
    if (!ctx) return VM_EINVAL;
    if (ctx->last_level < 0) return fail(ctx, VM_EINVAL, "no evaluation yet");
    hipStream_t s = ctx->stream;
    const size_t n = size_t(ctx->last_n);
    const size_t nleaf = size_t(1) << (3 * ctx->last_level);
    if (keys) VM_HIP(hipMemcpyAsync(keys, ctx->last_keys, n * 4, hipMemcpyDeviceToDevice, s), "copy keys");
    if (perm) VM_HIP(hipMemcpyAsync(perm, ctx->last_perm, n * 4, hipMemcpyDeviceToDevice, s), "copy perm");
    if (leaf_start)
        VM_HIP(hipMemcpyAsync(leaf_start, ctx->start.ptr, (nleaf + 1) * 4, hipMemcpyDeviceToDevice, s), "copy ranges");
    return VM_OK;
}

vm_status vm_debug_expansions(vm_ctx *ctx, int which, int level, void *out, int64_t *bytes) {
    if (!ctx || !bytes || (which != 0 && which != 1)) return VM_EINVAL;
    if (ctx->last_p < 1) return fail(ctx, VM_EINVAL, "no expansions in the last call");
    if (ctx->last_level < 0 || level < 0 || level > ctx->last_level)
        return fail(ctx, VM_EINVAL, "level not in the last evaluation");
    const int kp = coef_stride(ncoef(ctx->last_p));
    const size_t esz = ctx->last_mixed ? 4 : 8;
    const size_t row = size_t(3) * kp * esz;
    const size_t before = size_t(((int64_t(1) << (3 * level)) - 1) / 7);
    const size_t cnt = size_t(1) << (3 * level);
    *bytes = int64_t(cnt * row);
    if (!out) return VM_OK;
    const DevBuf &b = which == 0 ? ctx->mbuf : ctx->lbuf;
    VM_HIP(hipMemcpyAsync(out, static_cast<const char *>(b.ptr) + before * row, cnt * row,
                          hipMemcpyDeviceToDevice, ctx->stream), "copy expansions");
    return VM_OK;
}

vm_status vm_debug_far(vm_ctx *ctx, double *out) {
    if (!ctx || !out) return VM_EINVAL;
    const auto &ll = ctx->last_l2p;
    if (ctx->last_level < 0 || !ctx->last_far || !ll.valid)
        return fail(ctx, VM_EINVAL, "no far field in the last evaluation");
    VM_HIP(hipSetDevice(ctx->device), "hipSetDevice");
    if (ll.mixed)
        VM_HIP(launch_l2p<float>(ctx->stream, ll.nleaf, ll.n, ll.tparts, ll.tstart, ll.p, ll.kp, ll.inv_w, ll.w,
                                 ll.tab, static_cast<const float *>(ll.lptr), out),
               "far field");
    else
        VM_HIP(launch_l2p<double>(ctx->stream, ll.nleaf, ll.n, ll.tparts, ll.tstart, ll.p, ll.kp, ll.inv_w, ll.w,
                                  ll.tab, static_cast<const double *>(ll.lptr), out),
               "far field");
    return VM_OK;
}

vm_status vm_debug_offsets(int8_t *out, int *count) {
    if (!out || !count) return VM_EINVAL;
    const OffsetTable &t = offset_table();
    std::memcpy(out, t.d, sizeof(t.d));
    *count = 316;
    return VM_OK;
}

vm_status vm_debug_list(int level, int periodic, int32_t key, int32_t *src, int8_t *d, int8_t *img, int *count) {
    if (!src || !d || !img || !count) return VM_EINVAL;
    if (level < 1 || level > VM_MAX_LEVEL || (!periodic && level < 2)) return VM_EINVAL;
    if (key < 0 || int64_t(key) >= (int64_t(1) << (3 * level))) return VM_EINVAL;
    const OffsetTable &t = offset_table();
    const int side = 1 << level;
    int c[3] = {0, 0, 0};
    for (int b = 0; b < level; ++b)
        for (int k = 0; k < 3; ++k) c[k] |= ((key >> (3 * b + k)) & 1) << b;
    const int oct = (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2);
    int cnt = 0;
    for (int i = 0; i < 189; ++i) {
        const int8_t *o = t.d[t.list[oct][i]];
        int sc[3], im[3];
        bool ok = true;
        for (int k = 0; k < 3; ++k) {
            const int v = c[k] + o[k];
            if (periodic) {
                im[k] = v < 0 ? -1 : (v >= side ? 1 : 0);
                sc[k] = v - im[k] * side;
            } else {
                im[k] = 0;
                sc[k] = v;
                if (v < 0 || v >= side) ok = false;
            }
        }
        if (!ok) continue;
        int sk = 0;
        for (int b = 0; b < level; ++b)
            for (int k = 0; k < 3; ++k) sk |= ((sc[k] >> b) & 1) << (3 * b + k);
        src[cnt] = sk;
        for (int k = 0; k < 3; ++k) {
            d[3 * cnt + k] = o[k];
            img[3 * cnt + k] = int8_t(im[k]);
        }
        ++cnt;
    }
    *count = cnt;
    return VM_OK;
}

vm_status vm_debug_operator(int kind, int p, int index, double *out) {
    if (!out || p < 1 || p > VM_MAX_P) return VM_EINVAL;
    const OffsetTable &t = offset_table();
    if (kind == 0) {
        if (index < 0 || index >= 316) return VM_EINVAL;
        const double D[3] = {-double(t.d[index][0]), -double(t.d[index][1]), -double(t.d[index][2])};
        m2l_matrix(p, D, 1.0, 1.0, out);
        return VM_OK;
    }
    if (kind == 1 || kind == 2) {
        if (index < 0 || index >= 8) return VM_EINVAL;
        const double d[3] = {((index & 1) - 0.5) * 0.5, (((index >> 1) & 1) - 0.5) * 0.5,
                             (((index >> 2) & 1) - 0.5) * 0.5};
        if (kind == 1) m2m_matrix(p, d, 0.5, 1.0, out);
        else l2l_matrix(p, d, 1.0, 0.5, out);
        return VM_OK;
    }
    if (kind == 3) {
        if (index < 1 || index > 4) return VM_EINVAL;
        lattice_matrix(p, index, out);
        return VM_OK;
    }
    if (kind == 4) {
        // gradient of F(Y) = sum_t f_t c_t(Y): out[a][s][t], a < 3, s < p^2, t < C
        const AdjTables a = adj_tables(p);
        const int C = ncoef(p), rows = 3 * p * p;
        std::fill(out, out + size_t(rows) * C, 0.0);
        for (int r = 0; r < rows; ++r)
            for (int e = 0; e < a.width_g; ++e) out[size_t(r) * C + a.g_idx[size_t(r) * a.width_g + e]] += a.g_w[size_t(r) * a.width_g + e];
        return VM_OK;
    }
    return VM_EINVAL;
}

}  // extern "C"
