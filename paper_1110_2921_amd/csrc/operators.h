// Host-side generation of the FMM operators in the library's real basis.
//
// Basis (see include/vmfmm.h): balanced regular solid harmonics
//   Rb_n^m(x) = sqrt((n+m)!(n-m)!) r^n P_n^m(cos t) e^{i m phi} / (n+m)!
// and irregular ones Ib_n^m = (n-m)! P_n^m e^{i m phi} / (r^{n+1} sqrt((n+m)!(n-m)!)),
// so that 1/|x - y| = sum_{n,m} conj(Rb_n^m(y)) Ib_n^m(x) for |y| < |x|
// (the two-sided expansion behind the paper's eqs. 10-11), |Rb| <= r^n and
// |Ib| <= r^{-n-1}.  Every operator is generated in FP64.
#pragma once

#include <cstdint>
#include <vector>

namespace vmfmm {

inline int ncoef(int p) { return (p + 1) * (p + 1); }

// The 316 M2L offsets d = source - target (cells), sorted by (dz, dy, dx), and
// for each octant (bit 0 = x parity ...) the 189 indices of its list in the
// same order.
struct OffsetTable {
    int8_t d[316][3];
    int16_t list[8][189];
};
const OffsetTable &offset_table();

// Real C x C operators, row-major (row = output coefficient).
//   m2l: local of a target cell of width wt from the multipole of a source cell
//        of width ws, D = target centre - source centre (physical units).
//   m2m: parent (width wp) multipole from a child (width wc), d = child - parent centre.
//   l2l: child (width wc) local from the parent (width wp), d = child - parent centre.
void m2l_matrix(int p, const double D[3], double wt, double ws, double *out);
void m2m_matrix(int p, const double d[3], double wc, double wp, double *out);
void l2l_matrix(int p, const double d[3], double wp, double wc, double *out);

// Periodic lattice operator in root units: local at the root centre of the
// images of the block 3^K per side that lie outside the 3x3x3 block, as a
// function of the root multipole.  Zero for K <= 1.
void lattice_matrix(int p, int K, double *out);

// Far-field evaluation tables for one leaf.  From the leaf's local
// coefficients (3 components x C, component-major) they give
//   velocity expansions U_b (b = x,y,z), degree p-1: nu = p^2 coefficients,
//   gradient expansions G_ab (a,b = x,y,z, index 3a+b), degree p-2: ng = (p-1)^2,
// already multiplied by the evaluation weights (1 for m = 0, 2 for m > 0), so
// that with c(X) = [Rb^0, Re Rb^m, -Im Rb^m] (X = (x - c)/w):
//   u_b    = 1/(4 pi w^2) sum_s U_b[s] c_s(X)
//   J[a][b] = 1/(4 pi w^3) sum_s G_ab[s] c_s(X).
// Each output row is a short sparse combination of the 3C inputs: rows are
// padded to `width` entries of (input index, weight).
struct L2PTable {
    int p = 0, nu = 0, ng = 0, width = 0;
    std::vector<int32_t> idx;     // (3 nu + 9 ng) x width
    std::vector<double> w;        // same shape
};
L2PTable l2p_table(int p);

// Sparse tables of the adjoint (transposed) far field, from the same FP64
// derivative operators:
//   L2P^T: lam_bar[j] = 1/(4 pi w^2) sum_e w * V[idx]  for each of the 3C local
//          coefficients j, V[b*nu + s] = sum_i ubar_{i,b} c_s(X_i) (degree < p);
//   P2M gradient: for F(Y) = sum_t f_t c_t(Y) (degree p),
//          dF/dY_a = sum_s G[a*nu + s] c_s(Y),  G[a*nu + s] = sum_e w * f[idx].
struct AdjTables {
    int p = 0, nu = 0, width_t = 0, width_g = 0;
    std::vector<int32_t> t_idx;   // (3C) x width_t, indices into [0, 3 nu)
    std::vector<double> t_w;
    std::vector<int32_t> g_idx;   // (3 nu) x width_g, indices into [0, C)
    std::vector<double> g_w;
};
AdjTables adj_tables(int p);

// Cell-particle evaluation (M2P): the first and second derivatives at a point
// x of the multipole potential of a cell of width w, through the local
// expansion about x of degree <= 2 that the M2L theorem gives (target width
// w), from the balanced irregular harmonics H of X = (x - centre) / w, degree
// <= p + 2, packed [Ib_n^0, Re Ib_n^m, Im Ib_n^m]:
//   loc[k][r] = sum over the entries e of row r: w[e] Mb[k][col[e]] H[harm[e]],
// rows r < nrow = (min(2, p) + 1)^2 the packed local coefficients, then
//   out[o] = sum_q G[o][q] loc[q],  q = nrow k + r,
// u_b = out[b] / (4 pi w^2), J[a][b] = out[3 + 3a + b] / (4 pi w^3).
struct M2PTable {
    int p = 0, nrow = 0, nharm = 0;
    std::vector<int32_t> rowptr, col, harm;   // rowptr: nrow + 1 entry offsets
    std::vector<double> w;
    std::vector<double> G;                    // 12 x (3 nrow)
};
M2PTable m2p_table(int p);

// Recurrence constants for the balanced regular harmonics, index n(n+1)/2 + m:
//   Rb_m^m   = -(X + iY) diag[m] Rb_{m-1}^{m-1},  diag[m] = sqrt((2m-1)/(2m))
//   Rb_n^m   = c1 Z Rb_{n-1}^m - c2 r^2 Rb_{n-2}^m  (n > m)
//   c1 = (2n-1)/sqrt((n+m)(n-m)),  c2 = sqrt((n+m-1)(n-m-1)/((n+m)(n-m)))
struct RecTable {
    std::vector<double> c1, c2, diag;
};
RecTable rec_table(int p);

}  // namespace vmfmm
