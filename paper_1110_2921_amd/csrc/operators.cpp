// Host-side FP64 generation of the translation operators (M2M, M2L, L2L),
// the periodic lattice operator and the far-field evaluation tables.
//
// Derivation (unnormalised harmonics R_n^m = r^n P_n^m e^{im phi}/(n+m)!,
// I_n^m = (n-m)! P_n^m e^{im phi}/r^{n+1}, P with the Condon-Shortley phase):
//   1/|x - y|      = sum conj(R_n^m(y)) I_n^m(x)                    (|y| < |x|)
//   R_n^m(a + b)   = sum_{k,l} R_k^l(a) R_{n-k}^{m-l}(b)            (regular addition)
//   I_n^m(D + x')  = sum_{k,l} (-1)^{k+l} R_k^l(x') I_{n+k}^{m-l}(D) (|x'| < |D|)
//   dz R_n^m = R_{n-1}^m, (dx + i dy) R_n^m = R_{n-1}^{m+1}, (dx - i dy) R_n^m = -R_{n-1}^{m-1}
// These give, for multipoles M = sum q conj(R(y)) and locals phi = sum L R(x):
//   M2M  M'_n^m = sum conj(R_k^l(d)) M_{n-k}^{m-l},  d = child - parent centre
//   M2L  L_k^l  = sum (-1)^{k+l} I_{n+k}^{m-l}(D) M_n^m,  D = target - source centre
//   L2L  L'_k^l = sum R_{n-k}^{m-l}(d) L_n^m,  d = child - parent centre
// The library stores balanced, cell-scaled coefficients
//   Mb_n^m = M_n^m N_n^m / w^n,   Lb_n^m = L_n^m w^{n+1} / N_n^m,  N_n^m = sqrt((n+m)!(n-m)!),
// and packs the m >= 0 half of each symmetric set (F^{-m} = (-1)^m conj F^m)
// into (p+1)^2 reals.
#include "operators.h"

#include <cmath>
#include <complex>
#include <functional>
#include <mutex>
#include <stdexcept>

namespace vmfmm {

using cplx = std::complex<double>;

namespace {

double lfact(int n) { return std::lgamma(n + 1.0); }

double norm_nm(int n, int m) {
    m = std::abs(m);
    return std::exp(0.5 * (lfact(n + m) + lfact(n - m)));
}

// Unnormalised harmonics at a point, all m >= 0 up to degree `deg`;
// negative m through F^{-m} = (-1)^m conj(F^m).
struct Harm {
    int deg;
    std::vector<cplx> v;   // index n(n+1)/2 + m
    cplx operator()(int n, int m) const {
        if (n < 0 || std::abs(m) > n) return cplx(0.0, 0.0);
        if (m >= 0) return v[n * (n + 1) / 2 + m];
        cplx c = std::conj(v[n * (n + 1) / 2 - m]);
        return (m & 1) ? -c : c;
    }
};

Harm regular(const double x[3], int deg) {
    Harm h{deg, std::vector<cplx>((deg + 1) * (deg + 2) / 2)};
    const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    const cplx w(x[0], x[1]);
    cplx diag(1.0, 0.0);
    for (int m = 0; m <= deg; ++m) {
        if (m > 0) diag = -w / (2.0 * m) * diag;
        h.v[m * (m + 1) / 2 + m] = diag;
        cplx pm2(0.0, 0.0), pm1 = diag;
        for (int n = m + 1; n <= deg; ++n) {
            cplx cur = ((2.0 * n - 1.0) * x[2] * pm1 - r2 * pm2) / double((n + m) * (n - m));
            h.v[n * (n + 1) / 2 + m] = cur;
            pm2 = pm1;
            pm1 = cur;
        }
    }
    return h;
}

Harm irregular(const double x[3], int deg) {
    Harm h{deg, std::vector<cplx>((deg + 1) * (deg + 2) / 2)};
    const double r2 = x[0] * x[0] + x[1] * x[1] + x[2] * x[2];
    const cplx w(x[0], x[1]);
    cplx diag(1.0 / std::sqrt(r2), 0.0);
    for (int m = 0; m <= deg; ++m) {
        if (m > 0) diag = -(2.0 * m - 1.0) * w / r2 * diag;
        h.v[m * (m + 1) / 2 + m] = diag;
        cplx pm2(0.0, 0.0), pm1 = diag;
        for (int n = m + 1; n <= deg; ++n) {
            cplx cur = ((2.0 * n - 1.0) * x[2] * pm1 - double((n + m - 1) * (n - m - 1)) * pm2) / r2;
            h.v[n * (n + 1) / 2 + m] = cur;
            pm2 = pm1;
            pm1 = cur;
        }
    }
    return h;
}

// coef(tn, tm, sn, sm): complex factor of source coefficient (sn, sm) in target
// coefficient (tn, tm >= 0).  Builds the real matrix acting on packed vectors.
using CoefFn = std::function<cplx(int, int, int, int)>;

void real_matrix(int pt, int ps, const CoefFn &coef, double *out) {
    const int ct = ncoef(pt), cs = ncoef(ps);
    for (int i = 0; i < ct * cs; ++i) out[i] = 0.0;
    for (int tn = 0; tn <= pt; ++tn) {
        for (int tm = 0; tm <= tn; ++tm) {
            const int row_re = tm == 0 ? tn * tn : tn * tn + 2 * tm - 1;
            const int row_im = tn * tn + 2 * tm;
            for (int sn = 0; sn <= ps; ++sn) {
                for (int sm = 0; sm <= sn; ++sm) {
                    const double sgn = (sm & 1) ? -1.0 : 1.0;
                    if (sm == 0) {
                        cplx g = coef(tn, tm, sn, 0);
                        out[row_re * cs + sn * sn] = g.real();
                        if (tm > 0) out[row_im * cs + sn * sn] = g.imag();
                        continue;
                    }
                    const cplx a = coef(tn, tm, sn, sm), b = coef(tn, tm, sn, -sm);
                    // unit real part: F^m = 1, F^-m = (-1)^m
                    const cplx gre = a + b * sgn;
                    // unit imaginary part: F^m = i, F^-m = -i (-1)^m
                    const cplx gim = a * cplx(0.0, 1.0) + b * cplx(0.0, -sgn);
                    const int cre = sn * sn + 2 * sm - 1, cim = sn * sn + 2 * sm;
                    out[row_re * cs + cre] = gre.real();
                    out[row_re * cs + cim] = gim.real();
                    if (tm > 0) {
                        out[row_im * cs + cre] = gre.imag();
                        out[row_im * cs + cim] = gim.imag();
                    }
                }
            }
        }
    }
}

void matmul(int n, const double *a, const double *b, double *c) {
    std::vector<double> t(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < n; ++k) {
            const double aik = a[size_t(i) * n + k];
            if (aik == 0.0) continue;
            for (int j = 0; j < n; ++j) t[size_t(i) * n + j] += aik * b[size_t(k) * n + j];
        }
    std::copy(t.begin(), t.end(), c);
}

}  // namespace

const OffsetTable &offset_table() {
    static OffsetTable tab;
    static std::once_flag once;
    std::call_once(once, [] {
        // all offsets reachable from some octant, sorted by (dz, dy, dx)
        int count = 0;
        int index_of[7][7][7];
        for (int dz = -3; dz <= 3; ++dz)
            for (int dy = -3; dy <= 3; ++dy)
                for (int dx = -3; dx <= 3; ++dx) {
                    index_of[dz + 3][dy + 3][dx + 3] = -1;
                    if (std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) < 2) continue;
                    // d_i ranges over [-2 - par, 3 - par] for parity par: [-3, 3] overall,
                    // with -3 needing par = 1 and 3 needing par = 0
                    tab.d[count][0] = int8_t(dx);
                    tab.d[count][1] = int8_t(dy);
                    tab.d[count][2] = int8_t(dz);
                    index_of[dz + 3][dy + 3][dx + 3] = count++;
                }
        if (count != 316) throw std::logic_error("offset table size");
        for (int o = 0; o < 8; ++o) {
            const int px = o & 1, py = (o >> 1) & 1, pz = (o >> 2) & 1;
            int k = 0;
            for (int dz = -2 - pz; dz <= 3 - pz; ++dz)
                for (int dy = -2 - py; dy <= 3 - py; ++dy)
                    for (int dx = -2 - px; dx <= 3 - px; ++dx) {
                        if (std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) < 2) continue;
                        tab.list[o][k++] = int16_t(index_of[dz + 3][dy + 3][dx + 3]);
                    }
            if (k != 189) throw std::logic_error("octant list size");
        }
    });
    return tab;
}

void m2l_matrix(int p, const double D[3], double wt, double ws, double *out) {
    const Harm I = irregular(D, 2 * p);
    real_matrix(p, p, [&](int k, int l, int n, int m) -> cplx {
        const double sgn = ((k + l) & 1) ? -1.0 : 1.0;
        const double scale = std::pow(wt, k + 1) * std::pow(ws, n) / (norm_nm(k, l) * norm_nm(n, m));
        return sgn * scale * I(n + k, m - l);
    }, out);
}

void m2m_matrix(int p, const double d[3], double wc, double wp, double *out) {
    const Harm R = regular(d, p);
    real_matrix(p, p, [&](int n, int m, int n2, int m2) -> cplx {
        const int k = n - n2, l = m - m2;
        if (k < 0 || std::abs(l) > k) return cplx(0.0, 0.0);
        const double scale = norm_nm(n, m) / std::pow(wp, n) * std::pow(wc, n2) / norm_nm(n2, m2);
        return scale * std::conj(R(k, l));
    }, out);
}

void l2l_matrix(int p, const double d[3], double wp, double wc, double *out) {
    const Harm R = regular(d, p);
    real_matrix(p, p, [&](int k, int l, int n, int m) -> cplx {
        if (n < k || std::abs(m - l) > n - k) return cplx(0.0, 0.0);
        const double scale = std::pow(wc, k + 1) / norm_nm(k, l) * norm_nm(n, m) / std::pow(wp, n + 1);
        return scale * R(n - k, m - l);
    }, out);
}

void lattice_matrix(int p, int K, double *out) {
    const int C = ncoef(p);
    std::fill(out, out + size_t(C) * C, 0.0);
    if (K < 2) return;
    std::vector<double> msup(size_t(C) * C, 0.0), tmp(size_t(C) * C), acc(size_t(C) * C);
    for (int i = 0; i < C; ++i) msup[size_t(i) * C + i] = 1.0;
    for (int k = 2; k <= K; ++k) {
        if (k >= 3) {
            // supercell of width 3s from 27 copies of width s = 3^(k-3)
            const double s = std::pow(3.0, k - 3);
            std::fill(acc.begin(), acc.end(), 0.0);
            for (int ez = -1; ez <= 1; ++ez)
                for (int ey = -1; ey <= 1; ++ey)
                    for (int ex = -1; ex <= 1; ++ex) {
                        const double d[3] = {ex * s, ey * s, ez * s};
                        m2m_matrix(p, d, s, 3.0 * s, tmp.data());
                        for (size_t i = 0; i < acc.size(); ++i) acc[i] += tmp[i];
                    }
            matmul(C, acc.data(), msup.data(), msup.data());
        }
        // ring: 702 supercells of width s = 3^(k-2) at d s, d in [-4,4]^3 minus [-1,1]^3
        const double s = std::pow(3.0, k - 2);
        std::fill(acc.begin(), acc.end(), 0.0);
        for (int dz = -4; dz <= 4; ++dz)
            for (int dy = -4; dy <= 4; ++dy)
                for (int dx = -4; dx <= 4; ++dx) {
                    if (std::max(std::abs(dx), std::max(std::abs(dy), std::abs(dz))) <= 1) continue;
                    const double D[3] = {-dx * s, -dy * s, -dz * s};
                    m2l_matrix(p, D, 1.0, s, tmp.data());
                    for (size_t i = 0; i < acc.size(); ++i) acc[i] += tmp[i];
                }
        matmul(C, acc.data(), msup.data(), tmp.data());
        for (size_t i = 0; i < acc.size(); ++i) out[i] += tmp[i];
    }
}

namespace {

// Derivative d/dX_a of a balanced local expansion: degree pin -> pin - 1.
void deriv_matrix(int pin, int a, double *out) {
    real_matrix(pin - 1, pin, [&](int n2, int m2, int n, int m) -> cplx {
        if (n != n2 + 1) return cplx(0.0, 0.0);
        cplx f(0.0, 0.0);
        if (a == 2) {
            if (m == m2) f = 1.0;
        } else if (a == 0) {
            if (m == m2 - 1) f += 0.5;
            if (m == m2 + 1) f -= 0.5;
        } else {
            if (m == m2 - 1) f += cplx(0.0, -0.5);
            if (m == m2 + 1) f += cplx(0.0, -0.5);
        }
        // balanced in: A = Lb N ; balanced out: Lb' = A' / N'
        return f * norm_nm(n, m) / norm_nm(n2, m2);
    }, out);
}

}  // namespace

L2PTable l2p_table(int p) {
    L2PTable t;
    t.p = p;
    const int C = ncoef(p), nu = p * p, ng = (p - 1) * (p - 1);
    t.nu = nu;
    t.ng = ng;
    // dense: U (3 nu x 3C), G (9 ng x 3C)
    std::vector<double> D1[3], D2[3];
    for (int a = 0; a < 3; ++a) {
        D1[a].resize(size_t(nu) * C);
        deriv_matrix(p, a, D1[a].data());
        if (p >= 2) {
            D2[a].resize(size_t(ng) * nu);
            deriv_matrix(p - 1, a, D2[a].data());
        }
    }
    std::vector<double> U(size_t(3) * nu * 3 * C, 0.0), G(size_t(9) * ng * 3 * C, 0.0);
    const int eps[3][3][3] = {{{0, 0, 0}, {0, 0, 1}, {0, -1, 0}},
                              {{0, 0, -1}, {0, 0, 0}, {1, 0, 0}},
                              {{0, 1, 0}, {-1, 0, 0}, {0, 0, 0}}};
    for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) {
                if (!eps[b][c][d]) continue;
                for (int i = 0; i < nu; ++i)
                    for (int j = 0; j < C; ++j)
                        U[size_t(b * nu + i) * 3 * C + d * C + j] += eps[b][c][d] * D1[c][size_t(i) * C + j];
            }
    if (p >= 2) {
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                for (int i = 0; i < ng; ++i)
                    for (int k = 0; k < nu; ++k) {
                        const double dk = D2[a][size_t(i) * nu + k];
                        if (dk == 0.0) continue;
                        for (int j = 0; j < 3 * C; ++j)
                            G[size_t((3 * a + b) * ng + i) * 3 * C + j] += dk * U[size_t(b * nu + k) * 3 * C + j];
                    }
    }
    // evaluation weights: 1 for m = 0, 2 for m > 0 (both real and imaginary slots)
    auto weight = [](int s) { const int n = int(std::sqrt(double(s) + 0.5)); return s == n * n ? 1.0 : 2.0; };
    const int rows = 3 * nu + 9 * ng;
    int width = 0;
    std::vector<std::vector<std::pair<int, double>>> sparse(rows);
    for (int r = 0; r < rows; ++r) {
        const double *src;
        int s;
        if (r < 3 * nu) {
            src = &U[size_t(r) * 3 * C];
            s = r % nu;
        } else {
            src = &G[size_t(r - 3 * nu) * 3 * C];
            s = (r - 3 * nu) % ng;
        }
        for (int j = 0; j < 3 * C; ++j)
            if (std::abs(src[j]) > 1e-300) sparse[r].push_back({j, src[j] * weight(s)});
        width = std::max<int>(width, int(sparse[r].size()));
    }
    t.width = width;
    t.idx.assign(size_t(rows) * width, 0);
    t.w.assign(size_t(rows) * width, 0.0);
    for (int r = 0; r < rows; ++r)
        for (size_t e = 0; e < sparse[r].size(); ++e) {
            t.idx[size_t(r) * width + e] = sparse[r][e].first;
            t.w[size_t(r) * width + e] = sparse[r][e].second;
        }
    return t;
}

namespace {

// Compresses the rows of a dense matrix into fixed-width (index, weight) lists.
void compress(const std::vector<double> &dense, int rows, int cols, int &width, std::vector<int32_t> &idx,
              std::vector<double> &w) {
    width = 1;
    for (int r = 0; r < rows; ++r) {
        int k = 0;
        for (int c = 0; c < cols; ++c) k += dense[size_t(r) * cols + c] != 0.0;
        width = std::max(width, k);
    }
    idx.assign(size_t(rows) * width, 0);
    w.assign(size_t(rows) * width, 0.0);
    for (int r = 0; r < rows; ++r) {
        int k = 0;
        for (int c = 0; c < cols; ++c) {
            const double v = dense[size_t(r) * cols + c];
            if (v == 0.0) continue;
            idx[size_t(r) * width + k] = c;
            w[size_t(r) * width + k] = v;
            ++k;
        }
    }
}

double eval_weight(int s) {
    const int n = int(std::sqrt(double(s) + 0.5));
    return s == n * n ? 1.0 : 2.0;
}

}  // namespace

AdjTables adj_tables(int p) {
    AdjTables t;
    t.p = p;
    const int C = ncoef(p), nu = p * p;
    t.nu = nu;
    // velocity rows of the forward evaluation, U_eval (3 nu x 3C), then transposed
    std::vector<double> D1[3];
    for (int a = 0; a < 3; ++a) {
        D1[a].resize(size_t(nu) * C);
        deriv_matrix(p, a, D1[a].data());
    }
    const int eps[3][3][3] = {{{0, 0, 0}, {0, 0, 1}, {0, -1, 0}},
                              {{0, 0, -1}, {0, 0, 0}, {1, 0, 0}},
                              {{0, 1, 0}, {-1, 0, 0}, {0, 0, 0}}};
    std::vector<double> UT(size_t(3) * C * 3 * nu, 0.0);   // (3C) x (3 nu)
    for (int b = 0; b < 3; ++b)
        for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) {
                if (!eps[b][c][d]) continue;
                for (int i = 0; i < nu; ++i)
                    for (int j = 0; j < C; ++j) {
                        const double v = eps[b][c][d] * D1[c][size_t(i) * C + j] * eval_weight(i);
                        UT[size_t(d * C + j) * 3 * nu + b * nu + i] += v;
                    }
            }
    compress(UT, 3 * C, 3 * nu, t.width_t, t.t_idx, t.t_w);
    // gradient of F = sum_t f_t c_t: with lam = f / w_t, dF/dY_a = sum_s (D_a lam)_s w_s c_s
    std::vector<double> G(size_t(3) * nu * C, 0.0);
    for (int a = 0; a < 3; ++a)
        for (int s2 = 0; s2 < nu; ++s2)
            for (int j = 0; j < C; ++j)
                G[size_t(a * nu + s2) * C + j] = D1[a][size_t(s2) * C + j] * eval_weight(s2) / eval_weight(j);
    compress(G, 3 * nu, C, t.width_g, t.g_idx, t.g_w);
    return t;
}

M2PTable m2p_table(int p) {
    M2PTable t;
    t.p = p;
    const int kt = std::min(2, p), nrow = ncoef(kt), C = ncoef(p), deg = p + 2;
    t.nrow = nrow;
    t.nharm = ncoef(deg);
    // the map (Mb, H) -> loc is bilinear: the real M2L matrix of a unit
    // harmonic vector (one packed real of H set to 1) holds the weights of that
    // harmonic real, for every (row, col)
    std::vector<std::vector<std::pair<int, int>>> ent(nrow);   // (col, harm) per row
    std::vector<std::vector<double>> wts(nrow);
    std::vector<double> m(size_t(nrow) * C);
    for (int j = 0; j < t.nharm; ++j) {
        Harm H{deg, std::vector<cplx>((deg + 1) * (deg + 2) / 2, cplx(0.0, 0.0))};
        const int N = int(std::sqrt(double(j) + 0.5)), r = j - N * N;
        const int mu = (r + 1) / 2;
        H.v[N * (N + 1) / 2 + mu] = (r == 0 || (r & 1)) ? cplx(1.0, 0.0) : cplx(0.0, 1.0);
        real_matrix(kt, p, [&](int k, int l, int n, int mm) -> cplx {
            const double sgn = ((k + l) & 1) ? -1.0 : 1.0;
            return sgn * norm_nm(n + k, mm - l) / (norm_nm(k, l) * norm_nm(n, mm)) * H(n + k, mm - l);
        }, m.data());
        for (int row = 0; row < nrow; ++row)
            for (int c = 0; c < C; ++c) {
                const double v = m[size_t(row) * C + c];
                if (v != 0.0) {
                    ent[row].push_back({c, j});
                    wts[row].push_back(v);
                }
            }
    }
    t.rowptr.assign(1, 0);
    for (int row = 0; row < nrow; ++row) {
        for (size_t e = 0; e < ent[row].size(); ++e) {
            t.col.push_back(ent[row][e].first);
            t.harm.push_back(ent[row][e].second);
            t.w.push_back(wts[row][e]);
        }
        t.rowptr.push_back(int32_t(t.col.size()));
    }
    // slot 0 of the far-field evaluation tables: u and J at the expansion centre
    t.G.assign(size_t(12) * 3 * nrow, 0.0);
    const L2PTable l = l2p_table(p);
    auto take = [&](int o, int r) {
        for (int e = 0; e < l.width; ++e) {
            const double wv = l.w[size_t(r) * l.width + e];
            if (wv == 0.0) continue;
            const int j = l.idx[size_t(r) * l.width + e], comp = j / C, coef = j % C;
            if (coef >= nrow) throw std::logic_error("M2P: evaluation row beyond degree 2");
            t.G[size_t(o) * 3 * nrow + comp * nrow + coef] += wv;
        }
    };
    for (int b = 0; b < 3; ++b) take(b, b * l.nu);
    if (l.ng > 0)
        for (int k = 0; k < 9; ++k) take(3 + k, 3 * l.nu + k * l.ng);
    return t;
}

RecTable rec_table(int p) {
    RecTable t;
    const int n_ent = (p + 1) * (p + 2) / 2;
    t.c1.assign(n_ent, 0.0);
    t.c2.assign(n_ent, 0.0);
    t.diag.assign(p + 1, 0.0);
    for (int m = 1; m <= p; ++m) t.diag[m] = std::sqrt((2.0 * m - 1.0) / (2.0 * m));
    for (int m = 0; m <= p; ++m)
        for (int n = m + 1; n <= p; ++n) {
            const double a = double(n + m) * double(n - m);
            t.c1[n * (n + 1) / 2 + m] = (2.0 * n - 1.0) / std::sqrt(a);
            t.c2[n * (n + 1) / 2 + m] = std::sqrt(double(n + m - 1) * double(n - m - 1) / a);
        }
    return t;
}

}  // namespace vmfmm
