"""Pins of the oracle's expansions and FMM (no GPU).

* Expansion pieces against the direct 1/r sum: the multipole (eq. 10) and
  local (eq. 11) series converge, M2M and L2L are exact re-expansions, the
  local derivatives match finite differences and are harmonic.
* The FMM converges exponentially in p to the direct sum with the cutoff
  dropped beyond adjacent leaves (the far-field model of Sec. 3.1), in free
  space and for periodic image blocks.
* With no far field (free space, one leaf) the FMM is the direct sum.
* A quarter turn of the particle set about the box axis maps the tree onto
  itself; truncation at degree p is rotation invariant, so the FMM output
  must rotate with it to round-off.  A wrong sign, index or transposed
  operand in any translation breaks this.
"""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import direct as D
from oracle import fmm as F
from oracle import harmonics as H
from oracle import tree as T

L = 2 * math.pi


def _pot(x, src, q):
    return np.array([[np.sum(q[:, k] / np.linalg.norm(xx - src, axis=1)) for k in range(q.shape[1])]
                     for xx in x])


def test_multipole_and_local_series_converge():
    rng = np.random.default_rng(0)
    src = rng.uniform(-0.5, 0.5, (7, 3))
    q = rng.standard_normal((7, 2))
    x = np.array([[2.2, -1.5, 1.9], [0.4, 2.6, -1.7]])
    exact = _pot(x, src, q)
    errs = []
    for p in (4, 8, 12, 16):
        M = H.p2m(src, q, p)
        errs.append(np.abs(H.eval_multipole(M, x, p) - exact).max())
    assert all(b < a / 5 for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-9
    # M2L: local expansion about a far centre, evaluated near it
    t = np.array([3.0, 2.0, -2.5])
    near = t + rng.uniform(-0.4, 0.4, (3, 3))
    exact = _pot(near, src, q)
    errs = []
    for p in (4, 8, 12, 16):
        M = H.p2m(src, q, p)
        Lc = (H.m2l_matrix(-t, p) @ M.T).T
        errs.append(np.abs(H.eval_local(Lc, near - t, p) - exact).max())
    assert all(b < a / 5 for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-8


def test_m2m_and_l2l_are_exact():
    rng = np.random.default_rng(1)
    p = 10
    src = rng.uniform(-0.5, 0.5, (9, 3))
    q = rng.standard_normal((9, 3))
    M = H.p2m(src, q, p)
    c = np.array([0.25, -0.25, 0.25])
    M2 = (H.m2m_matrix(-c, p) @ M.T).T
    assert np.abs(M2 - H.p2m(src - c, q, p)).max() < 1e-13 * np.abs(M).max()
    t = np.array([3.0, -2.0, 2.0])
    Lc = (H.m2l_matrix(-t, p) @ M.T).T
    e = np.array([0.2, 0.1, -0.3])
    L2 = (H.l2l_matrix(-e, p) @ Lc.T).T
    pts = t + e + rng.uniform(-0.2, 0.2, (5, 3))
    assert np.abs(H.eval_local(L2, pts - t - e, p) - H.eval_local(Lc, pts - t, p)).max() < 1e-13


def test_local_derivatives_match_fd_and_are_harmonic():
    rng = np.random.default_rng(2)
    p = 8
    src = rng.uniform(-0.5, 0.5, (6, 3)) + np.array([3.0, 0.0, 0.0])
    q = rng.standard_normal((6, 1))
    M = H.p2m(src - np.array([3.0, 0, 0]), q, p)
    Lc = (H.m2l_matrix(np.array([3.0, 0, 0]), p) @ M.T).T
    x = rng.uniform(-0.3, 0.3, (4, 3))
    g, hs = H.local_derivs(Lc, x, p)
    h = 1e-4
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        f = lambda s: H.eval_local(Lc, x + s * e, p)
        fd = (8 * (f(1) - f(-1)) - (f(2) - f(-2))) / (12 * h)
        assert np.abs(fd - g[:, :, a]).max() < 1e-9 * np.abs(g).max()
    assert np.abs(np.trace(hs, axis1=2, axis2=3)).max() < 1e-12 * np.abs(hs).max()


def _model(x, a, sigma, level, periodic):
    tr = T.build(x, (0, 0, 0), L, level, periodic)
    c = tr["coords"]
    return D.direct(tr["xw"], tr["xw"], a, sigma, L, K=periodic, cells_t=c, cells_s=c, level=level)


@pytest.mark.parametrize("truncation", ["square", "triangular"])
@pytest.mark.parametrize("periodic", [0, 1, 2])
def test_fmm_converges_to_far_field_model(periodic, truncation):
    """Square truncation: error ratio below 1/4 per three degrees.  The
    triangular one converges at the slower rate of its error bound, governed by
    (a + b) / R = 0.87 per degree for cells one cell apart against
    a / (R - b) = 0.76 for the square form: below 1/2.5 per three degrees."""
    x, a = W.random_particles(300, 21)
    sigma = 0.2
    u0, J0 = _model(x, a, sigma, 2, periodic)
    eu, ej = [], []
    for p in (3, 6, 9):
        u, J = F.fmm(x, a, sigma, p, 2, periodic=periodic, truncation=truncation)
        eu.append(np.linalg.norm(u - u0) / np.linalg.norm(u0))
        ej.append(np.linalg.norm(J - J0) / np.linalg.norm(J0))
    f, last = (4, 2e-4) if truncation == "square" else (2.5, 2e-3)
    assert eu[1] < eu[0] / f and eu[2] < eu[1] / f
    assert ej[1] < ej[0] / f and ej[2] < ej[1] / f
    assert eu[2] < last and ej[2] < last


def test_fmm_without_far_field_is_direct_sum():
    x, a = W.random_particles(200, 22)
    for level in (0, 1):
        u, J = F.fmm(x, a, 0.3, 6, level, periodic=0)
        u0, J0 = D.direct(x, x, a, 0.3)
        assert np.abs(u - u0).max() < 1e-13 * np.abs(u0).max()
        assert np.abs(J - J0).max() < 1e-13 * np.abs(J0).max()


@pytest.mark.parametrize("periodic", [0, 2])
def test_fmm_rotates_with_its_input(periodic):
    x, a = W.random_particles(250, 23)
    sigma = 0.25
    p, level = 5, 2
    Rm = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    xr = np.stack([L - x[:, 1], x[:, 0], x[:, 2]], axis=1)   # quarter turn about the box axis
    ar = a @ Rm.T
    u, J = F.fmm(x, a, sigma, p, level, periodic=periodic)
    ur, Jr = F.fmm(xr, ar, sigma, p, level, periodic=periodic)
    assert np.abs(ur - u @ Rm.T).max() < 1e-12 * np.abs(u).max()
    assert np.abs(Jr - np.einsum("ia,nab,jb->nij", Rm, J, Rm)).max() < 1e-12 * np.abs(J).max()


def test_level_zero_periodic_is_images_plus_lattice():
    """One leaf with its 26 images in P2P and the lattice operator beyond:
    converges to the image block S_2 with the cutoff dropped outside S_1."""
    x, a = W.random_particles(120, 24)
    sigma = 0.3
    tr = T.build(x, (0, 0, 0), L, 0, 1)
    xw = tr["xw"]
    u1, J1 = D.direct(xw, xw, a, sigma, L, K=1)
    # images of S_2 outside S_1, singular kernel (rho >= 16 there, g = 1 to double precision)
    u2, J2 = _model(x, a, sigma, 0, 2)
    errs = []
    for p in (4, 8, 12):
        u, J = F.fmm(x, a, sigma, p, 0, periodic=2)
        errs.append(np.linalg.norm(u - u2) / np.linalg.norm(u2 - u1))
    assert errs[1] < errs[0] / 4 and errs[2] < errs[1] / 4


@pytest.mark.parametrize("k", [2, 3, 4])
def test_supercell_multipole_is_the_image_block_multipole(k):
    """Ring k of the lattice sum sees the block of 3^(k-2) image boxes per side
    through one multipole about the block's centre, built from the root
    multipole by M2M (27 copies per step).  Brute force: the multipole of every
    particle copy x_j + n L, n in {-R..R}^3 with R = (3^(k-2) - 1)/2, about that
    centre.  M2M is exact up to degree p, so the two agree to round-off; a wrong
    supercell spacing or centring does not."""
    x, a = W.random_particles(20, 27)
    p = 8
    c0 = np.full(3, L / 2)
    m0 = H.p2m(x - c0, a, p)
    R = (3 ** (k - 2) - 1) // 2
    img = np.array(list(itertools.product(range(-R, R + 1), repeat=3)), np.float64)
    copies = (x[None, :, :] - c0 + img[:, None, :] * L).reshape(-1, 3)
    brute = H.p2m(copies, np.tile(a, (len(img), 1)), p)
    msup = F.supercell_multipole(m0, p, L, k)
    assert np.abs(msup - brute).max() < 1e-12 * np.abs(brute).max()


@pytest.mark.parametrize("level", [0, 1])
def test_lattice_rings_beyond_s2_converge_to_image_sums(level):
    """The rings k >= 3 of the lattice operator (the paper's 27^3 block is K = 3)
    against the direct sum over the image boxes of S_K minus S_2 with the cutoff
    dropped (rho >= 16 there): the difference FMM(K) - FMM(2) isolates them, and
    so does model(K) - model(2).  Ring 3's supercells (3L wide, at >= 6L) bound
    the error by (sqrt(3)/2 (3 + 1) / 6)^p = 0.58^p: it must fall at least 4x
    every 4 degrees and reach 1e-4 at p = 12, for K = 3 and K = 4 alike.  The
    whole periodic sum S_K at level 0/1 converges to the image-block model too."""
    x, a = W.random_particles(30, 24)
    sigma = 0.3
    m1, m2, m3, m4 = (_model(x, a, sigma, level, K) for K in (1, 2, 3, 4))
    errs = {3: [], 4: []}
    errJ = {3: [], 4: []}
    full = []
    for p in (4, 8, 12):
        u2, J2 = F.fmm(x, a, sigma, p, level, periodic=2)
        for K, mk in ((3, m3), (4, m4)):
            uk, Jk = F.fmm(x, a, sigma, p, level, periodic=K)
            du, dJ = mk[0] - m2[0], mk[1] - m2[1]
            errs[K].append(np.linalg.norm((uk - u2) - du) / np.linalg.norm(du))
            errJ[K].append(np.linalg.norm((Jk - J2) - dJ) / np.linalg.norm(dJ))
            if K == 3:
                full.append(np.linalg.norm(uk - m3[0]) / np.linalg.norm(m3[0] - m1[0]))
    for e in list(errs.values()) + list(errJ.values()) + [full]:
        assert e[1] < e[0] / 4 and e[2] < e[1] / 4, e
    for K in (3, 4):
        assert errs[K][2] < 1e-4 and errJ[K][2] < 1e-4
    # ring 4 adds to ring 3 (a K = 4 sum is not a K = 3 sum)
    assert np.linalg.norm(m4[0] - m3[0]) > 1e-3 * np.linalg.norm(m3[0] - m2[0])


@pytest.mark.parametrize("periodic,level", [(3, 2), (0, 2), (1, 1), (2, 0)])
def test_sampled_fmm_equals_full_fmm(periodic, level):
    """The per-target variant used at full sizes repeats the full oracle's arithmetic."""
    x, a = W.random_field(16, 4.0, 3)
    h = L / 16
    u, J = F.fmm(x, a, h, 6, level, periodic=periodic)
    t = np.random.default_rng(0).choice(len(x), 40, replace=False)
    us, Js = F.fmm_at(x, a, h, 6, level, t, periodic=periodic, chunk=1000)
    assert np.abs(us - u[t]).max() < 1e-14 * np.abs(u).max()
    assert np.abs(Js - J[t]).max() < 1e-14 * np.abs(J).max()


@pytest.mark.parametrize("periodic", [0, 1, 2])
def test_fmm_at_points_converges_to_far_field_model(periodic):
    """Velocity at points other than the particles: the same far-field model
    (g = 1 between non-adjacent leaves, the point in the leaf its position
    falls in) is approached at the FMM's rate; the points' own leaves may be
    empty of particles."""
    x, a = W.random_particles(300, 25)
    rng = np.random.default_rng(26)
    y = rng.uniform(-2.0, L + 2.0, size=(60, 3)) if periodic else rng.uniform(0.0, L, size=(60, 3))
    sigma, level = 0.2, 2
    tr = T.build(x, (0, 0, 0), L, level, periodic)
    yw = T.wrap(y, (0, 0, 0), L) if periodic else y
    cy = T.leaf_coords(yw, (0, 0, 0), L, level)
    u0, J0 = D.direct(yw, tr["xw"], a, sigma, L, K=periodic, cells_t=cy, cells_s=tr["coords"], level=level)
    eu, ej = [], []
    for p in (3, 6, 9):
        u, J = F.fmm_points(x, a, sigma, p, level, y, periodic=periodic)
        eu.append(np.linalg.norm(u - u0) / np.linalg.norm(u0))
        ej.append(np.linalg.norm(J - J0) / np.linalg.norm(J0))
    assert eu[1] < eu[0] / 4 and eu[2] < eu[1] / 4
    assert ej[1] < ej[0] / 4 and ej[2] < ej[1] / 4
    # 60 points: the worst-placed ones weigh more than among 300 particles
    assert eu[2] < 5e-4 and ej[2] < 5e-4


def test_triangular_truncation_keeps_low_total_degree():
    """n + n' <= p keeps 2926 of the 14641 products per component at p = 10;
    below that bound the triangular operators equal the square ones."""
    import oracle.harmonics as Hm
    deg = np.floor(np.sqrt(np.arange(Hm.ncoef(10)) + 0.5)).astype(int)
    assert int(((deg[:, None] + deg[None, :]) <= 10).sum()) == 2926
    sq = F._m2l_matrices(2, 6, L)
    tr = F._m2l_matrices(2, 6, L, "triangular")
    d6 = deg[:Hm.ncoef(6)]
    keep = (d6[:, None] + d6[None, :]) <= 6
    for off in list(sq)[:20]:
        assert np.array_equal(tr[off][keep], sq[off][keep]) and not np.any(tr[off][~keep])
