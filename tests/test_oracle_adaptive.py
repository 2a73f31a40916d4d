"""Pins of the oracle's adaptive hybrid treecode-FMM (no GPU).

* Tree: every particle is found in the leaf that a walk from the root by its
  own coordinates reaches; a cell is split exactly when it holds more than
  ncrit particles above the finest level; cells are level-major and sorted by
  key; children tile their parent's particle range.
* Lists: every (target particle, source particle, image of S_1) triple is
  covered by exactly one interaction (brute force over all triples); each
  interaction has the geometry its kind requires (P2P: leaves that touch, or
  of different levels with the finer one's parent touching the other; M2L:
  one level, apart, parents touching; M2P: target leaf, finer split source
  apart whose parent touches it; P2L: the mirror image).
* On a tree that happens to be uniform the lists are the uniform FMM's (the
  189-offset interaction lists and the 27 neighbours, no cell-particle
  interactions) and the evaluation equals the uniform oracle FMM to
  round-off, free and periodic with the lattice (K = 3).
* On clustered particles the FMM converges geometrically in p to the sum it
  models (exact kernel on P2P pairs, g = 1 elsewhere), free and periodic.
* M2P and P2L on their own: a source cell's multipole at the particles of a
  coarser leaf, and a coarser leaf's particles in a cell's local expansion,
  converge to the direct g = 1 sums of their particles.
"""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import adaptive as A
from oracle import direct as D
from oracle import fmm as F
from oracle import harmonics as H
from oracle import tree as T

L = 2 * math.pi


@pytest.mark.parametrize("periodic", [0, 1])
def test_tree_structure(periodic):
    x, _ = W.clustered_particles(700, 3)
    ncrit, ml = 20, 5
    tr = A.build_tree(x, (0, 0, 0), L, ncrit, ml, periodic)
    lev, key, start, count, leaf, child = (tr[k] for k in ("level", "key", "start", "count", "leaf", "child"))
    # level-major, ascending key inside a level
    order = np.lexsort((key, lev))
    assert np.array_equal(order, np.arange(len(lev)))
    # split exactly when over ncrit above the finest level
    assert np.array_equal(~leaf, (count > ncrit) & (lev < ml))
    # children tile the parent's range
    for ci in np.nonzero(~leaf)[0]:
        ch = child[ci][child[ci] >= 0]
        assert count[ch].sum() == count[ci]
        assert start[ch].min() == start[ci]
        assert np.all(key[ch] >> 3 == key[ci]) and np.all(lev[ch] == lev[ci] + 1)
    # every particle lies in the leaf its own coordinates lead to from the root
    fc = T.leaf_coords(tr["xw"], (0, 0, 0), L, ml)
    pos = np.empty(len(x), np.int64)
    pos[tr["perm"]] = np.arange(len(x))
    for i in range(len(x)):
        ci = 0
        while not leaf[ci]:
            l = lev[ci] + 1
            c = fc[i] >> (ml - l)
            o = (c[0] & 1) | ((c[1] & 1) << 1) | ((c[2] & 1) << 2)
            ci = child[ci][o]
            assert ci >= 0
        assert start[ci] <= pos[i] < start[ci] + count[ci]


@pytest.mark.parametrize("periodic", [0, 1])
def test_every_pair_covered_once(periodic):
    x, _ = W.clustered_particles(260, 7)
    tr = A.build_tree(x, (0, 0, 0), L, 6, 4, periodic)
    ls = A.lists(tr)
    assert all(len(ls[k]) for k in ("p2p", "m2l", "m2p", "p2l"))
    n = len(x)
    nsh = 27 if periodic else 1
    cover = np.zeros((n, n, nsh), np.int16)

    def parts_below(ci):
        s0 = tr["start"][ci]
        return tr["perm"][s0:s0 + tr["count"][ci]]

    for k, arr in ls.items():
        for t, s, c in arr:
            ti, si = parts_below(t), parts_below(s)
            cover[np.ix_(ti, si, [c if periodic else 0])] += 1
    assert cover.min() == 1 and cover.max() == 1


@pytest.mark.parametrize("periodic", [0, 1])
def test_interaction_geometry(periodic):
    x, _ = W.clustered_particles(500, 11)
    tr = A.build_tree(x, (0, 0, 0), L, 8, 5, periodic)
    ls = A.lists(tr)
    lev, leaf, par = tr["level"], tr["leaf"], tr["parent"]
    touch = lambda a, b, c: A.touching(tr, a, b, A.code_shift(c))
    apart = 0
    for t, s, c in ls["p2p"]:
        assert leaf[t] and leaf[s]
        if not touch(t, s, c):
            # separated leaves are direct only across levels, with the finer
            # one's parent touching the coarser leaf
            assert lev[t] != lev[s]
            f, g = (t, s) if lev[t] > lev[s] else (s, t)
            assert touch(par[f], g, c) if f == t else touch(g, par[f], c)
            apart += 1
    assert apart > 0
    for t, s, c in ls["m2l"]:
        assert lev[t] == lev[s] and not touch(t, s, c)
        assert par[t] < 0 or touch(par[t], par[s], c)
    for t, s, c in ls["m2p"]:
        assert leaf[t] and not leaf[s] and lev[s] > lev[t] and not touch(t, s, c) and touch(t, par[s], c)
    for t, s, c in ls["p2l"]:
        assert leaf[s] and not leaf[t] and lev[t] > lev[s] and not touch(t, s, c) and touch(par[t], s, c)


@pytest.mark.parametrize("periodic", [0, 3])
def test_uniform_tree_is_the_uniform_fmm(periodic):
    # 8 particles in every level-2 leaf: ncrit 7 splits down to level 2 everywhere
    ml = 2
    x, a = W.particles_with_leaf_counts([8] * 64, ml, 5)
    sigma, p = 0.25, 6
    tr = A.build_tree(x, (0, 0, 0), L, 7, ml, periodic)
    assert np.all(tr["level"][tr["leaf"]] == ml) and tr["leaf"].sum() == 64
    ls = A.lists(tr)
    assert len(ls["m2p"]) == 0 and len(ls["p2l"]) == 0
    # M2L lists: the uniform interaction lists, cell by cell (keys at each level)
    lev, key = tr["level"], tr["key"]
    cell_of = {(int(lev[c]), int(key[c])): c for c in range(len(lev))}
    got = sorted(map(tuple, ls["m2l"].tolist()))
    want = []
    for ci in range(len(lev)):
        if lev[ci] < (1 if periodic else 2):
            continue
        for sk, _, img in T.interaction_list(int(key[ci]), int(lev[ci]), periodic):
            want.append((ci, cell_of[(int(lev[ci]), int(sk))], A.shift_code(img)))
    assert got == sorted(want)
    got = sorted(map(tuple, ls["p2p"].tolist()))
    want = []
    for ci in np.nonzero(tr["leaf"])[0]:
        c = T.demorton(np.array([key[ci]]), ml)[0]
        for nk, img in T.neighbours(c, ml, periodic):
            want.append((ci, cell_of[(ml, nk)], A.shift_code(img)))
    assert got == sorted(want)
    u, J = A.fmm(x, a, sigma, p, 7, ml, periodic=periodic, tree=tr, lst=ls)
    uu, Ju = F.fmm(x, a, sigma, p, ml, periodic=periodic)
    assert np.linalg.norm(u - uu) / np.linalg.norm(uu) < 1e-12
    assert np.linalg.norm(J - Ju) / np.linalg.norm(Ju) < 1e-12


@pytest.mark.parametrize("periodic", [0, 1])
def test_converges_to_the_model_sum(periodic):
    x, a = W.clustered_particles(250 if periodic else 400, 5)
    sigma, ncrit, ml = L / 64, 12 if periodic else 16, 4
    tr = A.build_tree(x, (0, 0, 0), L, ncrit, ml, periodic)
    ls = A.lists(tr)
    assert len(ls["m2p"]) and len(ls["p2l"])
    ud, Jd = A.model_direct(x, a, sigma, tr, ls)
    eu, eJ = [], []
    for p in (3, 6, 9):
        u, J = A.fmm(x, a, sigma, p, ncrit, ml, periodic=periodic, tree=tr, lst=ls)
        eu.append(np.linalg.norm(u - ud) / np.linalg.norm(ud))
        eJ.append(np.linalg.norm(J - Jd) / np.linalg.norm(Jd))
    assert all(b < a_ / 5 for a_, b in zip(eu, eu[1:])), eu
    assert all(b < a_ / 4 for a_, b in zip(eJ, eJ[1:])), eJ
    assert eu[-1] < 1e-4 and eJ[-1] < 1e-3, (eu, eJ)


def test_cell_particle_primitives():
    """M2P of a small cell's multipole at the particles of a larger leaf one
    cell width away, and P2L of a large leaf's particles into a small cell's
    local expansion, against direct g = 1 sums of the same particles."""
    rng = np.random.default_rng(2)
    ws = 0.5                                    # source cell width, centre 0
    src = rng.uniform(-ws / 2, ws / 2, (30, 3))
    q = rng.standard_normal((30, 3))
    tgt = np.array([1.5 * ws, 0, 0]) + rng.uniform(-0.0, 0.25, (12, 3))   # gap >= one source width
    cells = np.zeros((12, 3), np.int32), np.full((30, 3), 2, np.int32)
    ud, Jd = D.direct(tgt, src, q, 0.01, L, K=0, cells_t=cells[0], cells_s=cells[1], level=4)
    errs = []
    for p in (4, 8, 12):
        M = H.p2m(src, q, p)
        Lp = np.einsum("pij,kj->pki", H.m2l_matrices(-tgt, p), M)
        g, h = A._derivs_at_centre(Lp, p)
        u = A._curl(g) * F.INV4PI
        J = A._curl_grad(h) * F.INV4PI
        errs.append(max(np.abs(u - ud).max() / np.abs(ud).max(), np.abs(J - Jd).max() / np.abs(Jd).max()))
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10 and errs[2] < 2e-4, errs
    # P2L: target cell of width wt at the origin, sources of a coarser leaf beyond it
    wt = 0.25
    srcs = np.array([1.5 * wt + 0.6, 0.1, -0.2]) + rng.uniform(-0.3, 0.3, (25, 3))
    qs = rng.standard_normal((25, 3))
    pts = rng.uniform(-wt / 2, wt / 2, (10, 3))
    cells = np.zeros((10, 3), np.int32), np.full((25, 3), 2, np.int32)
    ud, Jd = D.direct(pts, srcs, qs, 0.01, L, K=0, cells_t=cells[0], cells_s=cells[1], level=4)
    errs = []
    for p in (4, 8, 12):
        Lc = np.zeros((3, H.ncoef(p)), np.complex128)
        for y, qq in zip(srcs, qs):
            Lc += H.p2m(np.zeros((1, 3)), qq[None], p) @ H.m2l_matrix(y, p).T
        g, h = H.local_derivs(Lc, pts, p)
        u = A._curl(g) * F.INV4PI
        J = A._curl_grad(h) * F.INV4PI
        errs.append(max(np.abs(u - ud).max() / np.abs(ud).max(), np.abs(J - Jd).max() / np.abs(Jd).max()))
    assert errs[1] < errs[0] / 10 and errs[2] < errs[1] / 10 and errs[2] < 2e-4, errs
