"""FMM evaluation of the regularised Biot-Savart velocity and its gradient.

Test infrastructure: the oracle.  The steps follow the paper's Sec. 3.1:

* the vector potential psi = G * omega has three Laplace components, one per
  strength component; each is expanded in multipoles (eq. 10) and locals
  (eq. 11) of degree 0..p in the nomenclature of Cheng et al.;
* far-field velocity u = curl psi (eqs. 12-13) and its gradient (the tensor
  the stretching term of eqs. 14-15 contracts) come from the first and
  second derivatives of the local expansions; the cutoff is dropped there;
* the near field (the 27 adjacent leaves) is the exact regularised direct
  sum (last paragraph of Sec. 3.1);
* periodic problems add the image boxes S_K minus S_1 by multipole
  expansions only, at a cost independent of N (same paragraph): rings of
  supercells 3^(k-2) L wide, built by M2M from the root multipole, each
  shifted to the root by M2L.

Step order: tree -> P2M -> M2M -> (lattice) -> L2L + M2L per level -> L2P ->
P2P -> sum.  Everything is complex128 / float64 NumPy, no blocking.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import direct as _direct
from . import harmonics as H
from . import tree as T

INV4PI = 1.0 / (4.0 * math.pi)


def _centres(keys, level, lo, box_len):
    w = box_len / (1 << level)
    return np.asarray(lo, np.float64) + (T.demorton(keys, level) + 0.5) * w


def supercell_multipole(m0, p, box_len, k):
    """Multipole, about its own centre, of the supercell of ring k >= 2: the
    block of 3^(k-2) image boxes per side.  Ring 2's supercell is the root box
    itself (``m0``); each further ring's is the M2M sum of 27 copies of the
    previous one, centred at e 3^(j-3) L for e in [-1, 1]^3."""
    block = np.array(list(itertools.product((-1, 0, 1), repeat=3)), np.float64)
    msup = m0
    for j in range(3, k + 1):
        s_small = 3.0 ** (j - 3) * box_len
        msup = sum(H.m2m_matrix(e * s_small, p) @ msup.T for e in block).T
    return msup


def lattice_local(m0, p, box_len, K):
    """Local expansion at the root centre of the images S_K minus S_1.

    ``m0``: root multipole, complex (ncomp, C).  Ring k (2 <= k <= K) is made
    of the 9^3 - 3^3 = 702 supercells of width s = 3^(k-2) L centred at d s,
    d in [-4, 4]^3 minus [-1, 1]^3 (together exactly the boxes of S_k minus
    S_(k-1)); a supercell's multipole is the M2M sum of the 27 copies of the
    next smaller one.
    """
    out = np.zeros_like(m0)
    if K < 2:
        return out
    ring = np.array([d for d in itertools.product(range(-4, 5), repeat=3)
                     if max(abs(v) for v in d) > 1], np.float64)
    for k in range(2, K + 1):
        msup = supercell_multipole(m0, p, box_len, k)
        s = 3.0 ** (k - 2) * box_len
        mats = H.m2l_matrices(ring * s, p)
        for T_d in mats:
            out = out + (T_d @ msup.T).T
    return out


def _m2l_matrices(level, p, box_len, truncation="square"):
    """M2L operators of the 316 offsets at a level.  "triangular" keeps the
    terms of target degree j and source degree n with j + n <= p only (the
    classical truncation of the local expansion of eq. 13); "square" keeps
    every j, n <= p."""
    w = box_len / (1 << level)
    offs = T.all_offsets()
    mats = H.m2l_matrices(np.array(offs, np.float64) * w, p)
    if truncation == "triangular":
        deg = np.floor(np.sqrt(np.arange(H.ncoef(p)) + 0.5)).astype(np.int64)
        mats = [m * ((deg[:, None] + deg[None, :]) <= p) for m in mats]
    elif truncation != "square":
        raise ValueError(truncation)
    return dict(zip(offs, mats))


def fmm(x, alpha, sigma, p, level, box_lo=(0.0, 0.0, 0.0), box_len=2 * math.pi, periodic=0, truncation="square"):
    """u (N,3) and J (N,3,3) (J[a,b] = d u_b / d x_a) in the caller's order."""
    x = np.asarray(x, np.float64)
    alpha = np.asarray(alpha, np.float64)
    n = x.shape[0]
    lo = np.asarray(box_lo, np.float64)
    tr = T.build(x, lo, box_len, level, periodic)
    xw, perm, start, count = tr["xw"], tr["perm"], tr["start"], tr["count"]
    leaf_of = tr["keys"]
    nleaf = 1 << (3 * level)
    C = H.ncoef(p)

    lmin = 0 if periodic else 2
    far = level >= lmin
    u_far = np.zeros((n, 3))
    J_far = np.zeros((n, 3, 3))
    if far:
        # P2M at the leaf centres (eq. 10: M = sum gamma rho^n Y_n^{-m}).
        centres = _centres(np.arange(nleaf), level, lo, box_len)
        M = {level: np.zeros((nleaf, 3, C), np.complex128)}
        for k in np.nonzero(count)[0]:
            ids = perm[start[k]:start[k] + count[k]]
            M[level][k] = H.p2m(xw[ids] - centres[k], alpha[ids], p)
        # M2M up to the top level.
        for l in range(level - 1, lmin - 1, -1):
            wc = box_len / (1 << (l + 1))
            ncell = 1 << (3 * l)
            M[l] = np.zeros((ncell, 3, C), np.complex128)
            for o in range(8):
                ob = np.array([(o >> d) & 1 for d in range(3)], np.float64)
                Tm = H.m2m_matrix((ob - 0.5) * wc, p)
                M[l] += M[l + 1][o::8] @ Tm.T
        # Downward pass.
        Lc = {}
        if periodic:
            Lc[0] = lattice_local(M[0][0], p, box_len, periodic)[None]
        for l in range(max(lmin, 1) if periodic else lmin, level + 1):
            ncell = 1 << (3 * l)
            Ll = np.zeros((ncell, 3, C), np.complex128)
            if (l - 1) in Lc:
                w = box_len / (1 << l)
                for o in range(8):
                    ob = np.array([(o >> d) & 1 for d in range(3)], np.float64)
                    Tl = H.l2l_matrix(-(ob - 0.5) * w, p)
                    Ll[o::8] += Lc[l - 1] @ Tl.T
            mats = _m2l_matrices(l, p, box_len, truncation)
            side = 1 << l
            keys = np.arange(ncell)
            coords = T.demorton(keys, l)
            for o in range(8):
                tk = keys[o::8]
                tc = coords[o::8]
                for d in T.offsets_for_octant(o):
                    sc = tc + np.array(d)
                    if periodic:
                        sc = np.mod(sc, side)
                        ok = np.ones(len(tk), bool)
                    else:
                        ok = np.all((sc >= 0) & (sc < side), axis=1)
                    if not np.any(ok):
                        continue
                    sk = T.morton(sc[ok], l)
                    Ll[tk[ok]] += M[l][sk] @ mats[d].T
            Lc[l] = Ll
        # L2P: first and second derivatives of the leaf local expansions.
        Lleaf = Lc[level]
        ctr = centres
        for k in np.nonzero(count)[0]:
            ids = perm[start[k]:start[k] + count[k]]
            g, h = H.local_derivs(Lleaf[k], xw[ids] - ctr[k], p)   # (P,3comp,3), (P,3comp,3,3)
            # d_c psi_d = g[:, d, c] / (4 pi); u_b = eps_bcd d_c psi_d
            u_far[ids, 0] = g[:, 2, 1] - g[:, 1, 2]
            u_far[ids, 1] = g[:, 0, 2] - g[:, 2, 0]
            u_far[ids, 2] = g[:, 1, 0] - g[:, 0, 1]
            for a in range(3):
                J_far[ids, a, 0] = h[:, 2, a, 1] - h[:, 1, a, 2]
                J_far[ids, a, 1] = h[:, 0, a, 2] - h[:, 2, a, 0]
                J_far[ids, a, 2] = h[:, 1, a, 0] - h[:, 0, a, 1]
        u_far *= INV4PI
        J_far *= INV4PI

    # P2P over the 27 adjacent leaves with the exact cutoff.
    u_near = np.zeros((n, 3))
    J_near = np.zeros((n, 3, 3))
    coords_leaf = T.demorton(np.arange(nleaf), level)
    for k in np.nonzero(count)[0]:
        ids = perm[start[k]:start[k] + count[k]]
        srcs, shifts = [], []
        for nk, img in T.neighbours(coords_leaf[k], level, periodic):
            if count[nk] == 0:
                continue
            sid = perm[start[nk]:start[nk] + count[nk]]
            srcs.append(sid)
            shifts.append(np.broadcast_to(np.array(img, np.float64) * box_len, (len(sid), 3)))
        sid = np.concatenate(srcs)
        xs = xw[sid] + np.concatenate(shifts)
        u, J = _direct.direct(xw[ids], xs, alpha[sid], sigma, box_len, K=0)
        u_near[ids] = u
        J_near[ids] = J
    del leaf_of
    return u_far + u_near, J_far + J_near


def fmm_at(x, alpha, sigma, p, level, targets, box_lo=(0.0, 0.0, 0.0), box_len=2 * math.pi, periodic=0,
           chunk=1 << 18, truncation="square"):
    """u and J of ``fmm`` at the particles ``targets`` only (indices in caller order).

    Same steps and arithmetic as ``fmm``: P2M for every leaf and M2M for every
    cell, but the downward pass only along the ancestors of the targets'
    leaves, and L2P / P2P only at the targets.  Used to check the full-size
    workloads one sampled particle at a time.
    """
    x = np.asarray(x, np.float64)
    return fmm_points(x, alpha, sigma, p, level, x[np.asarray(targets, np.int64)], box_lo, box_len, periodic,
                      chunk, truncation)


def fmm_points(x, alpha, sigma, p, level, y, box_lo=(0.0, 0.0, 0.0), box_len=2 * math.pi, periodic=0,
               chunk=1 << 18, truncation="square"):
    """u and J that the particles (x, alpha) induce at the points y (m, 3).

    The same model as at the particles: each point belongs to the leaf its
    position falls in (periodic: after the wrap, free space: clamped like a
    particle); the local expansion of that leaf gives the far field and the
    exact regularised sum over the 27 adjacent leaves the near field.
    """
    x = np.asarray(x, np.float64)
    alpha = np.asarray(alpha, np.float64)
    lo = np.asarray(box_lo, np.float64)
    tr = T.build(x, lo, box_len, level, periodic)
    xw, perm, start, count, keys = tr["xw"], tr["perm"], tr["start"], tr["count"], tr["keys"]
    yw = T.wrap(y, lo, box_len) if periodic else np.asarray(y, np.float64)
    nleaf = 1 << (3 * level)
    C = H.ncoef(p)
    lmin = 0 if periodic else 2
    far = level >= lmin
    nt = len(yw)
    u = np.zeros((nt, 3))
    J = np.zeros((nt, 3, 3))
    tleaf = T.morton(T.leaf_coords(yw, lo, box_len, level), level)
    if far:
        centres = _centres(np.arange(nleaf), level, lo, box_len)
        neg = np.array([H.idx(n, -m) for n in range(p + 1) for m in range(-n, n + 1)])
        M = {level: np.zeros((nleaf, 3, C), np.complex128)}
        # P2M, a run of whole leaves at a time (particles are contiguous per leaf);
        # M[leaf] = sum over its particles of alpha_j R^{-m}(y_j)
        leaf_lo = 0
        while leaf_lo < nleaf:
            leaf_hi = leaf_lo
            while leaf_hi < nleaf and start[leaf_hi] + count[leaf_hi] - start[leaf_lo] <= chunk:
                leaf_hi += 1
            leaf_hi = max(leaf_hi, leaf_lo + 1)
            a0, a1 = start[leaf_lo], start[leaf_hi - 1] + count[leaf_hi - 1]
            if a1 > a0:
                ids = perm[a0:a1]
                lf = keys[ids]
                R = H.regular(xw[ids] - centres[lf], p)[:, neg]
                al = alpha[ids]
                cnts = count[leaf_lo:leaf_hi]
                if np.all(cnts == cnts[0]):
                    k = int(cnts[0])
                    M[level][leaf_lo:leaf_hi] = np.einsum("lpk,lpc->lkc", al.reshape(-1, k, 3),
                                                          R.reshape(-1, k, C))
                else:
                    segs = start[leaf_lo:leaf_hi] - a0
                    occupied = cnts > 0
                    sums = np.add.reduceat(al[:, :, None] * R[:, None, :], segs[occupied], axis=0)
                    M[level][np.arange(leaf_lo, leaf_hi)[occupied]] = sums
            leaf_lo = leaf_hi
        for l in range(level - 1, lmin - 1, -1):
            wc = box_len / (1 << (l + 1))
            M[l] = np.zeros((1 << (3 * l), 3, C), np.complex128)
            for o in range(8):
                ob = np.array([(o >> d) & 1 for d in range(3)], np.float64)
                M[l] += M[l + 1][o::8] @ H.m2m_matrix((ob - 0.5) * wc, p).T
        # downward pass along the ancestor chains
        Lc = {}
        if periodic:
            Lc[0] = {0: lattice_local(M[0][0], p, box_len, periodic)}
        for l in range(1 if periodic else lmin, level + 1):
            cells = np.unique(tleaf >> (3 * (level - l)))
            Ll = {int(c): np.zeros((3, C), np.complex128) for c in cells}
            if (l - 1) in Lc:
                w = box_len / (1 << l)
                for c in cells:
                    o = int(c) & 7
                    ob = np.array([(o >> d) & 1 for d in range(3)], np.float64)
                    Ll[int(c)] += (H.l2l_matrix(-(ob - 0.5) * w, p) @ Lc[l - 1][int(c) >> 3].T).T
            mats = _m2l_matrices(l, p, box_len, truncation)
            side = 1 << l
            coords = T.demorton(cells, l)
            for c, cc in zip(cells, coords):
                o = int(c) & 7
                for d in T.offsets_for_octant(o):
                    sc = cc + np.array(d)
                    if periodic:
                        sc = np.mod(sc, side)
                    elif np.any(sc < 0) or np.any(sc >= side):
                        continue
                    sk = int(T.morton(sc[None], l)[0])
                    Ll[int(c)] += (mats[d] @ M[l][sk].T).T
            Lc[l] = Ll
        centres_t = centres[tleaf]
        for i in range(nt):
            g, h = H.local_derivs(Lc[level][int(tleaf[i])], (yw[i] - centres_t[i])[None], p)
            u[i] = [g[0, 2, 1] - g[0, 1, 2], g[0, 0, 2] - g[0, 2, 0], g[0, 1, 0] - g[0, 0, 1]]
            for a in range(3):
                J[i, a] = [h[0, 2, a, 1] - h[0, 1, a, 2], h[0, 0, a, 2] - h[0, 2, a, 0],
                           h[0, 1, a, 0] - h[0, 0, a, 1]]
        u *= INV4PI
        J *= INV4PI
    coords_leaf = T.demorton(np.unique(tleaf), level)
    leaf_coord = dict(zip(np.unique(tleaf).tolist(), coords_leaf))
    for i in range(nt):
        srcs, shifts = [], []
        for nk, img in T.neighbours(leaf_coord[int(tleaf[i])], level, periodic):
            if count[nk] == 0:
                continue
            sid = perm[start[nk]:start[nk] + count[nk]]
            srcs.append(sid)
            shifts.append(np.broadcast_to(np.array(img, np.float64) * box_len, (len(sid), 3)))
        if not srcs:
            continue
        sid = np.concatenate(srcs)
        xs = xw[sid] + np.concatenate(shifts)
        un, Jn = _direct.direct(yw[i][None], xs, alpha[sid], sigma, box_len, K=0)
        u[i] += un[0]
        J[i] += Jn[0]
    return u, J
