"""Adaptive hybrid treecode-FMM (test infrastructure: the oracle).

Sec. 3.2 of the paper replaces the uniform tree by an adaptive one whose
leaves hold at most a chosen number of particles, traversed by a stack-based
O(N) algorithm whose interactions are cell-cell or cell-particle, with the
number of particles per leaf tuned automatically.  The paper defers the
details to its companion publication; the readings used here (the GPU code
must reproduce the tree and the lists bit for bit):

* tree: particles keyed at the finest allowed level ``max_level`` exactly as
  the uniform tree (wrap, leaf coordinates, Morton bits, stable sort); a cell
  is split when it holds more than ``ncrit`` particles and lies above
  ``max_level``; only non-empty children exist.  Cells are numbered level by
  level, ascending key within a level.
* acceptance criterion (MAC): two cells interact through expansions when
  their closed cubes do not touch (integer test on the finest grid, the
  image shift included); cells that touch are refined further.  For cells of
  one level this is the uniform FMM's "not adjacent", so on a uniform tree
  the lists are the uniform FMM's.
* dual traversal: a stack of (target cell, source cell, image shift) pairs,
  starting from the root against itself (periodic: against its 27 images,
  the block S_1).  A pair that passes the MAC is an interaction: M2L
  (cell-cell, same level), M2P (cell-particle: the source cell's multipole
  at the target leaf's particles, source finer) or P2L (particle-cell: the
  source leaf's particles into the target cell's local expansion, source
  coarser).  A pair of touching leaves is P2P (exact regularised kernel).
  Otherwise the pair is refined: both cells when both are split and of one
  level, else the one that is split.  Every (target particle, source
  particle, image) triple is then covered by exactly one interaction.
* cost choice: the hybrid takes the cheaper of the interactions that are
  valid for a pair (Sec. 3.2 argues from the rule that a well-built FMM
  always does).  A cell-particle interaction replaces |cell| particles by
  one expansion of (p+1)^2 terms per component and costs thousands of
  operations per particle of the other side, while the exact kernel costs
  tens per pair, so the break-even cell holds some hundreds of particles.
  The reading: a cell-particle interaction needs a split cell (more than
  ncrit particles, ncrit being tuned) on its cell side; two leaves of
  different levels that do not touch are P2P as well.  Between cells of one
  level (M2L) nothing changes, so the uniform-tree reduction holds.
* the cutoff is dropped in all expansion interactions (text after
  eqs. 12-13); the separation of the cells, at least one width of the
  smaller cell, is what makes g = 1 there.
* periodic: images beyond S_1 by the lattice operator on the root multipole
  (Sec. 3.1 last paragraph), as in the uniform FMM.
* auto-tuning: the GPU code times candidate leaf sizes and keeps the fastest
  (``ncrit`` is an input here).

Every expansion step reuses the pinned primitives of ``harmonics``: P2M,
M2M, L2L and M2L as in ``fmm``; M2P is the M2L of the source multipole to a
local expansion about the target particle, whose first and second derivatives
at its centre are those of the multipole potential; P2L is the M2L of a
source particle's own point multipole (degree 0 only) into the target cell.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import direct as _direct
from . import harmonics as H
from . import tree as T
from .fmm import INV4PI, lattice_local

SHIFTS = [tuple(s) for s in itertools.product((-1, 0, 1), repeat=3)]   # (sx, sy, sz) order of codes below


def shift_code(s):
    """0..26 for an image shift s in {-1,0,1}^3: (sx+1) + 3(sy+1) + 9(sz+1)."""
    return (s[0] + 1) + 3 * (s[1] + 1) + 9 * (s[2] + 1)


def code_shift(c):
    return (c % 3 - 1, (c // 3) % 3 - 1, c // 9 - 1)


def build_tree(x, lo, box_len, ncrit, max_level, periodic):
    """Adaptive octree.  Returns a dict of per-cell arrays (level-major,
    ascending key within a level): level, key, start, count, parent, child
    (8 per cell, -1 if absent), leaf; plus the wrapped positions ``xw``, the
    stable sort permutation ``perm`` and the finest-level keys."""
    xw = T.wrap(x, lo, box_len) if periodic else np.asarray(x, np.float64)
    c = T.leaf_coords(xw, lo, box_len, max_level)
    fine = T.morton(c, max_level)
    perm = np.argsort(fine, kind="stable")
    sk = fine[perm]
    n = len(sk)
    level, key, start, count, parent = [0], [0], [0], [n], [-1]
    frontier = [0]
    for l in range(max_level):
        nxt = []
        for ci in frontier:
            if count[ci] <= ncrit:
                continue
            s0, s1 = start[ci], start[ci] + count[ci]
            pref = sk[s0:s1] >> (3 * (max_level - l - 1))
            for o in range(8):
                ck = (key[ci] << 3) | o
                a = s0 + int(np.searchsorted(pref, ck, side="left"))
                b = s0 + int(np.searchsorted(pref, ck, side="right"))
                if b > a:
                    level.append(l + 1)
                    key.append(ck)
                    start.append(a)
                    count.append(b - a)
                    parent.append(ci)
                    nxt.append(len(level) - 1)
        frontier = nxt
    ncell = len(level)
    level = np.array(level, np.int64)
    count = np.array(count, np.int64)
    parent = np.array(parent, np.int64)
    child = -np.ones((ncell, 8), np.int64)
    for ci in range(1, ncell):
        child[parent[ci], key[ci] & 7] = ci
    leaf = np.all(child < 0, axis=1)
    return {"level": level, "key": np.array(key, np.int64), "start": np.array(start, np.int64), "count": count,
            "parent": parent, "child": child, "leaf": leaf, "xw": xw, "perm": perm, "fine_keys": fine,
            "max_level": max_level, "lo": np.asarray(lo, np.float64), "box_len": float(box_len),
            "periodic": int(periodic)}


def cell_bounds(tree, ci):
    """Integer corner and side of cell ``ci`` on the grid of the finest level."""
    l = int(tree["level"][ci])
    side = 1 << (tree["max_level"] - l)
    c = T.demorton(np.array([tree["key"][ci]]), l)[0]
    return c * side, side


def touching(tree, a, b, s):
    """Do the closed cubes of cells a and b (b shifted by image s) touch?"""
    ca, na = cell_bounds(tree, a)
    cb, nb = cell_bounds(tree, b)
    cb = cb + np.asarray(s, np.int64) * (1 << tree["max_level"])
    return bool(np.all(ca <= cb + nb) and np.all(cb <= ca + na))


def cell_centre(tree, ci):
    l = int(tree["level"][ci])
    w = tree["box_len"] / (1 << l)
    c = T.demorton(np.array([tree["key"][ci]]), l)[0]
    return tree["lo"] + (c + 0.5) * w


def lists(tree):
    """Interaction lists by the dual traversal: dict name -> sorted int64
    array of (target cell, source cell, shift code) rows, names "p2p",
    "m2l", "m2p", "p2l"."""
    out = {"p2p": [], "m2l": [], "m2p": [], "p2l": []}
    lev, leaf, child = tree["level"], tree["leaf"], tree["child"]
    shifts = SHIFTS if tree["periodic"] else [(0, 0, 0)]
    stack = [(0, 0, s) for s in shifts]
    while stack:
        a, b, s = stack.pop()
        la, lb = lev[a], lev[b]
        if not touching(tree, a, b, s) and (la == lb or not leaf[b if la < lb else a]):
            name = "m2l" if la == lb else ("m2p" if la < lb else "p2l")
            out[name].append((a, b, shift_code(s)))
            continue
        if leaf[a] and leaf[b]:
            out["p2p"].append((a, b, shift_code(s)))
            continue
        ka = [c for c in child[a] if c >= 0]
        kb = [c for c in child[b] if c >= 0]
        if la == lb:
            if leaf[a]:
                stack.extend((a, cb, s) for cb in kb)
            elif leaf[b]:
                stack.extend((ca, b, s) for ca in ka)
            else:
                stack.extend((ca, cb, s) for ca in ka for cb in kb)
        elif la < lb:          # a is a coarser leaf, b is split
            stack.extend((a, cb, s) for cb in kb)
        else:                  # b is a coarser leaf, a is split
            stack.extend((ca, b, s) for ca in ka)
    res = {}
    for k, v in out.items():
        arr = np.array(v, np.int64).reshape(-1, 3)
        res[k] = arr[np.lexsort((arr[:, 2], arr[:, 1], arr[:, 0]))] if len(arr) else arr
    return res


def _particles(tree, ci):
    s0 = tree["start"][ci]
    return tree["perm"][s0:s0 + tree["count"][ci]]


def _curl(g):
    """u (P,3) from d_c psi_d = g[:, d, c]."""
    return np.stack([g[:, 2, 1] - g[:, 1, 2], g[:, 0, 2] - g[:, 2, 0], g[:, 1, 0] - g[:, 0, 1]], axis=1)


def _curl_grad(h):
    """J (P,3,3), J[a,b] = d_a u_b, from h[:, d, a, c] = d_a d_c psi_d."""
    J = np.zeros((h.shape[0], 3, 3))
    for a in range(3):
        J[:, a, 0] = h[:, 2, a, 1] - h[:, 1, a, 2]
        J[:, a, 1] = h[:, 0, a, 2] - h[:, 2, a, 0]
        J[:, a, 2] = h[:, 1, a, 0] - h[:, 0, a, 1]
    return J


def _derivs_at_centre(Lp, p):
    """Gradient (P, K, 3) and Hessian (P, K, 3, 3) at its centre of each
    particle's own local expansion Lp[i] (P, K, C): ``local_derivs`` with one
    expansion per point, evaluated at offset 0."""
    P = H.regular_poly(p)
    _, g, h = H.monomial_derivs(np.zeros((1, 3)), p)
    coef = Lp @ P                                  # (P, K, nmono)
    grad = np.real(np.einsum("pkm,am->pka", coef, g[0]))
    hess = np.real(np.einsum("pkm,abm->pkab", coef, h[0]))
    return grad, hess


def fmm(x, alpha, sigma, p, ncrit, max_level, box_lo=(0.0, 0.0, 0.0), box_len=2 * math.pi, periodic=0,
        tree=None, lst=None):
    """u (N,3) and J (N,3,3) of the adaptive FMM, in the caller's order."""
    x = np.asarray(x, np.float64)
    alpha = np.asarray(alpha, np.float64)
    n = len(x)
    lo = np.asarray(box_lo, np.float64)
    tr = tree if tree is not None else build_tree(x, lo, box_len, ncrit, max_level, periodic)
    ls = lst if lst is not None else lists(tr)
    xw = tr["xw"]
    ncell = len(tr["level"])
    C = H.ncoef(p)
    ctr = np.array([cell_centre(tr, ci) for ci in range(ncell)])
    img = lambda code: np.array(code_shift(int(code)), np.float64) * box_len

    # P2M at the leaves, M2M up the tree (children before parents: reverse order)
    M = np.zeros((ncell, 3, C), np.complex128)
    for ci in range(ncell - 1, -1, -1):
        if tr["leaf"][ci]:
            ids = _particles(tr, ci)
            M[ci] = H.p2m(xw[ids] - ctr[ci], alpha[ids], p)
        else:
            for ch in tr["child"][ci]:
                if ch >= 0:
                    M[ci] += M[ch] @ H.m2m_matrix(ctr[ch] - ctr[ci], p).T

    # downward: lattice at the root, then per cell L2L from the parent, M2L, P2L
    L = np.zeros((ncell, 3, C), np.complex128)
    if periodic:
        L[0] = lattice_local(M[0], p, box_len, periodic)
    by_target = {k: {} for k in ls}
    for k, arr in ls.items():
        for t, s_, c in arr:
            by_target[k].setdefault(int(t), []).append((int(s_), int(c)))
    for ci in range(ncell):
        par = tr["parent"][ci]
        if par >= 0:
            L[ci] += L[par] @ H.l2l_matrix(ctr[par] - ctr[ci], p).T
        for src, code in by_target["m2l"].get(ci, []):
            L[ci] += M[src] @ H.m2l_matrix(ctr[src] + img(code) - ctr[ci], p).T
        for src, code in by_target["p2l"].get(ci, []):
            ids = _particles(tr, src)
            ys = xw[ids] + img(code)
            Ts = H.m2l_matrices(ys - ctr[ci], p)
            for j, Tj in zip(ids, Ts):
                mj = H.p2m(np.zeros((1, 3)), alpha[j][None], p)      # point multipole at the source
                L[ci] += mj @ Tj.T

    u = np.zeros((n, 3))
    J = np.zeros((n, 3, 3))
    for ci in np.nonzero(tr["leaf"])[0]:
        ids = _particles(tr, ci)
        g, h = H.local_derivs(L[ci], xw[ids] - ctr[ci], p)
        uf, Jf = _curl(g), _curl_grad(h)
        # M2P: the source multipole's local expansion about each target particle
        for src, code in by_target["m2p"].get(ci, []):
            ds = ctr[src] + img(code) - xw[ids]
            Lp = np.einsum("pij,kj->pki", H.m2l_matrices(ds, p), M[src])    # local about each particle
            g1, h1 = _derivs_at_centre(Lp, p)
            uf += _curl(g1)
            Jf += _curl_grad(h1)
        u[ids] += uf * INV4PI
        J[ids] += Jf * INV4PI
        # P2P with the exact cutoff
        srcs, shifts = [], []
        for src, code in by_target["p2p"].get(ci, []):
            sid = _particles(tr, src)
            srcs.append(sid)
            shifts.append(np.broadcast_to(img(code), (len(sid), 3)))
        sid = np.concatenate(srcs)
        un, Jn = _direct.direct(xw[ids], xw[sid] + np.concatenate(shifts), alpha[sid], sigma, box_len, K=0)
        u[ids] += un
        J[ids] += Jn
    return u, J


def model_direct(x, alpha, sigma, tree, lst):
    """The sum the adaptive FMM converges to as p grows: the exact regularised
    kernel on the pairs of P2P interactions and g = 1 on every other pair of
    the block S_1 (free space: the box itself).  Periodic problems beyond S_1
    (K >= 2) add the lattice images, which this sum leaves out.  Caller
    order."""
    x = np.asarray(x, np.float64)
    alpha = np.asarray(alpha, np.float64)
    xw = tree["xw"]
    L = tree["box_len"]
    n = len(x)
    u = np.zeros((n, 3))
    J = np.zeros((n, 3, 3))
    near = {}
    for t, s_, c in lst["p2p"]:
        near.setdefault((int(t), int(c)), []).append(int(s_))
    leaf_of = np.empty(n, np.int64)
    for ci in np.nonzero(tree["leaf"])[0]:
        leaf_of[_particles(tree, ci)] = ci
    shifts = SHIFTS if tree["periodic"] else [(0, 0, 0)]
    for ci in np.nonzero(tree["leaf"])[0]:
        ids = _particles(tree, ci)
        for s in shifts:
            mask = np.isin(leaf_of, near.get((int(ci), shift_code(s)), []))
            ys = xw + np.array(s, np.float64) * L
            if np.any(mask):
                un, Jn = _direct.direct(xw[ids], ys[mask], alpha[mask], sigma, L, K=0)
                u[ids] += un
                J[ids] += Jn
            if np.any(~mask):
                # cells two apart: the direct sum's far-field model, g = 1
                ct = np.zeros((len(ids), 3), np.int32)
                cs = np.full((int(np.sum(~mask)), 3), 2, np.int32)
                un, Jn = _direct.direct(xw[ids], ys[~mask], alpha[~mask], sigma, L, K=0, cells_t=ct, cells_s=cs,
                                        level=4)
                u[ids] += un
                J[ids] += Jn
    return u, J
