"""Uniform octree by brute force (test infrastructure: the oracle).

The paper builds its tree on the CPU and leaves the details open (Sec. 2.2,
last paragraph).  The readings fixed here are the ones the GPU build must
reproduce bit for bit:

* periodic wrap: s = floor((x - lo) * inv_L), x_w = x - s * L, where
  inv_L = fl(1/L) and each product / difference is rounded on its own (no
  fused multiply-add);
* leaf coordinate: c = floor((x_w - lo) * inv_w) clamped to [0, 2^l - 1],
  inv_w = 2^l * inv_L (exact scaling);
* Morton key: bit b of c_x, c_y, c_z goes to key bits 3b, 3b+1, 3b+2;
* particles are ordered by key with ties kept in input order (stable sort);
* leaf ranges are dense over all 8^l keys: start[k] = first sorted index
  with key >= k;
* near field: the 27 leaves at Chebyshev distance <= 1 (periodic: modulo
  2^l with the image shift recorded);
* interaction list of a cell at level l >= 2 (free) or l >= 1 (periodic):
  children of the parent's 27 neighbours that are not adjacent to the cell,
  listed by offset d = source - target in (dz, dy, dx) lexicographic order.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def wrap(x, lo, box_len):
    x = np.asarray(x, np.float64)
    lo = np.asarray(lo, np.float64)
    inv_l = 1.0 / float(box_len)
    s = np.floor((x - lo) * inv_l)
    return x - s * float(box_len)


def leaf_coords(xw, lo, box_len, level):
    lo = np.asarray(lo, np.float64)
    inv_w = math.ldexp(1.0 / float(box_len), level)
    c = np.floor((np.asarray(xw, np.float64) - lo) * inv_w)
    return np.clip(c, 0, (1 << level) - 1).astype(np.int64)


def morton(c, level):
    """Key of integer coordinates ``c`` (n, 3), one bit at a time."""
    c = np.asarray(c, np.int64)
    key = np.zeros(c.shape[0], np.int64)
    for b in range(level):
        for d in range(3):
            key |= ((c[:, d] >> b) & 1) << (3 * b + d)
    return key


def demorton(key, level):
    key = np.asarray(key, np.int64)
    c = np.zeros((key.shape[0], 3), np.int64)
    for b in range(level):
        for d in range(3):
            c[:, d] |= ((key >> (3 * b + d)) & 1) << b
    return c


def build(x, lo, box_len, level, periodic):
    """Keys, stable sort permutation, leaf start/count, wrapped positions."""
    xw = wrap(x, lo, box_len) if periodic else np.asarray(x, np.float64)
    c = leaf_coords(xw, lo, box_len, level)
    keys = morton(c, level)
    perm = np.argsort(keys, kind="stable")
    sk = keys[perm]
    nleaf = 1 << (3 * level)
    start = np.searchsorted(sk, np.arange(nleaf), side="left")
    end = np.searchsorted(sk, np.arange(nleaf), side="right")
    return {"xw": xw, "coords": c, "keys": keys, "perm": perm,
            "start": start.astype(np.int64), "count": (end - start).astype(np.int64)}


def neighbours(coord, level, periodic):
    """The 27 (or fewer, free space) near leaves: (key, image shift) pairs."""
    side = 1 << level
    out = []
    for dz, dy, dx in itertools.product((-1, 0, 1), repeat=3):
        d = np.array([dx, dy, dz])
        s = np.asarray(coord) + d
        if periodic:
            img = np.floor_divide(s, side)
            s = s - img * side
        else:
            if np.any(s < 0) or np.any(s >= side):
                continue
            img = np.zeros(3, np.int64)
        out.append((int(morton(s[None], level)[0]), tuple(int(v) for v in img)))
    return out


def offsets_for_octant(octant):
    """Offsets d (source - target, in cells) of the M2L list of a cell whose
    coordinate parities are given by ``octant`` (bit 0 = x, 1 = y, 2 = z):
    children of the parent's neighbours that are not adjacent."""
    par = [(octant >> d) & 1 for d in range(3)]
    rng = []
    for d in range(3):
        # children of parent offsets -1..1: cells 2(P-1) .. 2(P+1)+1 relative to 2P + par
        rng.append(range(-2 - par[d], 4 - par[d]))
    out = []
    for dz in rng[2]:
        for dy in rng[1]:
            for dx in rng[0]:
                if max(abs(dx), abs(dy), abs(dz)) >= 2:
                    out.append((dx, dy, dz))
    return out


def all_offsets():
    s = set()
    for o in range(8):
        s.update(offsets_for_octant(o))
    return sorted(s, key=lambda d: (d[2], d[1], d[0]))


def interaction_list(key, level, periodic):
    """Brute-force M2L list of one cell: [(src_key, (dx,dy,dz), image)]."""
    c = demorton(np.array([key]), level)[0]
    side = 1 << level
    parent = c >> 1
    out = []
    for pz, py, px in itertools.product((-1, 0, 1), repeat=3):
        pc = parent + np.array([px, py, pz])
        for oz, oy, ox in itertools.product((0, 1), repeat=3):
            s = 2 * pc + np.array([ox, oy, oz])
            d = s - c
            if max(abs(d)) <= 1:
                continue
            if periodic:
                img = np.floor_divide(s, side)
                sw = s - img * side
            else:
                if np.any(s < 0) or np.any(s >= side):
                    continue
                img = np.zeros(3, np.int64)
                sw = s
            out.append((int(morton(sw[None], level)[0]), tuple(int(v) for v in d),
                        tuple(int(v) for v in img)))
    out.sort(key=lambda t: (t[1][2], t[1][1], t[1][0]))
    return out
