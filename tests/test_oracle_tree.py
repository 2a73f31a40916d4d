"""Pins of the oracle's octree against brute force (no GPU)."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

import workloads as W
from oracle import tree as T

L = 2 * math.pi


def _key_bits(c, level):
    bits = ""
    for b in reversed(range(level)):
        for d in (2, 1, 0):
            bits += str((int(c[d]) >> b) & 1)
    return int(bits, 2) if bits else 0


@pytest.mark.parametrize("level", [0, 1, 3, 6, 10])
def test_morton_matches_bit_string(level):
    rng = np.random.default_rng(level)
    c = rng.integers(0, 1 << level, size=(200, 3)) if level else np.zeros((5, 3), np.int64)
    k = T.morton(c, level)
    assert [int(v) for v in k] == [_key_bits(row, level) for row in c]
    assert np.array_equal(T.demorton(k, level), c)


def test_leaf_coordinate_is_exact_interval_membership():
    x, _ = W.random_particles(3000, 4)
    level = 5
    c = T.leaf_coords(x, (0, 0, 0), L, level)
    fl_l = Fraction(L)
    side = 1 << level
    for i in range(0, 3000, 7):
        for d in range(3):
            xv = Fraction(float(x[i, d]))
            lo_f = Fraction(int(c[i, d])) * fl_l / side
            hi_f = Fraction(int(c[i, d]) + 1) * fl_l / side
            # away from faces the rounded floor equals exact membership
            if min(abs(xv - lo_f), abs(xv - hi_f)) > Fraction(1, 10 ** 12):
                assert lo_f <= xv < hi_f


def test_wrap_and_faces():
    lo = np.array([0.0, 0.0, 0.0])
    pts = np.array([[0.0, L, -1e-300],
                    [np.nextafter(L, 0), -L, 3 * L + 0.5],
                    [-0.25, 1e-17, np.nextafter(0.0, -1)]])
    xw = T.wrap(pts, lo, L)
    # wrapped values land in [lo, lo + L] up to a rounding at either face
    assert np.all(xw >= -1e-300) and np.all(xw <= L)
    assert np.allclose(np.round((pts - xw) / L), (pts - xw) / L, rtol=0, atol=1e-12)
    c = T.leaf_coords(xw, lo, L, 4)
    assert np.all((c >= 0) & (c < 16))
    assert xw[2, 0] == L - 0.25 and c[2, 0] == 15
    assert abs(xw[1, 2] - 0.5) < 1e-14
    # a face value rounding to lo + L is clamped into the top cell
    top = T.leaf_coords(np.array([[L, L, L]]), lo, L, 4)
    assert np.all(top == 15)


def test_sort_is_stable_and_ranges_are_dense():
    x, _ = W.random_particles(4000, 6)
    level = 3
    tr = T.build(x, (0, 0, 0), L, level, periodic=1)
    keys = tr["keys"]
    ref = sorted(range(len(keys)), key=lambda i: int(keys[i]))
    assert list(tr["perm"]) == ref
    counts = np.zeros(8 ** level, np.int64)
    for k in keys:
        counts[k] += 1
    assert np.array_equal(tr["count"], counts)
    assert np.array_equal(tr["start"], np.concatenate([[0], np.cumsum(counts)[:-1]]))


def test_offset_tables():
    offs = T.all_offsets()
    assert len(offs) == 316
    for o in range(8):
        lst = T.offsets_for_octant(o)
        assert len(lst) == 189 and len(set(lst)) == 189
        assert lst == sorted(lst, key=lambda d: (d[2], d[1], d[0]))
    hist = {}
    for d in offs:
        k = sum(abs(v) == 3 for v in d)
        hist[k] = hist.get(k, 0) + 1
    assert hist == {0: 98, 1: 150, 2: 60, 3: 8}


@pytest.mark.parametrize("periodic,level", [(0, 3), (1, 2), (1, 1)])
def test_lists_cover_every_pair_once(periodic, level):
    """Every (target leaf, source leaf + image in S_1) pair is handled exactly
    once: by P2P at the leaves or by M2L at one ancestor level."""
    side = 1 << level
    lmin = 1 if periodic else 2
    lists = {}
    for l in range(lmin, level + 1):
        for key in range(8 ** l):
            for sk, d, img in T.interaction_list(key, l, periodic):
                lists.setdefault((l, key), set()).add(d)
    srcs = (range(-side, 2 * side) if periodic else range(side))
    step = 5 if 8 ** level > 100 else 1   # a spread sample of target leaves
    for tkey in range(0, 8 ** level, step):
        tc = T.demorton(np.array([tkey]), level)[0]
        near = {tuple(int(v) for v in (T.demorton(np.array([nk]), level)[0] + np.array(img) * side))
                for nk, img in T.neighbours(tc, level, periodic)}
        for sc in itertools.product(srcs, repeat=3):
            sc = np.array(sc)
            hits = int(tuple(int(v) for v in sc) in near)
            for l in range(lmin, level + 1):
                sh = level - l
                ta = tc >> sh
                sa = np.floor_divide(sc, 1 << sh)
                d = tuple(int(v) for v in (sa - ta))
                tk = int(T.morton(ta[None], l)[0])
                if d in lists.get((l, tk), ()):
                    hits += 1
            assert hits == 1, (tkey, sc)
