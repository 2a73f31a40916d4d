"""Gaussian smoothing sums and RBF interpolation (test infrastructure: the oracle).

Definitions (Sec. 2):

* the vorticity carried by the particles is the superposition of Gaussian
  bases, omega(x) = sum_j gamma_j zeta_sigma(x - x_j) (the smoothing-function
  equation), with zeta_sigma(r) = (2 pi sigma^2)^(-3/2) exp(-r^2 / (2 sigma^2))
  (the Gaussian equation);
* the sum is taken over neighbouring particles only, through the neighbour
  list of the FMM tree: for a target in leaf c, the sources in the 27 leaves
  c + d, d in {-1, 0, 1}^3, each counted once per d.  Periodic: the leaf index
  is taken modulo 2^level and the source shifted by the image n L, n = floor
  ((c + d) / 2^level); free space: leaves outside the domain are skipped.
  Positions of a periodic problem are wrapped into the box first (tree.wrap);
* RBF interpolation solves that linear system, A gamma = omega with
  A_ij = sum over the neighbour-list images of zeta_sigma(x_i - x_j - n L),
  for gamma given omega at the particle positions.  The paper iterates with
  GMRES from the initial guess gamma = omega h^3; here the system is solved
  directly (dense LU), the reference the iterative GPU solve converges to.

Everything is FP64 and meant for small N (the matrix is dense).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from . import tree as T


def zeta(r2, sigma):
    """Gaussian basis at squared distance r2 (the Gaussian equation)."""
    return np.exp(-0.5 * r2 / (sigma * sigma)) / (2.0 * math.pi * sigma * sigma) ** 1.5


def _leaves(x, level, box_len):
    """Leaf coordinates of every particle, the particles sorted by leaf index
    (cx + side (cy + side cz)) and each leaf's range in that order."""
    side = 1 << level
    c = T.leaf_coords(x, (0.0, 0.0, 0.0), box_len, level)
    key = c[:, 0] + side * (c[:, 1] + side * c[:, 2])
    order = np.argsort(key, kind="stable")
    bounds = np.searchsorted(key[order], np.arange(side ** 3 + 1))
    return c, order, bounds


def _slots(ck, side, periodic):
    """The 27 neighbour slots d of leaf ck: (source leaf index, image n) for
    each slot that exists (free space drops leaves outside the domain)."""
    for d in itertools.product((-1, 0, 1), repeat=3):
        cs = [ck[a] + d[a] for a in range(3)]
        if periodic:
            n = np.array([math.floor(v / side) for v in cs], np.float64)
            cs = [v % side for v in cs]
        else:
            if any(v < 0 or v >= side for v in cs):
                continue
            n = np.zeros(3)
        yield cs[0] + side * (cs[1] + side * cs[2]), n


def _neighbour_pairs(x, level, box_len, periodic):
    """Yields (targets, sources, shift) per (target leaf, d): particle index
    arrays and the image shift added to the source positions."""
    side = 1 << level
    _, order, bounds = _leaves(x, level, box_len)
    members = lambda k: order[bounds[k]:bounds[k + 1]]
    for ck in itertools.product(range(side), repeat=3):
        tgt = members(ck[0] + side * (ck[1] + side * ck[2]))
        if tgt.size == 0:
            continue
        for k, n in _slots(ck, side, periodic):
            src = members(k)
            if src.size:
                yield tgt, src, n * box_len


def gauss_matrix(x, sigma, level, box_len=2 * math.pi, periodic=0):
    """Dense A (n, n): A[i, j] = sum over neighbour-list images of zeta(x_i - x_j - shift)."""
    x = np.asarray(x, np.float64)
    if periodic:
        x = T.wrap(x, (0.0, 0.0, 0.0), box_len)
    A = np.zeros((len(x), len(x)))
    for tgt, src, shift in _neighbour_pairs(x, level, box_len, periodic):
        r = x[tgt][:, None, :] - (x[src][None, :, :] + shift)
        A[np.ix_(tgt, src)] += zeta(np.sum(r * r, axis=2), sigma)
    return A


def gauss_sum(x, gamma, sigma, level, box_len=2 * math.pi, periodic=0):
    """omega (n, 3) = A gamma."""
    return gauss_matrix(x, sigma, level, box_len, periodic) @ np.asarray(gamma, np.float64)


def rbf_solve(x, omega, sigma, level, box_len=2 * math.pi, periodic=0):
    """gamma (n, 3) with A gamma = omega, by a dense solve."""
    A = gauss_matrix(x, sigma, level, box_len, periodic)
    return np.linalg.solve(A, np.asarray(omega, np.float64))


def gauss_eval(y, x, gamma, sigma, level, box_len=2 * math.pi, periodic=0):
    """The vorticity the particles (x, gamma) carry, at points y (m, 3): for a
    point in leaf c, the sources in the 27 leaves c + d as in the matrix (the
    smoothing-function equation at arbitrary points, neighbour list only)."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    gamma = np.asarray(gamma, np.float64)
    if periodic:
        x = T.wrap(x, (0.0, 0.0, 0.0), box_len)
        y = T.wrap(y, (0.0, 0.0, 0.0), box_len)
    side = 1 << level
    _, order, bounds = _leaves(x, level, box_len)
    cy = T.leaf_coords(y, (0.0, 0.0, 0.0), box_len, level)
    out = np.zeros((len(y), 3))
    for i in range(len(y)):
        for k, n in _slots(tuple(int(v) for v in cy[i]), side, periodic):
            src = order[bounds[k]:bounds[k + 1]]
            r = y[i][None, :] - (x[src] + n * box_len)
            out[i] = out[i] + zeta(np.sum(r * r, axis=1), sigma) @ gamma[src]
    return out


def gauss_sum_at(x, gamma, sigma, level, targets, box_len=2 * math.pi, periodic=0):
    """Rows `targets` of A gamma (len(targets), 3): the same neighbour-list
    sum evaluated at the chosen particles, for inputs too large for the
    dense matrix."""
    return gauss_eval(np.asarray(x, np.float64)[np.asarray(targets)], x, gamma, sigma, level, box_len, periodic)


def lattice_sites(ng, box_len=2 * math.pi):
    """Cell centres (i + 1/2) h of the ng^3 lattice on the box, h = box_len / ng,
    site (ix ng + iy) ng + iz (x index slowest)."""
    h = box_len / ng
    i = np.arange(ng ** 3)
    ix, iy, iz = i // (ng * ng), (i // ng) % ng, i % ng
    return (np.stack([ix, iy, iz], axis=1) + 0.5) * h


def reinit(x, gamma, sigma, ng, sigma0, level, box_len=2 * math.pi, periodic=0):
    """Reinitialisation onto the lattice (the reinitialisation paragraph of
    Sec. 2.2): the vorticity the particles carry with core sigma, taken at the
    ng^3 lattice sites, becomes the right-hand side of the interpolation with
    the smaller core sigma0 on the lattice.  Returns (sites, new strengths,
    vorticity at the sites)."""
    y = lattice_sites(ng, box_len)
    om = gauss_eval(y, x, gamma, sigma, level, box_len, periodic)
    return y, rbf_solve(y, om, sigma0, level, box_len, periodic), om
