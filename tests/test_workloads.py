"""The seeded input generators (no GPU), checked against what their recipes
promise: a cell-centred lattice, zero net vorticity and a solenoidal field
for the random workloads, exact leaf populations, and clustered sets that
are far from uniform but keep a uniform background."""
import math

import numpy as np
import pytest

import workloads as W


def test_lattice_is_cell_centred():
    ng = 6
    x = W.lattice(ng)
    h = W.TWO_PI / ng
    assert x.shape == (ng ** 3, 3)
    frac = x / h - 0.5
    assert np.abs(frac - np.rint(frac)).max() < 1e-12
    assert x.min() == pytest.approx(0.5 * h) and x.max() == pytest.approx(W.TWO_PI - 0.5 * h)
    assert len(np.unique(np.rint(x / h - 0.5).astype(int), axis=0)) == ng ** 3


@pytest.mark.parametrize("ng,k0", [(16, 4.0), (24, 8.0)])
def test_random_field_has_no_net_vorticity_and_no_divergence(ng, k0):
    x, a = W.random_field(ng, k0, 3)
    h = W.TWO_PI / ng
    assert x.shape == a.shape == (ng ** 3, 3)
    assert np.abs(a.sum(axis=0)).max() < 1e-12 * np.abs(a).sum()
    # spectral divergence of omega on the lattice (the half-cell shift is a common phase)
    w = (a / h ** 3).T.reshape(3, ng, ng, ng)
    wh = np.fft.rfftn(w, axes=(1, 2, 3))
    k = np.fft.fftfreq(ng, d=1.0 / ng)
    kr = np.fft.rfftfreq(ng, d=1.0 / ng)
    kx, ky, kz = np.meshgrid(k, k, kr, indexing="ij")
    div = kx * wh[0] + ky * wh[1] + kz * wh[2]
    assert np.abs(div).max() < 1e-10 * np.abs(wh).max() * ng


def test_leaf_counts_are_exact():
    level = 2
    side = 1 << level
    counts = np.random.default_rng(5).integers(0, 7, size=side ** 3)
    x, a = W.particles_with_leaf_counts(counts, level, 9)
    c = np.floor(x / (W.TWO_PI / side)).astype(int)
    leaf = c[:, 0] + side * (c[:, 1] + side * c[:, 2])
    assert np.array_equal(np.bincount(leaf, minlength=side ** 3), counts)
    assert np.abs(a.sum(axis=0)).max() < 1e-12 * max(1.0, np.abs(a).sum())


def test_clustered_particles_are_far_from_uniform():
    n = 1 << 15
    x, a = W.clustered_particles(n, seed=41)
    assert x.shape == (n, 3) and np.all(x >= 0.0) and np.all(x < W.TWO_PI)
    assert np.abs(a.sum(axis=0)).max() < 1e-9
    side = 8
    c = np.floor(x / (W.TWO_PI / side)).astype(int)
    occ = np.bincount(c[:, 0] + side * (c[:, 1] + side * c[:, 2]), minlength=side ** 3)
    assert occ.max() > 20 * n / side ** 3          # dense clusters
    assert np.mean(occ == 0) < 0.05                # the uniform tenth reaches almost every cell
