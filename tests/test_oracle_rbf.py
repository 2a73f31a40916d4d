"""Pins of the oracle's Gaussian sums and RBF interpolation (no GPU).

* The Gaussian basis has unit mass: its samples on a fine lattice times the
  cell volume sum to 1 (Poisson summation: the error is exp(-2 pi^2 sigma^2/h^2)),
  which fixes the (2 pi sigma^2)^(-3/2) prefactor and the 2 sigma^2 in the exponent.
* A Fourier mode carried by a lattice (gamma_j = omega(x_j) h^3, sigma = h) is
  reproduced damped by exp(-sigma^2 k^2 / 2) when the sum covers every image
  within reach of the Gaussian (periodic, leaf level 1: the 27 neighbour
  leaves span one and a half boxes, 8 sigma beyond any target); the aliased
  modes k + 2 pi m / h add at most sum_i 2 exp(-2 pi^2 + 2 pi h |k_i|) (Poisson
  summation), about 2e-7 at 16^3 with |k_i| = 1.
* Interpolation inverts that: the strengths solving A gamma = omega for the
  mode are omega(x_j) h^3 exp(+sigma^2 k^2 / 2) to the same alias level.
* The matrix is symmetric and positive definite; the neighbour-list
  truncation (leaf level 2) drops only pairs farther apart than a leaf width.
"""
import math

import numpy as np

import workloads as W
from oracle import rbf as R

L = 2 * math.pi


def test_gaussian_has_unit_mass():
    sigma = 0.3
    h = sigma / 4
    g = np.arange(-40, 41) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    mass = np.sum(R.zeta(X * X + Y * Y + Z * Z, sigma)) * h ** 3
    assert abs(mass - 1.0) < 1e-12


def _mode(ng, k):
    x = W.lattice(ng)
    h = L / ng
    phase = x @ np.asarray(k, np.float64)
    om = np.stack([np.cos(phase), np.sin(phase), np.cos(phase + 0.3)], axis=1)
    return x, om, h


def _alias_bound(h, k):
    return sum(2 * math.exp(-2 * math.pi ** 2 + 2 * math.pi * h * abs(ki)) for ki in k)


def test_lattice_reproduces_a_fourier_mode():
    k = np.array([1.0, -1.0, 1.0])
    x, om, h = _mode(16, k)
    sigma = h
    got = R.gauss_sum(x, om * h ** 3, sigma, level=1, periodic=1)
    want = om * math.exp(-0.5 * sigma * sigma * (k @ k))
    assert np.abs(got - want).max() < 2 * _alias_bound(h, k)


def test_interpolation_inverts_the_smoothing():
    k = np.array([0.0, 1.0, -1.0])
    x, om, h = _mode(16, k)
    sigma = h
    gam = R.rbf_solve(x, om, sigma, level=1, periodic=1)
    want = om * h ** 3 * math.exp(0.5 * sigma * sigma * (k @ k))
    assert np.abs(gam - want).max() < 2 * _alias_bound(h, k) * np.abs(want).max()


def test_matrix_is_symmetric_positive_definite_and_local():
    x, _ = W.random_particles(600, 5)
    sigma = 0.4
    for periodic in (0, 1):
        A = R.gauss_matrix(x, sigma, level=2, periodic=periodic)
        assert np.allclose(A, A.T, rtol=0, atol=1e-15 * np.abs(A).max())
        assert np.linalg.eigvalsh(A).min() > 0
        # pairs kept are within the neighbour leaves: farther than 2 leaf widths never appear
        xw = x if not periodic else np.mod(x, L)
        d = xw[:, None, :] - xw[None, :, :]
        if periodic:
            d -= L * np.round(d / L)
        far = np.max(np.abs(d), axis=2) > 2 * L / 4
        assert np.all(A[far] == 0)


def test_rows_at_targets_match_the_matrix():
    x, g = W.random_particles(700, 9)
    for periodic, level in ((0, 2), (1, 2), (1, 1)):
        full = R.gauss_sum(x, g, 0.35, level=level, periodic=periodic)
        t = np.array([0, 5, 133, 699])
        rows = R.gauss_sum_at(x, g, 0.35, level, t, periodic=periodic)
        assert np.allclose(rows, full[t], rtol=0, atol=1e-13 * np.abs(full).max())


def test_smoothed_mode_at_points_off_the_lattice():
    """Poisson summation at any point y: sum_j omega(x_j) h^3 zeta(y - x_j) =
    omega(y) exp(-sigma^2 k^2 / 2) up to the same alias bound."""
    k = np.array([1.0, 0.0, -1.0])
    x, om, h = _mode(16, k)
    sigma = h
    rng = np.random.default_rng(3)
    y = rng.uniform(0, L, size=(40, 3))
    got = R.gauss_eval(y, x, om * h ** 3, sigma, level=1, periodic=1)
    phase = y @ k
    want = np.stack([np.cos(phase), np.sin(phase), np.cos(phase + 0.3)], axis=1) * math.exp(-0.5 * sigma * sigma * (k @ k))
    assert np.abs(got - want).max() < 2 * _alias_bound(h, k)


def test_lattice_sites_and_reinit_of_a_lattice_is_the_identity():
    y = R.lattice_sites(4, L)
    assert np.array_equal(y[1], np.array([0.5, 0.5, 1.5]) * L / 4)
    assert np.array_equal(y[4 * 4], np.array([1.5, 0.5, 0.5]) * L / 4)
    x = R.lattice_sites(8, L)
    h = L / 8
    g = np.random.default_rng(4).standard_normal((512, 3)) * h ** 3
    y, g2, om = R.reinit(x, g, h, 8, h, level=1, periodic=1)
    assert np.array_equal(y, x)
    assert np.allclose(om, R.gauss_sum(x, g, h, 1, periodic=1), rtol=0, atol=1e-14 * np.abs(om).max())
    assert np.abs(g2 - g).max() < 1e-9 * np.abs(g).max()
