"""Pins of the direct-sum oracle against closed forms (no GPU).

* A single Gaussian blob (eqs. 3-4) of strength alpha has the vector
  potential alpha * phi(r) with phi the textbook potential of a unit
  Gaussian charge, phi = erf(r / (sqrt 2 sigma)) / (4 pi r); so
  u = grad phi x alpha and J[a][b] = eps_bcd alpha_d d_a d_c phi.  phi is
  differentiated in 40-digit arithmetic, so these tests fix the cutoff
  (eq. 6), the sign of eq. 5, the gradient and the small-r series at once.
* The blob vorticity itself: laplacian(phi) = -zeta_sigma (eq. 4).
* The self term: curl u at a blob's own centre is (2/3) zeta(0) alpha.
* Periodic image sums approach the Taylor-Green closed form
  exp(-3 sigma^2 / 2) u_TG as the cubic image block grows.
"""
import math

import mpmath as mp
import numpy as np
import pytest

import workloads as W
from oracle import direct as D
from oracle import spectral as S

mp.mp.dps = 40


def _phi(r, sigma):
    return mp.erf(r / (mp.sqrt(2) * sigma)) / (4 * mp.pi * r)


def _blob_closed_form(x, alpha, sigma):
    r = mp.sqrt(sum(mp.mpf(float(v)) ** 2 for v in x))
    d1 = mp.diff(lambda t: _phi(t, sigma), r)
    d2 = mp.diff(lambda t: _phi(t, sigma), r, 2)
    rh = np.array([float(mp.mpf(float(v)) / r) for v in x])
    grad = float(d1) * rh
    u = np.cross(grad, alpha)
    hess = float(d2) * np.outer(rh, rh) + float(d1 / r) * (np.eye(3) - np.outer(rh, rh))
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1.0
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1.0
    J = np.einsum("bcd,d,ac->ab", eps, alpha, hess)
    return u, J


@pytest.mark.parametrize("rho", [1e-3, 0.05, 0.2499, 0.2501, 0.7, 1.0, 2.0, 4.0, 7.5, 20.0])
def test_single_blob_matches_gaussian_potential(rho):
    sigma = 0.3
    alpha = np.array([0.3, -1.1, 0.7])
    direction = np.array([0.48, -0.6, 0.64])
    x = direction / np.linalg.norm(direction) * rho * sigma
    u, J = D.direct(x[None], np.zeros((1, 3)), alpha[None], sigma)
    ue, Je = _blob_closed_form(x, alpha, sigma)
    assert np.allclose(u[0], ue, rtol=0, atol=1e-13 * np.abs(ue).max())
    assert np.allclose(J[0], Je, rtol=0, atol=1e-12 * np.abs(Je).max())
    if rho >= 0.5:   # the NumPy twin has no small-r series
        un, Jn = D.direct_numpy(x[None], np.zeros((1, 3)), alpha[None], sigma)
        assert np.allclose(un[0], ue, rtol=0, atol=1e-12 * np.abs(ue).max())


@pytest.mark.parametrize("r", [0.05, 0.3, 1.0, 2.5])
def test_gaussian_potential_is_blob_vorticity(r):
    sigma = mp.mpf("0.4")
    lap = mp.diff(lambda t: _phi(t, sigma), r, 2) + 2 * mp.diff(lambda t: _phi(t, sigma), r) / r
    zeta = (2 * mp.pi * sigma ** 2) ** mp.mpf(-1.5) * mp.exp(-mp.mpf(r) ** 2 / (2 * sigma ** 2))
    assert abs(float(lap + zeta)) < 1e-25


def test_self_vorticity_closed_form():
    sigma = 0.37
    alpha = np.array([[0.2, -0.5, 1.3]])
    _, J = D.direct(np.zeros((1, 3)), np.zeros((1, 3)), alpha, sigma)
    curl = np.array([J[0, 1, 2] - J[0, 2, 1], J[0, 2, 0] - J[0, 0, 2], J[0, 0, 1] - J[0, 1, 0]])
    zeta0 = (2 * math.pi * sigma * sigma) ** -1.5
    assert np.allclose(curl, 2.0 / 3.0 * zeta0 * alpha[0], rtol=1e-14, atol=0)


def test_gradient_is_traceless_and_matches_fd():
    x, a = W.random_particles(60, 11, box_len=1.0)
    sigma = 0.12
    u, J = D.direct(x, x, a, sigma)
    tr = np.trace(J, axis1=1, axis2=2)
    assert np.abs(tr).max() < 1e-13 * np.abs(J).max()
    h = 1e-4
    xt = x[:6] + 0.01   # off the sources
    _, J0 = D.direct(xt, x, a, sigma)
    for ax in range(3):
        e = np.zeros(3)
        e[ax] = h
        f = lambda s: D.direct(xt + s * e, x, a, sigma)[0]
        fd = (8 * (f(1) - f(-1)) - (f(2) - f(-2))) / (12 * h)
        assert np.allclose(fd, J0[:, ax, :], rtol=0, atol=1e-9 * np.abs(J0).max())


def test_c_and_numpy_direct_agree():
    x, a = W.random_particles(90, 5, box_len=1.0)
    for K in (0, 1):
        u, J = D.direct(x, x, a, 0.1, box_len=1.0, K=K)
        u2, J2 = D.direct_numpy(x, x, a, 0.1, box_len=1.0, K=K)
        assert np.abs(u - u2).max() < 1e-13 * np.abs(u).max()
        assert np.abs(J - J2).max() < 1e-13 * np.abs(J).max()


def test_transpose_stretching_conserves_total_vorticity():
    x, a = W.random_particles(200, 8, box_len=1.0)
    _, J = D.direct(x, x, a, 0.08)
    tot = D.stretching(J, a, "transpose").sum(axis=0)
    scale = np.abs(D.stretching(J, a, "transpose")).sum()
    assert np.abs(tot).max() < 1e-14 * scale
    # the classic form (alpha . grad) u is not conservative
    cl = D.stretching(J, a, "classic").sum(axis=0)
    assert np.abs(cl).max() > 1e-3 * np.abs(D.stretching(J, a, "classic")).sum()


def test_linearity_and_translation_invariance():
    x, a = W.random_particles(50, 9, box_len=1.0)
    u, J = D.direct(x, x, a, 0.1)
    u2, J2 = D.direct(x + 3.25, x + 3.25, -2.0 * a, 0.1)
    assert np.allclose(u2, -2.0 * u, rtol=0, atol=1e-12 * np.abs(u).max())
    assert np.allclose(J2, -2.0 * J, rtol=0, atol=1e-12 * np.abs(J).max())


def test_periodic_images_approach_taylor_green():
    ng = 8
    h = 2 * math.pi / ng
    x = W.lattice(ng)
    a = W.taylor_green_vorticity(x) * h ** 3
    exact = math.exp(-1.5 * h * h) * W.taylor_green_velocity(x)
    errs = []
    for K in (1, 2):
        u, _ = D.direct(x, x, a, h, K=K)
        u -= u.mean(axis=0)
        errs.append(np.linalg.norm(u - exact) / np.linalg.norm(exact))
    assert errs[0] < 2e-3
    assert errs[1] < 2e-5
    assert errs[1] < errs[0] / 50


def test_spectral_oracle_matches_taylor_green():
    ng = 16
    h = 2 * math.pi / ng
    x = W.lattice(ng)
    a = W.taylor_green_vorticity(x) * h ** 3
    u, J = S.lattice_velocity(a, ng, h)
    exact = math.exp(-1.5 * h * h) * W.taylor_green_velocity(x)
    # the lattice sampling adds alias modes k + 16 a, |k + 16 a|^2 >= 227,
    # damped by exp(-sigma^2 * 227 / 2) ~ 2.5e-8 and 1/|k|: ~5e-9 in all
    assert np.linalg.norm(u - exact) / np.linalg.norm(exact) < 1e-8
    assert np.abs(np.trace(J, axis1=1, axis2=2)).max() < 1e-12 * np.abs(J).max()


def test_image_sums_approach_spectral_mean_removed():
    # A random field has a non-zero dipole moment per box; the cubic image
    # block then misses a shape term that falls off like (L / R_K)^2, R_K the
    # block's half-width, on top of the uniform offset removed with the mean.
    ng = 8
    x, a = W.random_field(ng, 2.0, seed=3)
    h = 2 * math.pi / ng
    us, Js = S.lattice_velocity(a, ng, h)
    eu, eJ = [], []
    for K in (1, 2):
        ud, Jd = D.direct(x, x, a, h, K=K)
        ud -= ud.mean(axis=0)
        eu.append(np.linalg.norm(ud - us) / np.linalg.norm(us))
        eJ.append(np.linalg.norm(Jd - Js) / np.linalg.norm(Js))
    assert eu[1] < 5e-3 and eJ[1] < 2e-3
    assert eu[1] < eu[0] / 6 and eJ[1] < eJ[0] / 6
