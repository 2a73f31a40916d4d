"""Seeded synthetic particle fields for the regularised Biot-Savart FMM.

This module only draws inputs. It holds no part of the velocity / stretching
arithmetic, so both the CPU oracle (tests) and the GPU path (tests, bench,
smoke) can take their inputs from it.

Fields follow the paper's set-up (Sec. 4.1 calculation conditions, Sec. 4.2
initial condition, eq. 16):

* particles sit at the centres of the cells of an ``ng^3`` lattice on the
  periodic cube ``[0, 2*pi)^3`` (the paper's cube ``[-pi, pi]^3`` shifted; the
  translation changes nothing), spacing ``h = 2*pi/ng`` and core ``sigma = h``
  (overlap ratio ``h/sigma = 1``);
* strengths are ``alpha = omega(x) * h^3`` (the initial guess of the RBF
  solver in Sec. 5.4, used here in place of the RBF solve);
* the vorticity is either the Taylor-Green field (a closed form used for pins)
  or a random-phase solenoidal field with energy spectrum
  ``E(k) ~ k^4 exp(-2 k^2 / k0^2)`` (eq. 16), normalised to ``u' = 1``.

Everything is float64 and seeded with ``numpy.random.default_rng(seed)``.
Arrays are returned particle-major, shape ``(N, 3)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclass(frozen=True)
class Workload:
    """One named input configuration (sizes follow the paper's N=256^3 run)."""
    name: str
    ng: int                 # lattice points per side; N = ng^3
    p: int                  # expansion order (degrees 0..p)
    level: int              # leaf level of the uniform octree
    periodic: int           # 0 = free space; K >= 1: 3^K images per side
    field: str              # "taylor_green" or "random"
    k0: float = 4.0         # spectrum peak wavenumber (random field)
    jitter: float = 0.0     # uniform jitter, as a fraction of h
    seed: int = 0
    box_lo: tuple = (0.0, 0.0, 0.0)
    box_len: float = TWO_PI

    @property
    def n(self) -> int:
        return self.ng ** 3

    @property
    def h(self) -> float:
        return self.box_len / self.ng

    @property
    def sigma(self) -> float:
        return self.h


# Free-space Taylor-Green blobs (16^3, jittered), periodic random fields at
# 32^3 / 128^3 / 256^3, and the 64^3 field used for gradients.
WORKLOADS = {
    "tg16_free": Workload("tg16_free", 16, 6, 2, 0, "taylor_green", jitter=0.1, seed=1),
    "rand32_periodic": Workload("rand32_periodic", 32, 8, 3, 3, "random", k0=4.0, seed=2),
    "rand128_periodic": Workload("rand128_periodic", 128, 10, 5, 3, "random", k0=8.0, seed=3),
    "rand256_periodic": Workload("rand256_periodic", 256, 10, 6, 3, "random", k0=8.0, seed=4),
    "rand64_periodic": Workload("rand64_periodic", 64, 8, 4, 3, "random", k0=8.0, seed=5),
    "rand16_k1": Workload("rand16_k1", 16, 8, 2, 1, "random", k0=4.0, seed=101),
}


def lattice(ng: int, box_len: float = TWO_PI, lo=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Cell-centred lattice points ``lo + (i + 1/2) h``, x index slowest."""
    h = box_len / ng
    c = (np.arange(ng, dtype=np.float64) + 0.5) * h
    gx, gy, gz = np.meshgrid(c + lo[0], c + lo[1], c + lo[2], indexing="ij")
    return np.stack([gx.ravel(), gy.ravel(), gz.ravel()], axis=1)


def taylor_green_vorticity(x: np.ndarray) -> np.ndarray:
    """Curl of u = (sin x cos y cos z, -cos x sin y cos z, 0)."""
    sx, sy, sz = np.sin(x[:, 0]), np.sin(x[:, 1]), np.sin(x[:, 2])
    cx, cy, cz = np.cos(x[:, 0]), np.cos(x[:, 1]), np.cos(x[:, 2])
    return np.stack([-cx * sy * sz, -sx * cy * sz, 2.0 * sx * sy * cz], axis=1)


def taylor_green_velocity(x: np.ndarray) -> np.ndarray:
    sx, sy = np.sin(x[:, 0]), np.sin(x[:, 1])
    cx, cy, cz = np.cos(x[:, 0]), np.cos(x[:, 1]), np.cos(x[:, 2])
    return np.stack([sx * cy * cz, -cx * sy * cz, np.zeros_like(sx)], axis=1)


def _wavenumbers(ng: int):
    k = np.fft.fftfreq(ng, d=1.0 / ng)
    kr = np.fft.rfftfreq(ng, d=1.0 / ng)
    kx, ky, kz = np.meshgrid(k, k, kr, indexing="ij")
    return kx, ky, kz


def random_velocity_hat(ng: int, k0: float, rng: np.random.Generator):
    """Random-phase solenoidal velocity with E(k) ~ k^4 exp(-2 k^2/k0^2).

    Steps: white noise -> rfft -> solenoidal projection -> amplitude
    sqrt(E(k) / (4 pi k^2)) -> zero the mean and Nyquist planes.  Returns the
    half-spectrum of u (shape (3, ng, ng, ng//2+1)), not yet normalised.
    """
    xi = rng.standard_normal((3, ng, ng, ng))
    xh = np.fft.rfftn(xi, axes=(1, 2, 3))
    kx, ky, kz = _wavenumbers(ng)
    k2 = kx * kx + ky * ky + kz * kz
    k2s = np.where(k2 == 0, 1.0, k2)
    kdot = (kx * xh[0] + ky * xh[1] + kz * xh[2]) / k2s
    uh = np.stack([xh[0] - kx * kdot, xh[1] - ky * kdot, xh[2] - kz * kdot])
    kk = np.sqrt(k2)
    energy = kk ** 4 * np.exp(-2.0 * k2 / (k0 * k0))
    amp = np.sqrt(energy / (4.0 * math.pi * k2s))
    uh *= amp[None]
    nyq = ng // 2
    mask = (k2 == 0) | (np.abs(kx) == nyq) | (np.abs(ky) == nyq) | (np.abs(kz) == nyq)
    uh[:, mask] = 0.0
    return uh


def random_field(ng: int, k0: float, seed: int, box_len: float = TWO_PI):
    """(x, alpha) for a random isotropic field on the cell-centred lattice.

    The velocity is scaled so that u' = sqrt(<|u|^2>/3) = 1 on the spectral
    grid; the vorticity omega = curl u is taken spectrally and evaluated at
    the cell centres by the half-cell phase shift, then alpha = omega h^3.
    """
    rng = np.random.default_rng(seed)
    uh = random_velocity_hat(ng, k0, rng)
    u = np.fft.irfftn(uh, s=(ng, ng, ng), axes=(1, 2, 3))
    uprime = math.sqrt(float(np.mean(np.sum(u * u, axis=0))) / 3.0)
    uh /= uprime
    del u
    kx, ky, kz = _wavenumbers(ng)
    scale = TWO_PI / box_len
    kx, ky, kz = kx * scale, ky * scale, kz * scale
    h = box_len / ng
    shift = np.exp(1j * (kx + ky + kz) * (h / 2.0))
    wh = np.stack([
        1j * (ky * uh[2] - kz * uh[1]),
        1j * (kz * uh[0] - kx * uh[2]),
        1j * (kx * uh[1] - ky * uh[0]),
    ]) * shift[None]
    del uh
    omega = np.fft.irfftn(wh, s=(ng, ng, ng), axes=(1, 2, 3))
    del wh
    alpha = omega.reshape(3, -1).T * h ** 3
    x = lattice(ng, box_len)
    return x, np.ascontiguousarray(alpha)


def taylor_green_field(ng: int, jitter: float, seed: int, box_len: float = TWO_PI):
    rng = np.random.default_rng(seed)
    h = box_len / ng
    x = lattice(ng, box_len)
    if jitter:
        x = x + rng.uniform(-jitter * h, jitter * h, size=x.shape)
    alpha = taylor_green_vorticity(x) * h ** 3
    return x, alpha


def make(w: Workload | str):
    """Particles (x, alpha), both float64 of shape (N, 3), for a workload."""
    if isinstance(w, str):
        w = WORKLOADS[w]
    if w.field == "taylor_green":
        return taylor_green_field(w.ng, w.jitter, w.seed, w.box_len)
    return random_field(w.ng, w.k0, w.seed, w.box_len)


def random_particles(n: int, seed: int, box_len: float = TWO_PI, lo=(0.0, 0.0, 0.0),
                     zero_sum: bool = True):
    """Uniformly scattered particles with N(0,1) strengths (small test cases)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, box_len, size=(n, 3)) + np.asarray(lo)
    a = rng.standard_normal((n, 3))
    if zero_sum and n > 1:
        a -= a.mean(axis=0, keepdims=True)
    return x, a


def clustered_particles(n: int, seed: int, nclusters: int = 8, background: float = 0.1,
                        box_len: float = TWO_PI, lo=(0.0, 0.0, 0.0)):
    """A non-uniform particle set for the adaptive tree: `nclusters` Gaussian
    clusters at uniformly drawn centres, with standard deviations spread
    log-uniformly over [box_len/64, box_len/8] and Dirichlet(1) shares of
    (1 - background) n particles, plus background n uniform ones; positions
    wrapped into the box [lo, lo + box_len)^3; N(0,1) strengths with zero sum."""
    rng = np.random.default_rng(seed)
    nb = int(round(background * n))
    shares = rng.dirichlet(np.ones(nclusters))
    counts = np.floor(shares * (n - nb)).astype(np.int64)
    counts[: (n - nb) - int(counts.sum())] += 1
    centres = rng.uniform(0.0, box_len, size=(nclusters, 3))
    widths = box_len * np.exp(rng.uniform(np.log(1 / 64), np.log(1 / 8), size=nclusters))
    xs = [rng.normal(centres[k], widths[k], size=(int(counts[k]), 3)) for k in range(nclusters)]
    xs.append(rng.uniform(0.0, box_len, size=(nb, 3)))
    x = np.mod(np.concatenate(xs, axis=0), box_len)
    x = rng.permutation(x) + np.asarray(lo)
    a = rng.standard_normal((n, 3))
    if n > 1:
        a -= a.mean(axis=0, keepdims=True)
    return x, a


def particles_with_leaf_counts(counts, level: int, seed: int, box_len: float = TWO_PI):
    """Particles placed uniformly inside the leaves of a uniform octree at
    `level`, counts[i] of them in the leaf with cell coordinates
    (i % s, (i // s) % s, i // s^2), s = 2^level; N(0,1) strengths, zero sum.
    Points keep a margin of 1e-3 leaf widths from the leaf faces so rounding
    cannot move them across."""
    rng = np.random.default_rng(seed)
    side = 1 << level
    wl = box_len / side
    xs = []
    for i, c in enumerate(counts):
        cell = np.array([i % side, (i // side) % side, i // (side * side)], np.float64)
        xs.append((cell + rng.uniform(1e-3, 1 - 1e-3, size=(int(c), 3))) * wl)
    x = np.concatenate(xs, axis=0)
    a = rng.standard_normal(x.shape)
    if len(x) > 1:
        a -= a.mean(axis=0, keepdims=True)
    return x, a
