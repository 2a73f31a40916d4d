"""Infinite-lattice velocity of lattice-placed Gaussian blobs (test oracle).

For blobs on the cell-centred lattice x_j = (j + 1/2) h of the periodic cube
[0, 2 pi)^3, the periodic vorticity of eqs. 3-4 has Fourier coefficients

    omega_k = (1/L^3) sum_j alpha_j exp(-i k.x_j) exp(-sigma^2 |k|^2 / 2)

and the Biot-Savart velocity u = curl (G * omega) (eqs. 1, 5) is
u_k = i k x omega_k / |k|^2 with the mean (k = 0) set to zero; the gradient
is J_k[a, b] = i k_a u_k[b].  Evaluated back on the same lattice, a
wavevector k = m + ng a (m in the DFT box, a in Z^3) carries the same phase
as m, so the sum over a folds into one DFT per component; |a_i| <= 2 makes
the folded sum exact in double precision for sigma >= h.
"""
from __future__ import annotations

import math

import numpy as np


def lattice_velocity(alpha, ng, sigma, box_len=2 * math.pi, alias=2):
    """u (N,3) and J (N,3,3) at the lattice points; alpha in lattice order."""
    alpha = np.asarray(alpha, np.float64).reshape(ng, ng, ng, 3)
    h = box_len / ng
    A = np.fft.fftn(np.moveaxis(alpha, -1, 0), axes=(1, 2, 3))   # (3, ng, ng, ng)
    m = np.fft.fftfreq(ng, d=1.0 / ng)
    M = np.stack(np.meshgrid(m, m, m, indexing="ij"))              # (3, ng, ng, ng)
    scale = 2 * math.pi / box_len
    Bu = np.zeros_like(A)
    BJ = np.zeros((3, 3) + A.shape[1:], np.complex128)
    rng = range(-alias, alias + 1)
    for ax in rng:
        for ay in rng:
            for az in rng:
                k = (M + ng * np.array([ax, ay, az])[:, None, None, None]) * scale
                k2 = np.sum(k * k, axis=0)
                zero = k2 == 0
                k2s = np.where(zero, 1.0, k2)
                f = np.where(zero, 0.0, np.exp(-0.5 * sigma * sigma * k2) / k2s)
                # i k x A
                cx = 1j * (k[1] * A[2] - k[2] * A[1]) * f
                cy = 1j * (k[2] * A[0] - k[0] * A[2]) * f
                cz = 1j * (k[0] * A[1] - k[1] * A[0]) * f
                c = np.stack([cx, cy, cz])
                Bu += c
                for a in range(3):
                    BJ[a] += 1j * k[a] * c
    norm = 1.0 / box_len ** 3 * ng ** 3
    u = np.real(np.fft.ifftn(Bu, axes=(1, 2, 3))) * norm
    J = np.real(np.fft.ifftn(BJ, axes=(2, 3, 4))) * norm
    u = np.moveaxis(u, 0, -1).reshape(-1, 3)
    J = np.moveaxis(J, (0, 1), (-2, -1)).reshape(-1, 3, 3)
    return u, J


def energy_spectrum(u, ng, kmax):
    """Shell energy spectrum of a velocity sampled on an ng^3 lattice of the
    periodic cube (lattice order, x index slowest; u (ng^3, 3)):

        E(s) = 1/2 sum_{m : rint(|m|) = s} |u_m|^2,  s = 0 .. kmax,

    u_m the Fourier coefficients (1/ng^3) sum_x u(x) exp(-i k.x) on the integer
    wavevectors m of the DFT box (k = 2 pi m / box_len), so that sum_s E(s) is
    1/2 <|u|^2> when kmax covers every shell.  Full complex FFT, no symmetry
    folding.
    """
    u = np.asarray(u, np.float64).reshape(ng, ng, ng, 3)
    U = np.fft.fftn(np.moveaxis(u, -1, 0), axes=(1, 2, 3)) / ng ** 3
    m = np.fft.fftfreq(ng, d=1.0 / ng)
    M = np.stack(np.meshgrid(m, m, m, indexing="ij"))
    shell = np.rint(np.sqrt(np.sum(M * M, axis=0))).astype(np.int64)
    power = 0.5 * np.sum(np.abs(U) ** 2, axis=0)
    E = np.zeros(kmax + 1)
    keep = shell <= kmax
    np.add.at(E, shell[keep], power[keep])
    return E
