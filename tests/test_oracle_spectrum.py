"""Pins of the oracle's shell energy spectrum (no GPU).

* A single Fourier mode u = A sin(m.x + phi) e (e perpendicular to m) carries
  <|u|^2>/2 = A^2/4, all of it in the shell rint(|m|): the spectrum is A^2/4
  there and zero elsewhere, whatever the phase and the direction of m.
* Parseval on a random lattice field: sum_s E(s) = <|u|^2>/2 when kmax covers
  the corner of the DFT box (sqrt(3) ng/2).
* Shell membership follows rint(|m|): modes with |m| = 2.4 and 2.6 land in
  shells 2 and 3.
"""
import math

import numpy as np

from oracle import spectral as S

L = 2 * math.pi


def _lattice(ng):
    c = np.arange(ng) * (L / ng)
    return np.stack(np.meshgrid(c, c, c, indexing="ij"), axis=-1).reshape(-1, 3)


def _mode(x, m, e, amp, phi):
    return amp * np.sin(x @ np.asarray(m, np.float64) + phi)[:, None] * np.asarray(e, np.float64)[None, :]


def test_single_mode_lands_in_its_shell():
    ng = 16
    x = _lattice(ng)
    for m, e in (([3, 0, 0], [0, 1, 0]), ([1, 2, 2], [2, -1, 0]), ([0, -4, 3], [1, 0, 0])):
        e = np.asarray(e, np.float64) / np.linalg.norm(e)
        E = S.energy_spectrum(_mode(x, m, e, 1.7, 0.4), ng, 12)
        s = int(round(np.linalg.norm(m)))
        want = np.zeros(13)
        want[s] = 1.7 ** 2 / 4
        assert np.allclose(E, want, rtol=0, atol=1e-14)


def test_parseval():
    ng = 12
    u = np.random.default_rng(5).standard_normal((ng ** 3, 3))
    E = S.energy_spectrum(u, ng, int(math.ceil(math.sqrt(3) * ng / 2)))
    assert abs(E.sum() - 0.5 * np.mean(np.sum(u * u, axis=1))) < 1e-13


def test_shell_rounding():
    ng = 16
    x = _lattice(ng)
    # |(2, 1, 0)| = 2.236 -> shell 2; |(2, 1, 1)| = 2.449 -> 2; |(2, 2, 1)| = 3 -> 3; |(2, 2, 0)| = 2.83 -> 3
    for m, s in (([2, 1, 0], 2), ([2, 1, 1], 2), ([2, 2, 0], 3), ([2, 2, 1], 3)):
        e = np.cross(m, [0.3, 0.5, 0.7])
        e /= np.linalg.norm(e)
        E = S.energy_spectrum(_mode(x, m, e, 1.0, 0.0), ng, 8)
        assert abs(E[s] - 0.25) < 1e-14 and abs(E.sum() - 0.25) < 1e-14
