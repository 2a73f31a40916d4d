"""Direct regularised Biot-Savart sums (test infrastructure: the oracle).

``direct`` calls the C implementation in ``direct.c`` (built into
``oracle/_direct.so`` by ``oracle.build``); ``direct_numpy`` is an
independent NumPy transcription of the same definitions for tiny inputs.
Definitions (paper eqs. 3-8; the cutoff is eq. 6):

    u_i      = 1/(4 pi) sum_{n in S_K} sum_j q(r) alpha_j x r,  r = x_i - x_j - n L
    J_i[a,b] = d u_b / d x_a
    q(r)     = g(r/sigma) / r^3,  g(rho) = erf(rho/sqrt 2) - sqrt(2/pi) rho exp(-rho^2/2)

Stretching (eq. 8, "classic"): dalpha_i/dt = sum_a alpha_{i,a} J_i[a, :].
"Transpose" variant: dalpha_i/dt = J_i[:, b] alpha_{i,b}.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
from scipy.special import erf

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "_direct.so")
        if not os.path.exists(path):
            from . import build
            build.build()
        lib = ctypes.CDLL(path)
        f = lib.oracle_direct
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int32)
        f.argtypes = [ctypes.c_int64, dp, ctypes.c_int64, dp, dp, ctypes.c_double,
                      ctypes.c_double, ctypes.c_int, ip, ip, ctypes.c_int, dp, dp]
        f.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def direct(xt, xs, alpha, sigma, box_len=2 * math.pi, K=0, cells_t=None, cells_s=None,
           level=0, want_grad=True):
    """Velocity (nt,3) and gradient (nt,3,3) at targets ``xt`` from sources.

    ``K``: 0 for free space, else the image block S_K of period ``box_len``.
    ``cells_t``/``cells_s``: leaf coordinates at ``level``; when given, pairs
    in non-adjacent leaves use g = 1 (the FMM's far-field model).
    Positions of a periodic problem must already be wrapped into the box.
    """
    xt = np.ascontiguousarray(xt, dtype=np.float64)
    xs = np.ascontiguousarray(xs, dtype=np.float64)
    al = np.ascontiguousarray(alpha, dtype=np.float64)
    nt, ns = xt.shape[0], xs.shape[0]
    u = np.zeros((nt, 3))
    J = np.zeros((nt, 9)) if want_grad else None
    ct = cs = None
    if cells_t is not None:
        ct = np.ascontiguousarray(cells_t, dtype=np.int32)
        cs = np.ascontiguousarray(cells_s, dtype=np.int32)
    rc = _lib().oracle_direct(nt, _dptr(xt), ns, _dptr(xs), _dptr(al), float(sigma),
                              float(box_len), int(K),
                              _iptr(ct) if ct is not None else None,
                              _iptr(cs) if cs is not None else None,
                              int(level), _dptr(u), _dptr(J) if J is not None else None)
    if rc != 0:
        raise ValueError("oracle_direct rejected its arguments")
    return u, (J.reshape(nt, 3, 3) if J is not None else None)


def image_block(K):
    r = (3 ** K - 1) // 2
    rng = np.arange(-r, r + 1)
    return np.stack(np.meshgrid(rng, rng, rng, indexing="ij"), -1).reshape(-1, 3)


def direct_numpy(xt, xs, alpha, sigma, box_len=2 * math.pi, K=0):
    """NumPy twin of ``direct`` (exact kernel everywhere), O(nt*ns) memory."""
    xt = np.asarray(xt, np.float64)
    xs = np.asarray(xs, np.float64)
    alpha = np.asarray(alpha, np.float64)
    u = np.zeros((len(xt), 3))
    J = np.zeros((len(xt), 3, 3))
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1.0
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1.0
    for n in image_block(K):
        r = xt[:, None, :] - xs[None, :, :] - n[None, None, :] * box_len
        r2 = np.sum(r * r, axis=-1)
        rr = np.sqrt(r2)
        rho = rr / sigma
        e = np.exp(-0.5 * rho * rho)
        with np.errstate(divide="ignore", invalid="ignore"):
            g = erf(rho / math.sqrt(2.0)) - math.sqrt(2.0 / math.pi) * rho * e
            q = g / (r2 * rr)
            dq = (math.sqrt(2.0 / math.pi) * e / sigma ** 3 - 3.0 * q) / r2
        zero = r2 == 0.0
        q = np.where(zero, math.sqrt(2.0 / math.pi) / (3.0 * sigma ** 3), q)
        dq = np.where(zero, 0.0, dq)
        c = np.cross(alpha[None, :, :], r)
        u += np.einsum("ij,ijb->ib", q, c)
        # q eps_{bca} alpha_c  ->  J[a][b]
        J += np.einsum("ij,bca,jc->iab", q, eps, alpha)
        J += np.einsum("ij,ija,ijb->iab", dq, r, c)
    return u / (4 * math.pi), J / (4 * math.pi)


def stretching(J, alpha, scheme="classic"):
    """dalpha/dt from the gradient: classic (alpha . grad) u, or J . alpha."""
    if scheme == "classic":
        return np.einsum("ia,iab->ib", alpha, J)
    if scheme == "transpose":
        return np.einsum("iab,ib->ia", J, alpha)
    raise ValueError(scheme)
