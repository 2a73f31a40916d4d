"""Spherical-harmonic expansions in the paper's nomenclature (test oracle).

The paper writes the Laplace kernel's expansions (eqs. 10-11) with the
operators of Cheng, Greengard & Rokhlin:

    S_i = r^{-n-1} Y_n^m(theta, phi),   M_j = rho^n Y_n^{-m}(alpha, beta)
    R_i = r^n Y_n^m(theta, phi),        L_j = rho^{-n-1} Y_n^{-m}(alpha, beta)

with Y_n^m = sqrt((n-|m|)!/(n+|m|)!) P_n^{|m|}(cos theta) e^{i m phi}.  Here
``regular(x)`` returns r^n Y_n^m (the R operator evaluated at x) and
``irregular(x)`` returns r^{-n-1} Y_n^m (the S operator), both for
0 <= n <= deg and -n <= m <= n, stored at index n^2 + n + m.

P_n^{|m|}(t) (1-t^2)^{-|m|/2} is the |m|-th derivative of the Legendre
polynomial, summed from its explicit coefficients, so r^n Y_n^m is the
polynomial sqrt(...) (x +/- i y)^{|m|} sum_k c_k z^{n-|m|-2k} r^{2k}.
The same polynomial is expanded into monomials x^a y^b z^c to give exact
first and second derivatives for the local-to-particle step.

Translation operators follow Cheng et al. (their Theorems 3.3-3.5), with
A_n^m = (-1)^n / sqrt((n-m)!(n+m)!):

    M2M  M'_j^k = sum_{n,m} M_{j-n}^{k-m} i^{|k|-|m|-|k-m|} A_n^m A_{j-n}^{k-m}
                  rho^n Y_n^{-m}(alpha,beta) / A_j^k,       (rho,alpha,beta) = old - new centre
    M2L  L_j^k  = sum_{n,m} M_n^m i^{|k-m|-|k|-|m|} A_n^m A_j^k Y_{j+n}^{m-k}(alpha,beta)
                  / ((-1)^n A_{j+n}^{m-k} rho^{j+n+1}),     (rho,alpha,beta) = source - target centre
    L2L  L'_j^k = sum_{n>=j,m} L_n^m i^{|m|-|m-k|-|k|} A_{n-j}^{m-k} A_j^k
                  Y_{n-j}^{m-k}(alpha,beta) rho^{n-j} / ((-1)^{n+j} A_n^m),  (rho,alpha,beta) = old - new centre
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np


def idx(n, m):
    return n * n + n + m


def ncoef(p):
    return (p + 1) ** 2


def _legendre_deriv(n, m):
    """[(k, c_k)] with d^m/dt^m P_n(t) = sum_k c_k t^(n - 2k - m)."""
    out = []
    for k in range(n // 2 + 1):
        e = n - 2 * k
        if e < m:
            break
        c = ((-1) ** k * math.comb(n, k) * math.comb(2 * n - 2 * k, n) / 2.0 ** n
             * math.factorial(e) / math.factorial(e - m))
        out.append((k, c))
    return out


def _norm(n, m):
    return math.sqrt(math.factorial(n - abs(m)) / math.factorial(n + abs(m)))


def regular(x, deg):
    """r^n Y_n^m(theta, phi) at points x (P, 3) -> complex (P, (deg+1)^2)."""
    x = np.atleast_2d(np.asarray(x, np.float64))
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    r2 = X * X + Y * Y + Z * Z
    w = X + 1j * Y
    # power tables z^e, (r^2)^k, (x + i y)^m
    zp = [np.ones_like(Z)]
    r2p = [np.ones_like(Z)]
    wp = [np.ones_like(w)]
    for _ in range(deg):
        zp.append(zp[-1] * Z)
        r2p.append(r2p[-1] * r2)
        wp.append(wp[-1] * w)
    out = np.zeros((x.shape[0], ncoef(deg)), np.complex128)
    for n in range(deg + 1):
        for m in range(n + 1):
            s = np.zeros_like(X)
            for k, c in _legendre_deriv(n, m):
                s = s + c * (zp[n - 2 * k - m] * r2p[k])
            v = _norm(n, m) * wp[m] * s
            out[:, idx(n, m)] = v
            out[:, idx(n, -m)] = np.conj(v)
    return out


def irregular(x, deg):
    """r^{-n-1} Y_n^m(theta, phi) = r^n Y_n^m / r^{2n+1} (Kelvin transform)."""
    x = np.atleast_2d(np.asarray(x, np.float64))
    r2 = np.sum(x * x, axis=1)
    reg = regular(x, deg)
    for n in range(deg + 1):
        reg[:, n * n:(n + 1) ** 2] /= (r2 ** (n + 0.5))[:, None]
    return reg


@lru_cache(maxsize=None)
def _monomials(deg):
    return [(a, b, c) for t in range(deg + 1) for a in range(t + 1)
            for b in range(t - a + 1) for c in [t - a - b]]


@lru_cache(maxsize=None)
def regular_poly(deg):
    """Monomial coefficients: r^n Y_n^m = sum_q P[idx(n,m), q] x^a y^b z^c."""
    mon = _monomials(deg)
    pos = {e: i for i, e in enumerate(mon)}
    P = np.zeros((ncoef(deg), len(mon)), np.complex128)
    for n in range(deg + 1):
        for m in range(n + 1):
            # (x + i y)^m as {(a, b): coef}
            xy = {}
            for a in range(m + 1):
                xy[(a, m - a)] = math.comb(m, a) * (1j) ** (m - a)
            for k, c in _legendre_deriv(n, m):
                ez = n - 2 * k - m
                # (x^2 + y^2 + z^2)^k expanded
                for i2 in range(k + 1):
                    for j2 in range(k - i2 + 1):
                        l2 = k - i2 - j2
                        cm = math.factorial(k) / (math.factorial(i2) * math.factorial(j2)
                                                  * math.factorial(l2))
                        for (a, b), cxy in xy.items():
                            e = (a + 2 * i2, b + 2 * j2, ez + 2 * l2)
                            P[idx(n, m), pos[e]] += _norm(n, m) * c * cm * cxy
            if m > 0:
                P[idx(n, -m)] = np.conj(P[idx(n, m)])
    return P


def monomial_derivs(x, deg):
    """Values, gradients (3) and Hessians (3,3) of all monomials of degree <= deg."""
    x = np.atleast_2d(np.asarray(x, np.float64))
    mon = _monomials(deg)
    npt = x.shape[0]
    pw = np.ones((3, deg + 1, npt))
    for d in range(3):
        for e in range(1, deg + 1):
            pw[d, e] = pw[d, e - 1] * x[:, d]

    def power(d, e):
        return pw[d, e] if e >= 0 else np.zeros(npt)

    val = np.zeros((npt, len(mon)))
    grad = np.zeros((npt, 3, len(mon)))
    hess = np.zeros((npt, 3, 3, len(mon)))
    for q, e in enumerate(mon):
        val[:, q] = power(0, e[0]) * power(1, e[1]) * power(2, e[2])
        for a in range(3):
            ea = list(e)
            ca = ea[a]
            ea[a] -= 1
            grad[:, a, q] = ca * power(0, ea[0]) * power(1, ea[1]) * power(2, ea[2]) if ca else 0.0
            for b in range(3):
                eb = list(ea)
                cb = eb[b]
                eb[b] -= 1
                if ca and cb:
                    hess[:, a, b, q] = ca * cb * power(0, eb[0]) * power(1, eb[1]) * power(2, eb[2])
    return val, grad, hess


def A(n, m):
    return (-1.0) ** n / math.sqrt(math.factorial(n - m) * math.factorial(n + m))


def _ipow(e):
    return (1j) ** (e % 4)


@lru_cache(maxsize=None)
def _m2l_index(p):
    rows, cols, src, fac = [], [], [], []
    for j in range(p + 1):
        for k in range(-j, j + 1):
            for n in range(p + 1):
                for m in range(-n, n + 1):
                    rows.append(idx(j, k))
                    cols.append(idx(n, m))
                    src.append(idx(j + n, m - k))
                    fac.append(_ipow(abs(k - m) - abs(k) - abs(m)) * A(n, m) * A(j, k)
                               / ((-1.0) ** n * A(j + n, m - k)))
    return (np.array(rows), np.array(cols), np.array(src), np.array(fac))


def m2l_matrix(d, p):
    """T with L = T @ M for a multipole at (target centre + d)."""
    return m2l_matrices(np.asarray(d, np.float64)[None], p)[0]


def m2l_matrices(ds, p):
    """M2L matrices for several source-centre offsets ds (K, 3) at once."""
    rows, cols, src, fac = _m2l_index(p)
    S = irregular(np.asarray(ds, np.float64), 2 * p)
    T = np.zeros((len(ds), ncoef(p), ncoef(p)), np.complex128)
    T[:, rows, cols] = fac[None, :] * S[:, src]
    return T


@lru_cache(maxsize=None)
def _m2m_index(p):
    rows, cols, src, fac = [], [], [], []
    for j in range(p + 1):
        for k in range(-j, j + 1):
            for n in range(j + 1):
                for m in range(-n, n + 1):
                    if abs(k - m) > j - n:
                        continue
                    rows.append(idx(j, k))
                    cols.append(idx(j - n, k - m))
                    src.append(idx(n, -m))
                    fac.append(_ipow(abs(k) - abs(m) - abs(k - m)) * A(n, m) * A(j - n, k - m)
                               / A(j, k))
    return (np.array(rows), np.array(cols), np.array(src), np.array(fac))


def m2m_matrix(d, p):
    """M_new = T @ M_old for d = old centre - new centre."""
    rows, cols, src, fac = _m2m_index(p)
    R = regular(np.asarray(d, np.float64)[None], p)[0]
    T = np.zeros((ncoef(p), ncoef(p)), np.complex128)
    np.add.at(T, (rows, cols), fac * R[src])
    return T


@lru_cache(maxsize=None)
def _l2l_index(p):
    rows, cols, src, fac = [], [], [], []
    for j in range(p + 1):
        for k in range(-j, j + 1):
            for n in range(j, p + 1):
                for m in range(-n, n + 1):
                    if abs(m - k) > n - j:
                        continue
                    rows.append(idx(j, k))
                    cols.append(idx(n, m))
                    src.append(idx(n - j, m - k))
                    fac.append(_ipow(abs(m) - abs(m - k) - abs(k)) * A(n - j, m - k) * A(j, k)
                               / ((-1.0) ** (n + j) * A(n, m)))
    return (np.array(rows), np.array(cols), np.array(src), np.array(fac))


def l2l_matrix(d, p):
    """L_new = T @ L_old for d = old centre - new centre."""
    rows, cols, src, fac = _l2l_index(p)
    R = regular(np.asarray(d, np.float64)[None], p)[0]
    T = np.zeros((ncoef(p), ncoef(p)), np.complex128)
    np.add.at(T, (rows, cols), fac * R[src])
    return T


def p2m(y, q, p):
    """M_n^m = sum_j q_j rho_j^n Y_n^{-m}(alpha_j, beta_j) for offsets y (P,3), charges q (P,K)."""
    R = regular(y, p)
    neg = np.array([idx(n, -m) for n in range(p + 1) for m in range(-n, n + 1)])
    return np.einsum("pk,pc->kc", np.asarray(q, np.float64), R[:, neg])


def eval_multipole(M, x, p):
    """Potential sum_n,m M_n^m S_n^m(x) (real part) at points x for each row of M."""
    S = irregular(x, p)
    return np.real(S @ np.asarray(M).T)


def eval_local(L, x, p):
    R = regular(x, p)
    return np.real(R @ np.asarray(L).T)


def local_derivs(L, x, p):
    """Gradient (P, K, 3) and Hessian (P, K, 3, 3) of sum L_n^m R_n^m(x)."""
    P = regular_poly(p)
    _, g, h = monomial_derivs(x, p)
    coef = np.asarray(L) @ P           # (K, nmono): potential as a polynomial
    grad = np.real(np.einsum("km,pam->pka", coef, g))
    hess = np.real(np.einsum("km,pabm->pkab", coef, h))
    return grad, hess
