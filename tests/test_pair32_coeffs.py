"""The FP32 pair kernel's erfcx polynomial (no GPU).

The coefficients compiled into csrc/kernels_p2p.hip must be the output of
paper_1110_2921_amd/gen_pair32_coeffs.py.  Evaluated as the kernel does (FP32:
reciprocal square root, 1/rho = sigma rinv, Horner, exp2, the final FMA), the
cutoff g of eq. (6) must stay within 1.5e-6 relative of its definition
(erf and exp in double) for rho in [1, 14], no worse than the rational erf
approximation it replaced (1.3e-6 in the same FP32 evaluation), and the fit
itself, in double, within 2e-7.
"""
import os
import re
import subprocess
import sys

import numpy as np
from scipy.special import erf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _generated():
    return subprocess.run([sys.executable, "-m", "paper_1110_2921_amd.gen_pair32_coeffs"], cwd=ROOT,
                          capture_output=True, text=True, check=True).stdout.strip()


def _coeffs(text):
    m = re.search(r"kErfcxU32\[\] = \{([^}]*)\}", text)
    return [np.float32(v.strip().rstrip("f")) for v in m.group(1).split(",")]


def _g_exact(rho):
    return erf(rho / np.sqrt(2.0)) - np.sqrt(2.0 / np.pi) * rho * np.exp(-0.5 * rho * rho)


def _g_fp32(r, sigma, c):
    f = np.float32
    r2 = f(r) * f(r)
    rinv = (f(1) / np.sqrt(r2.astype(np.float64))).astype(np.float32)   # a correctly rounded rsqrt
    rr = f(r2 * rinv)
    u = f(f(sigma) * rinv)
    ex = c[-1]
    for ck in c[-2::-1]:
        ex = f(ex * u + ck)
    ke = f(-0.5 * np.log2(np.e) / (sigma * sigma))
    e = np.exp2(f(r2 * ke).astype(np.float64)).astype(np.float32)
    ks = f(np.sqrt(2.0 / np.pi) / sigma)
    return (f(1) - e * f(ks * rr + ex)).astype(np.float64), (rr / f(sigma)).astype(np.float64)


def test_kernel_holds_generated_coefficients():
    gen = _generated()
    src = open(os.path.join(ROOT, "paper_1110_2921_amd", "csrc", "kernels_p2p.hip")).read()
    assert gen in src


def test_fit_bound_in_double():
    from paper_1110_2921_amd import gen_pair32_coeffs as G
    c, err = G.fit()
    assert err < 2e-7
    rho = np.linspace(1.0, 14.0, 50001)
    from scipy.special import erfcx
    w = np.exp(-0.5 * rho * rho) / _g_exact(rho)
    approx = np.polynomial.polynomial.polyval(1.0 / rho, c)
    assert np.max(np.abs(approx - erfcx(rho / np.sqrt(2.0))) * w) < 2e-7


def test_cutoff_in_fp32():
    c = _coeffs(_generated())
    for sigma in (2 * np.pi / 256, 0.1, 1.0):
        r = np.linspace(1.0, 14.0, 200001) * sigma
        g, rho = _g_fp32(r, sigma, c)
        rel = np.abs(g - _g_exact(rho)) / _g_exact(rho)
        assert rel.max() < 1.5e-6, (sigma, rel.max())
