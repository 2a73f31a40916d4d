"""The FP64 pair kernel's polynomial approximations (no GPU).

The coefficients compiled into csrc/kernels_p2p.hip must be the output of
paper_1110_2921_amd/gen_pair64_coeffs.py, and, evaluated as the kernel does
(Horner in double), they must give 2^f to two ulp (4.5e-16) on |f| <= 1/2 and
erfcx(x) = exp(x^2) erfc(x) to 1e-15 relative on [0.75/sqrt2, 6.5], checked
against mpmath at 2000 points each.
"""
import math
import os
import re
import subprocess
import sys

import mpmath as mp
import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _generated():
    out = subprocess.run([sys.executable, "-m", "paper_1110_2921_amd.gen_pair64_coeffs"], cwd=ROOT,
                         capture_output=True, text=True, check=True).stdout
    return out.strip()


def _arr(text, name):
    m = re.search(name + r"\[\] = \{([^}]*)\}", text)
    return np.array([float(v) for v in m.group(1).split(",")])


def _const(text, name):
    return float(re.search(name + r" = ([^;]*);", text).group(1))


def test_kernel_holds_generated_coefficients():
    gen = _generated()
    src = open(os.path.join(ROOT, "paper_1110_2921_amd", "csrc", "kernels_p2p.hip")).read()
    assert gen in src


def test_polynomials_meet_their_accuracy():
    gen = _generated()
    e2, ex = _arr(gen, "kExp2C"), _arr(gen, "kErfcxC")
    mp.mp.dps = 30
    f = np.linspace(-0.5, 0.5, 2001)
    p = np.zeros_like(f) + e2[-1]
    for c in e2[-2::-1]:
        p = p * f + c
    ref = np.array([float(mp.power(2, mp.mpf(v))) for v in f])
    assert np.max(np.abs(p / ref - 1)) < 4.5e-16      # two ulp: the rounding of the evaluation
    cmap, ym, iyh = _const(gen, "kErfcxMapC"), _const(gen, "kErfcxYmid"), _const(gen, "kErfcxInvYhalf")
    x = np.linspace(0.75 / math.sqrt(2), 6.5, 2001)
    u = ((x - cmap) / (x + cmap) - ym) * iyh
    q = np.zeros_like(u) + ex[-1]
    for c in ex[-2::-1]:
        q = q * u + c
    ref = np.array([float(mp.exp(mp.mpf(v) ** 2) * mp.erfc(mp.mpf(v))) for v in x])
    assert np.max(np.abs(q / ref - 1)) < 1e-15
