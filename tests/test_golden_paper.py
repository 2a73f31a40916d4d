"""The paper's printed base parameters and accuracy statement (Sec. 4.1),
read from tests/golden/paper_base_parameters.txt (no GPU).

* The headline workload, the library's time-loop defaults and the
  benchmark's loop use the base parameters: N = 256^3 in a cube of side
  2 pi, p = 10, 3^3 x 3^3 x 3^3 - 1 periodic images, forward Euler with
  dt = 0.005, reinitialisation every 10 steps, Krylov drop tolerance 1e-3.
* The oracle FMM at p = 10 on the same recipe (a 16^3 field, leaves of
  4 x 4 x 4 particles as at 256^3 on level 6, sigma = h) gives u and the
  stretching dalpha/dt to the four significant digits the paper states, and
  not to single precision: relative L2 error against the exact sum over the
  27 boxes of S_1 within (2^-24, 5e-4], k significant digits being read as a
  relative error of at most half a unit in the k-th digit, 5 x 10^-k.
"""
import inspect
import math
import os

import numpy as np

import workloads as W
from oracle import direct as D
from oracle import fmm as F

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    vals = {}
    with open(os.path.join(HERE, "golden", "paper_base_parameters.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = (s.strip() for s in line.split("=", 1))
                vals[k] = float(v)
    return vals


def test_headline_workload_uses_the_base_parameters():
    g = _golden()
    w = W.WORKLOADS["rand256_periodic"]
    assert w.n == int(g["n"]) and w.ng ** 3 == int(g["n"])
    assert w.p == int(g["p"])
    assert (3 ** w.periodic) ** 3 - 1 == int(g["periodic_images"])
    assert math.isclose(w.box_len, g["domain_side"], rel_tol=1e-15)


def test_time_loop_uses_the_base_parameters():
    """The library's loop defaults and the benchmark's loop."""
    import bench
    import paper_1110_2921_amd as vm
    g = _golden()
    run = inspect.signature(vm.FMM.run).parameters
    reinit = inspect.signature(vm.FMM.reinit).parameters
    assert run["integrator"].default == "euler"
    assert run["tol"].default == g["krylov_tolerance"]
    assert reinit["tol"].default == g["krylov_tolerance"]
    assert bench.PAPER_DT == g["dt"]
    assert bench.PAPER_REINIT_EVERY == int(g["reinit_every"])
    assert bench.PAPER_TOL == g["krylov_tolerance"]


def test_p10_gives_four_significant_digits_not_single_precision():
    g = _golden()
    digits, p = int(g["significant_digits"]), int(g["p"])
    ng = 16
    x, a = W.random_field(ng, 4.0, 7)
    h = W.TWO_PI / ng
    u, J = F.fmm(x, a, h, p, 2, periodic=1)
    s = np.random.default_rng(3).choice(len(x), 256, replace=False)
    u0, J0 = D.direct(x[s], x, a, h, K=1)
    eu = np.linalg.norm(u[s] - u0) / np.linalg.norm(u0)
    da, da0 = D.stretching(J[s], a[s]), D.stretching(J0, a[s])
    ed = np.linalg.norm(da - da0) / np.linalg.norm(da0)
    upper, lower = 5.0 * 10.0 ** -digits, 2.0 ** -24
    assert lower < eu <= upper, eu
    assert lower < ed <= upper, ed
