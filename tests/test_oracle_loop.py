"""Pins of the oracle's time loop (no GPU).

* A lone particle in free space neither moves nor stretches (its self
  velocity is zero and the self gradient's contraction alpha_a J[a][:] is
  q(0)/(4 pi) alpha x alpha = 0), so only core spreading acts:
  sigma^2 = sigma0^2 + 2 nu t exactly, for both integrators.
* With dt = 0 a loop on the lattice that reinitialises every step returns its
  input (reinitialisation of a lattice state with the same core is the
  identity, to the interpolation matrix's conditioning).
* Order of accuracy: against a reference with 16 steps, the error of the
  state at t = 0.2 falls by about 2 per halving of dt for Euler and about 4
  for Heun with the core spreading (the second stage must see the new core
  for that).
"""
import math

import numpy as np

import workloads as W
from oracle import loop as LP
from oracle import rbf as R

L = 2 * math.pi


def test_lone_particle_only_spreads():
    x = np.array([[3.0, 2.5, 3.5]])
    a = np.array([[0.3, -0.2, 0.5]])
    for integ in ("euler", "heun"):
        x1, a1, s1 = LP.run(x, a, 0.4, 4, 2, 0, 0.05, 0.3, 4, integrator=integ)
        assert np.array_equal(x1, x) and np.allclose(a1, a, rtol=0, atol=1e-17)
        assert abs(s1 - math.sqrt(0.16 + 2 * 0.3 * 0.05 * 4)) < 1e-15


def test_zero_time_step_with_reinit_is_identity():
    x = R.lattice_sites(8, L)
    h = L / 8
    a = W.taylor_green_vorticity(x) * h ** 3
    x1, a1, s1 = LP.run(x, a, h, 4, 1, 1, 0.0, 0.0, 2, reinit_every=1, ng=8)
    assert np.array_equal(x1, x) and s1 == h
    assert np.abs(a1 - a).max() < 1e-9 * np.abs(a).max()


def test_integrators_converge_at_their_order():
    x, a = W.random_particles(40, 21, box_len=2.0, lo=(2.0, 2.0, 2.0))
    a *= 0.5
    sigma, nu, T = 0.35, 0.2, 0.2
    kw = dict(p=6, level=2, periodic=0, nu=nu)
    ref = {}
    for integ in ("euler", "heun"):
        ref[integ] = LP.run(x, a, sigma, dt=T / 16, steps=16, integrator=integ, **kw)
    err = {}
    for integ in ("euler", "heun"):
        e = []
        for steps in (2, 4):
            xs, as_, ss = LP.run(x, a, sigma, dt=T / steps, steps=steps, integrator=integ, **kw)
            e.append(np.linalg.norm(xs - ref[integ][0]) + np.linalg.norm(as_ - ref[integ][1]))
        err[integ] = e[0] / e[1]
    assert 1.6 < err["euler"] < 2.6
    assert 3.2 < err["heun"] < 5.0
