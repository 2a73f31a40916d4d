"""The vortex method's time loop (test infrastructure: the oracle).

Sec. 2.2: the three terms of the vorticity equation update three separate
particle variables at the same time -- positions by convection (eq. 7),
strengths by stretching (eq. 8) and the core by diffusion, d sigma^2/dt = 2 nu
(core spreading).  To keep sigma small the particles are reinitialised every
few steps onto the lattice by RBF interpolation with the original core
(the reinitialisation paragraph; Sec. 5 studies how often).

One step from (x, alpha, sigma), with rates (u, s) = FMM(x, alpha, sigma):

* "euler" (the paper's integrator): x + dt u, alpha + dt s;
* "heun": the trapezoid of the rates at the start and at the Euler
  prediction, the second taken with the core the step ends with;

then sigma^2 + 2 nu dt, and periodic positions are wrapped into the box.
After every `reinit_every`-th step (0: never) the state is replaced by the
lattice sites, the interpolated strengths and the core sigma0.
"""
from __future__ import annotations

import math

import numpy as np

from . import direct as D
from . import fmm as F
from . import rbf as R
from . import tree as T


def rates(x, alpha, sigma, p, level, periodic, box_len, scheme):
    u, J = F.fmm(x, alpha, sigma, p, level, box_len=box_len, periodic=periodic)
    return u, D.stretching(J, alpha, scheme)


def run(x, alpha, sigma, p, level, periodic, dt, nu, steps, reinit_every=0, ng=0, integrator="euler",
        scheme="classic", box_len=2 * math.pi):
    """State (x, alpha, sigma) after `steps` steps."""
    x = np.array(x, np.float64)
    alpha = np.array(alpha, np.float64)
    sigma0 = sigma
    for step in range(steps):
        sigma_next = math.sqrt(sigma * sigma + 2.0 * nu * dt)
        u1, s1 = rates(x, alpha, sigma, p, level, periodic, box_len, scheme)
        if integrator == "euler":
            x = x + dt * u1
            alpha = alpha + dt * s1
        elif integrator == "heun":
            u2, s2 = rates(x + dt * u1, alpha + dt * s1, sigma_next, p, level, periodic, box_len, scheme)
            x = x + 0.5 * dt * (u1 + u2)
            alpha = alpha + 0.5 * dt * (s1 + s2)
        else:
            raise ValueError(integrator)
        if periodic:
            x = T.wrap(x, (0.0, 0.0, 0.0), box_len)
        sigma = sigma_next
        if reinit_every and (step + 1) % reinit_every == 0:
            x, alpha, _ = R.reinit(x, alpha, sigma, ng, sigma0, level, box_len, periodic)
            sigma = sigma0
    return x, alpha, sigma
