"""Advection of the vortex particles with their own velocity (eq. 5).

Test infrastructure (see ``oracle/__init__``).

The particles move with the velocity the particle sum gives at their position,
dx_i/dt = u(x_i) (eq. 5; the viscous diffusion of eq. 1 is not part of this
step).  The paper names no time integrator; this follows the explicit
two-stage Runge-Kutta method of Heun (the explicit trapezoidal rule):

    x*      = x_n + dt u(x_n)
    x_{n+1} = x_n + (dt / 2) (u(x_n) + u(x*))

with the velocity of every stage evaluated afresh at the current positions:
by the FMM (a new tree on the moved particles, its root the bounding square of
the stage's positions) or by the direct sum.
"""
from __future__ import annotations

import numpy as np

from . import fmm as F
from . import kernel as K


def heun_step(x, y, velocity, dt):
    """One step of Heun's method for dx/dt = velocity(x, y)."""
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    u1, v1 = velocity(x, y)
    xs = x + dt * u1
    ys = y + dt * v1
    u2, v2 = velocity(xs, ys)
    return x + 0.5 * dt * (u1 + u2), y + 0.5 * dt * (v1 + v2)


def advect(x, y, gamma, sigma, dt, steps, p=None, levels=None, radius=0.0, direct=False):
    """``steps`` Heun steps with the FMM velocity (p, levels, near radius) or,
    with ``direct``, the direct sum (eq. 7)."""
    gamma = np.asarray(gamma, np.float64)

    def vel(xx, yy):
        if direct:
            return K.direct_velocity(xx, yy, gamma, sigma)
        r = F.fmm_velocity(xx, yy, gamma, sigma, p, levels, radius=radius)
        return r.u, r.v

    for _ in range(steps):
        x, y = heun_step(x, y, vel, dt)
    return x, y
