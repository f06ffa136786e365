"""Pins of the advection oracle (eq. 5, Heun's two-stage Runge-Kutta method).

* Two well separated Gaussian blobs behave as point vortices: they turn about
  their circulation centroid at the rate (G1 + G2) / (2 pi d^2) on circles;
  Heun's method follows the closed-form positions with a global error of
  second order in dt (halving dt divides it by about 4).
* The direct sum is antisymmetric (sum_i G_i u_i = 0), so every Heun step
  conserves the linear impulse sum_i G_i x_i to rounding; with the FMM the
  impulse moves only by the FMM error.
* One step written out with plain loops (stage velocities from eq. 6 pair by
  pair) equals ``heun_step``; a planted mistake (the first stage velocity used
  twice) is caught.
"""
import math

import numpy as np

import workloads as W
from oracle import advect as A
from oracle import kernel as K


def _pair_orbit(T, dt):
    g = np.array([1.0, 0.5])
    d = 0.5
    x = np.array([-d / 2, d / 2]); y = np.zeros(2)
    xf, yf = A.advect(x, y, g, 0.02, dt, int(round(T / dt)), direct=True)
    xc = (g @ x) / g.sum(); yc = 0.0
    om = g.sum() / (2 * math.pi * d * d)
    ang = om * T
    ex = xc + (x - xc) * math.cos(ang) - (y - yc) * math.sin(ang)
    ey = yc + (x - xc) * math.sin(ang) + (y - yc) * math.cos(ang)
    return float(np.max(np.hypot(xf - ex, yf - ey)))


def test_blob_pair_orbit_second_order():
    e1 = _pair_orbit(1.0, 0.05)
    e2 = _pair_orbit(1.0, 0.025)
    assert e2 < 1e-3
    assert 3.5 < e1 / e2 < 4.5


def test_linear_impulse_conserved():
    P = W.uniform(300, seed=8, sigma=0.05)
    i0 = np.array([P.gamma @ P.x, P.gamma @ P.y])
    scale = np.abs(P.gamma) @ np.hypot(P.x, P.y)
    xd, yd = A.advect(P.x, P.y, P.gamma, P.sigma, 0.002, 5, direct=True)
    assert np.max(np.abs(np.array([P.gamma @ xd, P.gamma @ yd]) - i0)) < 1e-13 * scale
    xf, yf = A.advect(P.x, P.y, P.gamma, P.sigma, 0.002, 5, p=20, levels=3)
    assert np.max(np.abs(np.array([P.gamma @ xf, P.gamma @ yf]) - i0)) < 1e-8 * scale
    assert np.max(np.hypot(xf - xd, yf - yd)) > 0.0


def _loops_velocity(x, y, g, s):
    n = len(x)
    u = np.zeros(n); v = np.zeros(n)
    for i in range(n):
        for j in range(n):
            dx, dy = x[i] - x[j], y[i] - y[j]
            r2 = dx * dx + dy * dy
            if r2 == 0.0:
                continue
            f = g[j] * (1.0 - math.exp(-r2 / (2 * s * s))) / (2 * math.pi * r2)
            u[i] -= f * dy
            v[i] += f * dx
    return u, v


def test_single_step_plain_loops_and_planted_mistake(monkeypatch):
    x = np.array([0.0, 0.3, -0.2]); y = np.array([0.0, 0.1, 0.25]); g = np.array([1.0, -0.7, 0.4])
    s, dt = 0.1, 0.05
    u1, v1 = _loops_velocity(x, y, g, s)
    u2, v2 = _loops_velocity(x + dt * u1, y + dt * v1, g, s)
    ex, ey = x + 0.5 * dt * (u1 + u2), y + 0.5 * dt * (v1 + v2)
    vel = lambda xx, yy: K.direct_velocity(xx, yy, g, s)
    hx, hy = A.heun_step(x, y, vel, dt)
    assert np.max(np.abs(hx - ex)) < 1e-15 and np.max(np.abs(hy - ey)) < 1e-15

    def euler_like(xx, yy, velocity, dt_):
        a, b = velocity(xx, yy)
        return xx + dt_ * a, yy + dt_ * b
    monkeypatch.setattr(A, "heun_step", euler_like)
    bx, by = A.advect(x, y, g, s, dt, 1, direct=True)
    assert np.max(np.hypot(bx - ex, by - ey)) > 1e-6
