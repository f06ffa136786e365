"""Regularised and singular Biot-Savart kernels and the direct sums.

Test infrastructure (see ``oracle/__init__``).

Paper references (Cruz & Barba 2008):

* eq. 6  -- K_sigma(x) = (-y, x) (1 - exp(-r^2 / 2 sigma^2)) / (2 pi r^2),
  the velocity kernel of a Gaussian vortex blob (cut-off of eq. 3);
* eq. 7 / eq. 9 -- u(x_i) = sum_{j != i} Gamma_j K_sigma(x_i - x_j), evaluated
  at the particles with no self-interaction;
* eq. 15 / eq. 27 -- the singular kernel K' = (-y, x) / (2 pi r^2) used for the
  far field.

Readings:

* the self term and coincident distinct particles contribute zero (the limit
  of eq. 6 as r -> 0 is zero);
* ``1 - exp(-a)`` is evaluated as ``-expm1(-a)``, the same function computed
  without cancellation for small a.
"""
from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def regularized_kernel(dx, dy, sigma):
    """eq. 6: velocity at offset (dx, dy) from a unit-circulation Gaussian blob."""
    dx = np.asarray(dx, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    r2 = dx * dx + dy * dy
    pos = r2 > 0.0
    safe = np.where(pos, r2, 1.0)
    coef = np.where(pos, -np.expm1(-safe / (2.0 * sigma * sigma)) / (TWO_PI * safe), 0.0)
    return -dy * coef, dx * coef


def singular_kernel(dx, dy):
    """eq. 15 / eq. 27: the point-vortex kernel (-y, x) / (2 pi r^2); zero at r = 0."""
    dx = np.asarray(dx, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    r2 = dx * dx + dy * dy
    pos = r2 > 0.0
    safe = np.where(pos, r2, 1.0)
    coef = np.where(pos, 1.0 / (TWO_PI * safe), 0.0)
    return -dy * coef, dx * coef


def _chunk_size(n_sources: int) -> int:
    return max(1, (1 << 22) // max(1, n_sources))


def direct_velocity(x, y, gamma, sigma, targets=None):
    """eq. 7 / eq. 9: exact regularised velocity at the particles (or a subset).

    ``targets`` -- optional int array of particle indices; the self term of each
    target is excluded (j != i).  Returns (u, v) float64 arrays of len(targets)
    (or N).
    """
    x = np.asarray(x, np.float64); y = np.asarray(y, np.float64)
    g = np.asarray(gamma, np.float64)
    n = x.shape[0]
    tidx = np.arange(n) if targets is None else np.asarray(targets, dtype=np.int64)
    u = np.zeros(tidx.shape[0]); v = np.zeros(tidx.shape[0])
    cs = _chunk_size(n)
    for s in range(0, tidx.shape[0], cs):
        ti = tidx[s:s + cs]
        dx = x[ti, None] - x[None, :]
        dy = y[ti, None] - y[None, :]
        ku, kv = regularized_kernel(dx, dy, sigma)
        ku[np.arange(ti.shape[0]), ti] = 0.0  # j != i
        kv[np.arange(ti.shape[0]), ti] = 0.0
        u[s:s + cs] = ku @ g
        v[s:s + cs] = kv @ g
    return u, v


def direct_velocity_at(xe, ye, x, y, gamma, sigma):
    """eq. 8 with the kernel of eq. 6: velocity at separate evaluation points."""
    xe = np.asarray(xe, np.float64); ye = np.asarray(ye, np.float64)
    g = np.asarray(gamma, np.float64)
    u = np.zeros(xe.shape[0]); v = np.zeros(xe.shape[0])
    cs = _chunk_size(np.asarray(x).shape[0])
    for s in range(0, xe.shape[0], cs):
        ku, kv = regularized_kernel(xe[s:s + cs, None] - x[None, :],
                                    ye[s:s + cs, None] - y[None, :], sigma)
        u[s:s + cs] = ku @ g
        v[s:s + cs] = kv @ g
    return u, v


def direct_velocity_loop(x, y, gamma, sigma):
    """eq. 9 written as two plain Python loops (only for tiny N)."""
    n = len(x)
    u = [0.0] * n; v = [0.0] * n
    for i in range(n):
        su = 0.0; sv = 0.0
        for j in range(n):
            if j == i:
                continue
            dx = x[i] - x[j]; dy = y[i] - y[j]
            r2 = dx * dx + dy * dy
            if r2 == 0.0:
                continue
            c = -math.expm1(-r2 / (2.0 * sigma * sigma)) / (TWO_PI * r2)
            su += gamma[j] * (-dy) * c
            sv += gamma[j] * dx * c
        u[i] = su; v[i] = sv
    return np.array(u), np.array(v)
