"""Pins of the oracle FMM at separate evaluation points (eq. 8, Section 5.2) and
of the per-particle error map (Section 5).

* Section 5.2 set-up: one unit source at the centre of the domain, evaluation
  points on the paper's lattice.  Points whose leaf is adjacent to the source's
  leaf get the regularised kernel (eq. 6) in closed form; every other point
  gets the point-vortex velocity Gamma / (2 pi r) (eq. 15) in closed form, to
  the truncation error of p = 40.
* Brute force on a tiny set: for every point and every particle, with plain
  Python loops, the regularised kernel if their leaves are adjacent and the
  singular kernel otherwise (the p -> infinity limit of the FMM).
* Points outside the closed root square are NaN; points on its edge are not.
* A planted mistake (the near field taken with the singular kernel, or the
  far field evaluated about a shifted centre) breaks the brute-force pin.
"""
import math

import numpy as np

import workloads as W
from oracle import fmm as F
from oracle import metrics as M


def _leaf(xv, yv, root, level):
    """Leaf (ix, iy) by the floor-and-clamp rule, written out for scalars."""
    x0, y0, s = root
    m = 2 ** level
    ix = min(max(math.floor((xv - x0) / s * m), 0), m - 1)
    iy = min(max(math.floor((yv - y0) / s * m), 0), m - 1)
    return ix, iy


def _velocity_pair(dx, dy, gamma, sigma, regularised):
    r2 = dx * dx + dy * dy
    if r2 == 0.0:
        return 0.0, 0.0
    f = gamma / (2.0 * math.pi * r2)
    if regularised:
        f *= -math.expm1(-r2 / (2.0 * sigma * sigma))
    return -dy * f, dx * f


def _brute(x, y, g, sigma, xe, ye, root, level):
    out = []
    for k in range(len(xe)):
        ex, ey = _leaf(xe[k], ye[k], root, level)
        su = sv = 0.0
        for j in range(len(x)):
            sx, sy = _leaf(x[j], y[j], root, level)
            near = abs(ex - sx) <= 1 and abs(ey - sy) <= 1
            du, dv = _velocity_pair(xe[k] - x[j], ye[k] - y[j], g[j], sigma, near)
            su += du
            sv += dv
        out.append((su, sv))
    return np.array(out)


def test_single_source_on_paper_lattice_closed_form():
    """Section 5.2 with separate evaluation points: the only particle is the
    unit source at the domain centre; the 94 x 94 lattice is evaluated."""
    P = W.paper_single_source(8836)
    side = P.meta["side"]
    dom = (-side / 2, -side / 2, side)
    xe, ye = P.x[1:], P.y[1:]
    lev = 4
    r = F.fmm_velocity_at(P.x[:1], P.y[:1], P.gamma[:1], P.sigma, 40, lev, xe, ye, domain=dom)
    sx, sy = _leaf(0.0, 0.0, dom, lev)
    exp_u = np.empty_like(xe); exp_v = np.empty_like(xe)
    near = np.zeros(len(xe), bool)
    for k in range(len(xe)):
        ex, ey = _leaf(xe[k], ye[k], dom, lev)
        near[k] = abs(ex - sx) <= 1 and abs(ey - sy) <= 1
        exp_u[k], exp_v[k] = _velocity_pair(xe[k], ye[k], 1.0, P.sigma, near[k])
    assert near.sum() > 100 and (~near).sum() > 5000
    vmax = np.max(np.hypot(exp_u, exp_v))
    d = np.hypot(r.u - exp_u, r.v - exp_v)
    assert np.max(d[near]) <= 1e-15 * vmax
    assert np.max(d[~near]) <= 1e-13 * vmax


def _tiny_case(seed=11):
    rng = np.random.default_rng(seed)
    n = 40
    x = rng.uniform(-1, 1, n); y = rng.uniform(-1, 1, n); g = rng.uniform(-1, 1, n)
    dom = (-1.0, -1.0, 2.0)
    xe = list(rng.uniform(-1, 1, 20)); ye = list(rng.uniform(-1, 1, 20))
    # a point on a particle, points on leaf edges and on the root's upper edges
    xe += [x[3], -0.5, 0.25, 1.0, 1.0, -1.0]
    ye += [y[3], 0.0, -0.75, 1.0, 0.3, -1.0]
    return x, y, g, 0.05, np.array(xe), np.array(ye), dom


def test_brute_force_loops_tiny():
    x, y, g, s, xe, ye, dom = _tiny_case()
    for lev in (2, 3):
        r = F.fmm_velocity_at(x, y, g, s, 40, lev, xe, ye, domain=dom)
        ref = _brute(x, y, g, s, xe, ye, dom, lev)
        scale = np.max(np.hypot(ref[:, 0], ref[:, 1]))
        assert np.max(np.hypot(r.u - ref[:, 0], r.v - ref[:, 1])) <= 1e-12 * scale, lev


def test_at_particles_equals_evaluation_at_particles():
    P = W.config("uniform_1k")
    tg = np.arange(0, P.n, 7)
    a = F.fmm_velocity_at(P.x, P.y, P.gamma, P.sigma, 12, 3, P.x[tg], P.y[tg])
    b = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, 12, 3, targets=tg)
    assert np.allclose(a.u, b.u, rtol=0, atol=1e-14) and np.allclose(a.v, b.v, rtol=0, atol=1e-14)


def test_outside_root_is_nan_and_edges_are_not():
    x, y, g, s, _, _, dom = _tiny_case()
    xe = np.array([-1.0, 1.0, 1.0 + 1e-12, 0.0, -1.0 - 1e-12, 0.0, np.nan])
    ye = np.array([-1.0, 1.0, 0.0, 1.0 + 1e-9, 0.0, 0.0, 0.0])
    r = F.fmm_velocity_at(x, y, g, s, 10, 3, xe, ye, domain=dom)
    assert np.isfinite(r.u[[0, 1, 5]]).all() and np.isfinite(r.v[[0, 1, 5]]).all()
    assert np.isnan(r.u[[2, 3, 4, 6]]).all() and np.isnan(r.v[[2, 3, 4, 6]]).all()


def test_planted_mistakes_break_the_brute_force_pin(monkeypatch):
    x, y, g, s, xe, ye, dom = _tiny_case()
    ref = _brute(x, y, g, s, xe, ye, dom, 3)
    scale = np.max(np.hypot(ref[:, 0], ref[:, 1]))

    def err():
        r = F.fmm_velocity_at(x, y, g, s, 40, 3, xe, ye, domain=dom)
        return np.max(np.hypot(r.u - ref[:, 0], r.v - ref[:, 1])) / scale

    monkeypatch.setattr(F, "regularized_kernel", lambda dx, dy, sigma: F.singular_kernel(dx, dy))
    assert err() > 1e-6
    monkeypatch.undo()
    good = F.l2p
    monkeypatch.setattr(F, "l2p", lambda b, c, z: good(b, c + 0.25, z))
    assert err() > 1e-6
    monkeypatch.undo()
    assert err() <= 1e-12


def test_log10_error_map_special_values():
    ur = np.array([3.0, 0.0, -4.0, 1.0]); vr = np.array([4.0, 1.0, 3.0, 0.0])  # max |W| = 5
    u = ur.copy(); v = vr.copy()
    u[1] += 5e-7                  # |dW| = 5e-7 -> log10(1e-7) = -7
    v[2] -= 0.5; u[2] += 1.2      # |dW| = 1.3 -> log10(0.26)
    m = M.log10_error_map(u, v, ur, vr)
    assert m[0] == -300.0 and m[3] == -300.0
    assert abs(m[1] + 7.0) < 1e-12
    assert abs(m[2] - math.log10(1.3 / 5.0)) < 1e-12
