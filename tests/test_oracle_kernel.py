"""Pins of the oracle's kernels and direct sum (eq. 3, 4, 6, 7, 9, 32).

Each check compares the oracle with something derived independently of the
formula it implements: Stokes' theorem on the Gaussian cut-off of eq. 3, the
cross product of eq. 4, the exact convolution of two Gaussians (smoothed
Lamb-Oseen vortex of eq. 32), antisymmetry invariants, and plain loops.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import kernel as K


def _blob_azimuthal_from_vorticity(r, sigma, gamma=1.0):
    """u_theta(r) = (circulation inside radius r) / (2 pi r), integrating eq. 3."""
    zeta = lambda s: gamma * math.exp(-s * s / (2 * sigma * sigma)) / (2 * math.pi * sigma * sigma)
    circ, _ = integrate.quad(lambda s: zeta(s) * 2 * math.pi * s, 0.0, r, epsabs=0, epsrel=1e-13, limit=200)
    return circ / (2 * math.pi * r)


@pytest.mark.parametrize("r", [1e-4, 0.003, 0.01, 0.02, 0.05, 0.1, 0.5])
def test_single_blob_matches_stokes(r):
    sigma = 0.02
    # one source at the origin, one zero-circulation evaluation particle at
    # angle 0.7 rad, distance r
    th = 0.7
    x = np.array([0.0, r * math.cos(th)]); y = np.array([0.0, r * math.sin(th)])
    g = np.array([1.0, 0.0])
    u, v = K.direct_velocity(x, y, g, sigma)
    ut = _blob_azimuthal_from_vorticity(r, sigma)
    exp_u, exp_v = -ut * math.sin(th), ut * math.cos(th)
    assert abs(u[1] - exp_u) <= 1e-12 * abs(ut)
    assert abs(v[1] - exp_v) <= 1e-12 * abs(ut)
    # the zero-circulation particle induces nothing on the source
    assert u[0] == 0.0 and v[0] == 0.0


def test_singular_kernel_is_eq4_cross_product():
    rng = np.random.default_rng(7)
    d = rng.normal(size=(50, 2))
    d3 = np.concatenate([d, np.zeros((50, 1))], axis=1)
    k = np.array([0.0, 0.0, 1.0])
    ref = -np.cross(d3, k)[:, :2] / (2 * math.pi * np.sum(d * d, axis=1))[:, None]
    su, sv = K.singular_kernel(d[:, 0], d[:, 1])
    assert np.allclose(su, ref[:, 0], rtol=1e-15, atol=0)
    assert np.allclose(sv, ref[:, 1], rtol=1e-15, atol=0)
    # far away the regularised kernel equals the singular one
    ru, rv = K.regularized_kernel(d[:, 0] * 10, d[:, 1] * 10, 0.02)
    su, sv = K.singular_kernel(d[:, 0] * 10, d[:, 1] * 10)
    assert np.array_equal(ru, su) and np.array_equal(rv, sv)


def test_two_blobs_rotate_about_centroid():
    # two equal blobs co-rotate: velocities equal and opposite, perpendicular to
    # the joining line, magnitude u_theta(d) of the Stokes integral
    sigma, d = 0.02, 0.03
    x = np.array([-d / 2, d / 2]); y = np.array([0.0, 0.0]); g = np.array([1.0, 1.0])
    u, v = K.direct_velocity(x, y, g, sigma)
    ut = _blob_azimuthal_from_vorticity(d, sigma)
    assert abs(u[0]) < 1e-18 and abs(u[1]) < 1e-18
    assert abs(v[0] + ut) <= 1e-12 * ut and abs(v[1] - ut) <= 1e-12 * ut


def test_invariants_antisymmetry():
    P = W.uniform(600, seed=11, sigma=0.05)
    u, v = K.direct_velocity(P.x, P.y, P.gamma, P.sigma)
    scale = np.sum(np.abs(P.gamma)) * np.max(np.hypot(u, v))
    assert abs(np.dot(P.gamma, u)) <= 1e-13 * scale
    assert abs(np.dot(P.gamma, v)) <= 1e-13 * scale
    assert abs(np.dot(P.gamma, P.x * u + P.y * v)) <= 1e-13 * scale


def test_lamb_oseen_smoothed_closed_form():
    """Lattice sum of eq. 32 blobs vs the Gaussian-smoothed Lamb-Oseen vortex.

    Convolving the Lamb-Oseen vorticity (variance 2 nu t per axis) with the
    blob of eq. 3 (variance sigma^2) gives a Gaussian of variance
    2 nu t + sigma^2, whose velocity is
    Gamma0 (1 - exp(-r^2 / (4 nu t + 2 sigma^2))) / (2 pi r).
    """
    P = W.paper_lamb_oseen(3969)
    assert P.n == 3969
    assert abs(np.sum(P.gamma) - 1.0) < 1e-12
    u, v = K.direct_velocity(P.x, P.y, P.gamma, P.sigma)
    r = np.hypot(P.x, P.y)
    s2 = 4 * W.PAPER_NU * W.PAPER_T + 2 * P.sigma ** 2
    ut = np.where(r > 0, -np.expm1(-r * r / s2) / (2 * math.pi * np.where(r > 0, r, 1)), 0.0)
    with np.errstate(invalid="ignore", divide="ignore"):
        eu = np.where(r > 0, -ut * P.y / np.where(r > 0, r, 1), 0.0)
        ev = np.where(r > 0, ut * P.x / np.where(r > 0, r, 1), 0.0)
    err = np.max(np.hypot(u - eu, v - ev)) / np.max(np.hypot(eu, ev))
    assert err < 1e-11


def test_brute_force_loops_small():
    P = W.uniform(48, seed=5, sigma=0.1)
    # duplicate one particle: coincident distinct particles contribute zero
    x = np.append(P.x, P.x[3]); y = np.append(P.y, P.y[3]); g = np.append(P.gamma, 0.7)
    u, v = K.direct_velocity(x, y, g, P.sigma)
    ul, vl = K.direct_velocity_loop(list(x), list(y), list(g), P.sigma)
    assert np.allclose(u, ul, rtol=0, atol=1e-15 * np.max(np.abs(ul)))
    assert np.allclose(v, vl, rtol=0, atol=1e-15 * np.max(np.abs(vl)))


def test_direct_targets_subset():
    P = W.uniform(300, seed=2)
    u, v = K.direct_velocity(P.x, P.y, P.gamma, P.sigma)
    t = W.sample_targets(P.n, 37, seed=9)
    ut, vt = K.direct_velocity(P.x, P.y, P.gamma, P.sigma, targets=t)
    assert np.allclose(ut, u[t], rtol=1e-14, atol=0)
    assert np.allclose(vt, v[t], rtol=1e-14, atol=0)


def test_paper_lattice_sizes():
    want = [int(l) for l in open(__file__.replace("test_oracle_kernel.py", "golden/lattice_sizes.txt"))
            if l.strip() and not l.startswith("#")]
    got = [W.paper_lamb_oseen(n).n for n in want]
    assert got == want
    assert W.paper_single_source(8836).n == 8837


# ---------------------------------------------------------------- eq. 8: separate points

@pytest.mark.parametrize("r", [1e-4, 0.01, 0.03, 0.2])
def test_direct_at_single_source_matches_stokes(r):
    """One blob away from the origin, points on a circle around it: the
    velocity is tangential (counter-clockwise for positive circulation) with
    the magnitude given by Stokes' theorem on eq. 3.  A reversed offset
    (source minus point) flips the direction and fails here."""
    sigma, gam = 0.02, 1.7
    xs, ys = 0.3, -0.45
    th = np.linspace(0.0, 2 * math.pi, 7, endpoint=False) + 0.1
    xe = xs + r * np.cos(th); ye = ys + r * np.sin(th)
    u, v = K.direct_velocity_at(xe, ye, np.array([xs]), np.array([ys]), np.array([gam]), sigma)
    ut = gam * _blob_azimuthal_from_vorticity(r, sigma)
    assert np.max(np.abs(u - (-ut * np.sin(th)))) <= 1e-12 * ut
    assert np.max(np.abs(v - ut * np.cos(th))) <= 1e-12 * ut


def test_direct_at_equals_direct_at_the_particles():
    """Evaluated at the particles' own positions, eq. 8 is eq. 9: the point's
    own particle sits at zero offset and contributes nothing."""
    P = W.clusters(900, seed=21, n_clusters=3)
    u, v = K.direct_velocity(P.x, P.y, P.gamma, P.sigma)
    ua, va = K.direct_velocity_at(P.x, P.y, P.x, P.y, P.gamma, P.sigma)
    scale = np.max(np.hypot(u, v))
    assert np.max(np.abs(ua - u)) <= 1e-14 * scale
    assert np.max(np.abs(va - v)) <= 1e-14 * scale


def test_direct_at_brute_force_loop():
    """Plain Python loops over (point, particle) at off-particle points, with
    one point exactly on a particle."""
    P = W.uniform(40, seed=23, sigma=0.08)
    rng = np.random.default_rng(24)
    xe = np.append(rng.uniform(-1.2, 1.2, 15), P.x[7]); ye = np.append(rng.uniform(-1.2, 1.2, 15), P.y[7])
    ua, va = K.direct_velocity_at(xe, ye, P.x, P.y, P.gamma, P.sigma)
    for t in range(xe.shape[0]):
        su = sv = 0.0
        for j in range(P.n):
            dx = xe[t] - P.x[j]; dy = ye[t] - P.y[j]
            r2 = dx * dx + dy * dy
            if r2 == 0.0:
                continue
            r = math.sqrt(r2)
            mag = P.gamma[j] * (1.0 - math.exp(-r2 / (2 * P.sigma ** 2))) / (2 * math.pi * r)
            su += -mag * dy / r; sv += mag * dx / r
        assert abs(ua[t] - su) <= 1e-13 * max(1.0, abs(su))
        assert abs(va[t] - sv) <= 1e-13 * max(1.0, abs(sv))


def test_direct_at_far_point_is_point_vortex():
    """Far from every blob the kernel of eq. 6 is the point vortex of eq. 15:
    a single source seen from 50 sigma away gives Gamma / (2 pi r) exactly
    (the Gaussian factor is below the float64 rounding unit)."""
    sigma = 0.01
    u, v = K.direct_velocity_at(np.array([0.5]), np.array([0.0]), np.array([0.0]),
                                np.array([0.0]), np.array([2.0]), sigma)
    assert u[0] == 0.0
    assert abs(v[0] - 2.0 / (2 * math.pi * 0.5)) <= 2e-16 * v[0]
