"""Pins of the adaptive-quadtree oracle (oracle/adaptive.py).

Checked against things the adaptive code does not compute itself: the tree
rules (counts, splits, leaves tiling the particles), the list-cover invariant
(every pair covered exactly once), the special cases that reduce to
already-pinned routines (one leaf: the direct sum; every leaf at Lmax: the
uniform FMM), the p -> infinity limit (p = 40 equals the brute-force hybrid
sum, also written as plain Python loops), and planted mistakes.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import adaptive as A
from oracle import fmm as F
from oracle import kernel as K
from oracle import quadtree as qt


def _clusters(n=2500, seed=51):
    return W.clusters(n, seed=seed, n_clusters=3, std_range=(0.03, 0.2), sigma=0.01)


def test_tree_rules():
    P = _clusters()
    at = A.build_adaptive(P.x, P.y, 6, 40)
    seen = np.zeros(P.n, np.int64)
    levels = set()
    for l, ix, iy, n in at.leaves:
        cx, cy = qt.leaf_coords(P.x, P.y, at.root, l)
        inside = (cx == ix) & (cy == iy)
        assert inside.sum() == n
        assert n <= 40 or l == 6
        seen += inside
        levels.add(l)
        if l > 0:  # the parent was split: it held more than s particles
            px, py = qt.parent(ix, iy)
            qx, qy = qt.leaf_coords(P.x, P.y, at.root, l - 1)
            assert ((qx == px) & (qy == py)).sum() > 40
    assert np.all(seen == 1)  # every particle in exactly one leaf
    assert len(levels) >= 3   # a genuinely non-uniform tree
    # the leaves tile the root square: their areas add up to it
    assert math.isclose(sum(4.0 ** -l for l, *_ in at.leaves), 1.0, rel_tol=1e-15)


def test_every_pair_covered_exactly_once():
    P = _clusters(1200, seed=52)
    at = A.build_adaptive(P.x, P.y, 5, 25)
    m = 1 << at.lmax
    for l, ix, iy, n in at.leaves:
        if n == 0:
            continue
        for sy in range(m):
            for sx in range(m):
                assert len(A.covering(at, l, ix, iy, sx, sy)) == 1, (l, ix, iy, sx, sy)


def test_single_leaf_is_the_direct_sum():
    P = _clusters(600, seed=53)
    r = A.fmm_velocity_adaptive(P.x, P.y, P.gamma, P.sigma, 10, 5, P.n)  # the root is a leaf
    u, v = K.direct_velocity(P.x, P.y, P.gamma, P.sigma)
    scale = np.max(np.hypot(u, v))
    assert np.max(np.abs(r.u - u)) <= 1e-15 * scale and np.max(np.abs(r.v - v)) <= 1e-15 * scale


@pytest.mark.parametrize("radius", [0.0, 0.03])
def test_all_leaves_at_lmax_is_the_uniform_fmm(radius):
    P = _clusters(1500, seed=54)
    r = A.fmm_velocity_adaptive(P.x, P.y, P.gamma, P.sigma, 12, 4, 0, radius=radius)
    rad = min(radius, 4 * qt.box_side(qt.root_square(P.x, P.y), 4))
    ru = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, 12, 4, radius=rad)
    scale = np.max(np.hypot(ru.u, ru.v))
    assert np.max(np.hypot(r.u - ru.u, r.v - ru.v)) <= 1e-14 * scale


@pytest.mark.parametrize("radius", [0.0, 0.035])
def test_p40_equals_the_adaptive_hybrid(radius):
    P = _clusters(2000, seed=55)
    r = A.fmm_velocity_adaptive(P.x, P.y, P.gamma, P.sigma, 40, 6, 30, radius=radius)
    hu, hv = A.hybrid_velocity_adaptive(P.x, P.y, P.gamma, P.sigma, 6, 30, radius=radius)
    scale = np.max(np.hypot(hu, hv))
    assert np.max(np.hypot(r.u - hu, r.v - hv)) <= 1e-13 * scale
    # the error falls with p
    e = []
    for p in (6, 12, 20):
        rp = A.fmm_velocity_adaptive(P.x, P.y, P.gamma, P.sigma, p, 6, 30, radius=radius)
        e.append(np.max(np.hypot(rp.u - hu, rp.v - hv)) / scale)
    assert e[0] > 10 * e[1] > 100 * e[2]


def test_hybrid_against_plain_loops():
    """The adaptive hybrid sum written as two plain Python loops: for each
    target, the level of its leaf, then every source by the near rule."""
    P = _clusters(180, seed=56)
    lmax, s, radius = 4, 12, 0.05
    hu, hv = A.hybrid_velocity_adaptive(P.x, P.y, P.gamma, P.sigma, lmax, s, radius=radius)
    x0, y0, S = qt.root_square(P.x, P.y)

    def box(xv, yv, l):
        m = 2 ** l
        return (min(max(math.floor((xv - x0) / S * m), 0), m - 1),
                min(max(math.floor((yv - y0) / S * m), 0), m - 1))

    def count(l, b):
        return sum(1 for j in range(P.n) if box(P.x[j], P.y[j], l) == b)

    for i in range(P.n):
        l = 0
        while l < lmax and count(l, box(P.x[i], P.y[i], l)) > s:
            l += 1
        bi = box(P.x[i], P.y[i], l)
        rl = min(radius, 4 * S / 2 ** l)
        su = sv = 0.0
        for j in range(P.n):
            if j == i:
                continue
            dx = P.x[i] - P.x[j]; dy = P.y[i] - P.y[j]
            r2 = dx * dx + dy * dy
            if r2 == 0.0:
                continue
            bj = box(P.x[j], P.y[j], l)
            near = (abs(bj[0] - bi[0]) <= 1 and abs(bj[1] - bi[1]) <= 1) or r2 < rl * rl
            f = (1.0 - math.exp(-r2 / (2 * P.sigma ** 2))) if near else 1.0
            su += -P.gamma[j] * dy * f / (2 * math.pi * r2)
            sv += P.gamma[j] * dx * f / (2 * math.pi * r2)
        assert abs(hu[i] - su) <= 1e-13 * max(1.0, abs(su))
        assert abs(hv[i] - sv) <= 1e-13 * max(1.0, abs(sv))


def test_planted_mistakes_are_caught(monkeypatch):
    """Two plausible mistakes in the adaptive evaluation: a local list without
    the neighbours (the leaf alone), and the local expansion evaluated about a
    shifted centre.  The p = 40 pin rejects both."""
    P = _clusters(1500, seed=57)
    hu, hv = A.hybrid_velocity_adaptive(P.x, P.y, P.gamma, P.sigma, 5, 30)
    scale = np.max(np.hypot(hu, hv))

    real_local = qt.local_list
    monkeypatch.setattr(A.qt, "local_list", lambda level, ix, iy: real_local(level, ix, iy)[:1])
    r = A.fmm_velocity_adaptive(P.x, P.y, P.gamma, P.sigma, 40, 5, 30)
    assert np.max(np.hypot(r.u - hu, r.v - hv)) > 1e-6 * scale
    monkeypatch.setattr(A.qt, "local_list", real_local)

    real_l2p = F.l2p
    monkeypatch.setattr(A.F, "l2p", lambda b, centre, zz: real_l2p(b, centre + 0.01, zz))
    r = A.fmm_velocity_adaptive(P.x, P.y, P.gamma, P.sigma, 40, 5, 30)
    assert np.max(np.hypot(r.u - hu, r.v - hv)) > 1e-6 * scale
