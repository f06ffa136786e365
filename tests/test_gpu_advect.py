"""Advection with the FMM velocity (eq. 5, Heun's method), GPU vs the float64
oracle, through the C ABI.

Tolerances: float64 positions after 5 steps within 1e-12 of the oracle's
(absolute, positions of order 1); float32 displacements within 1e-6 of the
oracle's relative to the largest displacement; with the distance cut-off the
same bars against the oracle with the effective radius.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import advect as A
from oracle import quadtree as qt
from tests.gpu_util import dev, host, print_case, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vf():
    return require_gpu()


@pytest.mark.parametrize("levels,p,cut", [(3, 12, False), (2, 20, False), (3, 12, True)])
def test_advect_matches_oracle(vf, levels, p, cut):
    P = W.uniform(1500, seed=12, sigma=0.06)
    dt, steps = 0.002, 5
    print_case("advect", levels=levels, p=p, cut=cut)
    radius = 0.0
    if cut:
        # the oracle's effective radius; the bounding square changes with the
        # positions, so a radius below 2 w_L of every stage is used
        radius = 0.8 * 2 * qt.box_side(qt.root_square(P.x, P.y), levels)
    xo, yo = A.advect(P.x, P.y, P.gamma, P.sigma, dt, steps, p=p, levels=levels, radius=radius)
    x, y = dev(P.x), dev(P.y)
    t = vf.Tree(x, y, levels, p_max=p)
    t.set_near_radius(radius)
    t.advect(x, y, dev(P.gamma), P.sigma, p, dt, steps, vf.FP64)
    xg, yg = host(x), host(y)
    assert np.max(np.hypot(xg - xo, yg - yo)) < 1e-12
    x32, y32 = dev(P.x), dev(P.y)
    t.advect(x32, y32, dev(P.gamma), P.sigma, p, dt, steps, vf.FP32)
    d = np.hypot(xo - P.x, yo - P.y).max()
    assert np.max(np.hypot(host(x32) - xo, host(y32) - yo)) < 1e-6 * d


def test_advect_impulse_and_zero_steps(vf):
    P = W.uniform(3000, seed=13, sigma=0.04)
    x, y, g = dev(P.x), dev(P.y), dev(P.gamma)
    t = vf.Tree(x, y, 4, p_max=20)
    t.advect(x, y, g, P.sigma, 20, 0.002, 0, vf.FP64)
    assert np.array_equal(host(x), P.x)
    t.advect(x, y, g, P.sigma, 20, 0.002, 4, vf.FP64)
    scale = np.abs(P.gamma) @ np.hypot(P.x, P.y)
    i0 = np.array([P.gamma @ P.x, P.gamma @ P.y])
    i1 = np.array([P.gamma @ host(x), P.gamma @ host(y)])
    assert np.max(np.abs(i1 - i0)) < 1e-8 * scale
    with pytest.raises(vf.VfmmError):
        t.advect(x, y, g, P.sigma, 20, float("nan"), 1, vf.FP64)
