"""FMM on an adaptive quadtree (vfmm_fmm_velocity_adaptive) against the float64
oracle of the same reading (oracle/adaptive.py), through the C ABI.

* leaf capacity 0 (every leaf at the tree's leaf level): bit-identical to the
  uniform evaluation, in float64 and float32, with and without the cut-off;
* clustered particles with leaves on several levels: float64 within 1e-12 of
  the oracle (whole velocity and the near and far parts separately), float32
  within 1e-6, with and without the distance cut-off;
* a capacity at least N: the root is the only leaf, the result is the direct
  sum (eq. 7);
* the float64-shift path (p > 16) reads every level's local expansions.
"""
import numpy as np
import pytest

import workloads as W
from oracle import adaptive as A
from oracle import kernel as K
from tests.gpu_util import dev, host, print_case, rel_err, require_gpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vf():
    return require_gpu()


def _clusters(n, seed):
    return W.clusters(n, seed=seed, n_clusters=4, std_range=(0.02, 0.25), sigma=0.004)


@pytest.mark.parametrize("radius", [0.0, 0.02])
def test_capacity_zero_is_the_uniform_path(vf, radius):
    P = _clusters(30000, 61)
    L, p = 6, 12
    print_case("adaptive_s0", n=P.n, levels=L, radius=radius)
    t = vf.Tree(dev(P.x), dev(P.y), L, p_max=p)
    t.set_near_radius(radius)
    g = dev(P.gamma)
    for prec in (vf.FP64, vf.FP32):
        u, v = (host(a).copy() for a in t.velocity(g, P.sigma, p, prec))
        ua, va = (host(a) for a in t.velocity_adaptive(g, P.sigma, p, 0, prec))
        assert np.array_equal(ua, u) and np.array_equal(va, v), prec
    t.close()


@pytest.mark.parametrize("s,radius", [(64, 0.0), (16, 0.0), (48, 0.02)])
def test_adaptive_matches_oracle(vf, s, radius):
    P = _clusters(20000, 62)
    L, p = 7, 12
    print_case("adaptive_vs_oracle", n=P.n, levels=L, s=s, radius=radius)
    at = A.build_adaptive(P.x, P.y, L, s)
    levels = sorted({l for l, *_ in at.leaves})
    print("leaf levels", levels, "leaves", len(at.leaves))
    assert len(levels) >= 3
    tg = W.sample_targets(P.n, 1500, seed=s)
    r = A.fmm_velocity_adaptive(P.x, P.y, P.gamma, P.sigma, p, L, s, targets=tg, radius=radius)
    t = vf.Tree(dev(P.x), dev(P.y), L, p_max=p)
    t.set_near_radius(radius)
    g = dev(P.gamma)
    u, v = (host(a) for a in t.velocity_adaptive(g, P.sigma, p, s, vf.FP64))
    e = rel_err(u[tg], v[tg], r.u, r.v)[0]
    nu, nv = (host(a) for a in t.velocity_adaptive(g, P.sigma, p, s, vf.FP64, parts=vf.PART_NEAR))
    fu, fv = (host(a) for a in t.velocity_adaptive(g, P.sigma, p, s, vf.FP64, parts=vf.PART_FAR))
    den = np.max(np.hypot(r.u, r.v))
    en = np.max(np.hypot(nu[tg] - r.near_u, nv[tg] - r.near_v)) / den
    ef = np.max(np.hypot(fu[tg] - r.far_u, fv[tg] - r.far_v)) / den
    u32, v32 = (host(a) for a in t.velocity_adaptive(g, P.sigma, p, s, vf.FP32))
    e32 = rel_err(u32[tg], v32[tg], r.u, r.v)[0]
    t.close()
    print(f"fp64 {e:.2e} (near {en:.2e}, far {ef:.2e}), fp32 {e32:.2e}")
    assert e < 1e-12 and en < 1e-12 and ef < 1e-12
    assert e32 < 1e-6


def test_root_leaf_is_the_direct_sum(vf):
    P = _clusters(3000, 63)
    L, p = 5, 10
    print_case("adaptive_root_leaf", n=P.n, levels=L)
    t = vf.Tree(dev(P.x), dev(P.y), L, p_max=p)
    u, v = (host(a) for a in t.velocity_adaptive(dev(P.gamma), P.sigma, p, P.n, vf.FP64))
    t.close()
    ud, vd = K.direct_velocity(P.x, P.y, P.gamma, P.sigma)
    assert rel_err(u, v, ud, vd)[0] < 1e-13


def test_adaptive_high_order_shift64(vf):
    """p > 16 in float32: the leaves' local expansions of every level come from
    the float64 shifts."""
    P = _clusters(20000, 64)
    L, p, s = 6, 20, 40
    print_case("adaptive_shift64", n=P.n, levels=L, p=p, s=s)
    tg = W.sample_targets(P.n, 800, seed=5)
    r = A.fmm_velocity_adaptive(P.x, P.y, P.gamma, P.sigma, p, L, s, targets=tg)
    t = vf.Tree(dev(P.x), dev(P.y), L, p_max=p)
    u, v = (host(a) for a in t.velocity_adaptive(dev(P.gamma), P.sigma, p, s, vf.FP32))
    t.close()
    assert rel_err(u[tg], v[tg], r.u, r.v)[0] < 1e-6
