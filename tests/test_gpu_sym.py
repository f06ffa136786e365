"""Symmetric near field (VFMM_TUNE_P2P_SYMMETRIC), through the C ABI.

K_sigma is odd (eq. 6: K(-x) = -K(x)), so a pair of particles needs one kernel
value for both directions.  With the setting on, a tree with 64-particle tiles
evaluates each pair of two different tiles of the local list that hold 96 or
more particles together once, by the tile that comes first in (row, leaf,
tile) order, which adds the opposite contributions to the source particles;
the later tile skips the pair, and smaller pairs take one direction per tile.  Every pair must still be
counted exactly once in each direction, which the float64 comparison with the
oracle checks to 1e-12 of the maximum velocity (near part 1e-13): a missing or
doubled leaf pair, a wrong lane rotation or a sign error would show at the
1e-3 level.  Inputs with several tiles per leaf and ragged last tiles, the
domain edges, the distance cut-off (whose ring pairs are still taken one
direction at a time), float32 (1e-6 of the oracle, and within the two
roundings of the one-direction kernel's result), and the paths that must
ignore the setting (32-particle tiles, evaluation points, the adaptive tree).
"""
import numpy as np
import pytest

import workloads as W
from oracle import fmm as F
from oracle import quadtree as qt
from tests.gpu_util import dev, host, print_case, rel_err, require_gpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vf():
    return require_gpu()


@pytest.fixture()
def sym_on(vf):
    old = vf.get_tuning()
    vf.set_tuning(tile=64, sym=1)
    yield
    vf.set_tuning(**old)


@pytest.mark.parametrize("case,levels,waves", [("clusters_20k", 3, 1), ("clusters_20k", 5, 4),
                                               ("uniform_3k", 4, 8), ("uniform_3k", 1, 2),
                                               ("uniform_3k", 0, 1)])
def test_sym_fp64_matches_oracle(vf, sym_on, case, levels, waves):
    P = W.clusters(20000, seed=61, sigma=0.01) if case == "clusters_20k" else \
        W.uniform(3000, seed=62, sigma=0.03)
    vf.set_tuning(waves=waves)
    print_case("sym_fp64", case=case, n=P.n, levels=levels, waves=waves)
    t = vf.Tree(dev(P.x), dev(P.y), levels, p_max=16)
    assert t.tuning()["sym"] == 1
    g = dev(P.gamma)
    p = 16
    u, v = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP64))
    un, vn = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP64, parts=vf.PART_NEAR))
    r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, p, levels)
    assert rel_err(u, v, r.u, r.v)[0] < 1e-12
    den = np.max(np.hypot(r.u, r.v))
    assert np.max(np.hypot(un - r.near_u, vn - r.near_v)) / den < 1e-13
    t.close()


@pytest.mark.parametrize("levels,radius", [(4, "auto"), (5, 0.2)])
def test_sym_with_cutoff(vf, sym_on, levels, radius):
    """The rings beyond the local list keep one direction per tile; the local
    list's leaf pairs are symmetric.  float64 1e-12 and float32 1e-6."""
    import math
    P = W.uniform(4000, seed=63, sigma=0.05)
    w = qt.box_side(qt.root_square(P.x, P.y), levels)
    r_lib = vf.NEAR_RADIUS_AUTO if radius == "auto" else radius
    r64 = min(math.sqrt(76.0) * P.sigma if radius == "auto" else radius, vf.NEAR_RINGS_MAX * w)
    print_case("sym_cutoff", n=P.n, levels=levels, radius=radius)
    t = vf.Tree(dev(P.x), dev(P.y), levels, p_max=16)
    t.set_near_radius(r_lib)
    g = dev(P.gamma)
    u, v = (host(a) for a in t.velocity(g, P.sigma, 16, vf.FP64))
    r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, 16, levels, radius=r64)
    assert rel_err(u, v, r.u, r.v)[0] < 1e-12
    r32 = min(6.0 * P.sigma if radius == "auto" else radius, vf.NEAR_RINGS_MAX * w)
    u32, v32 = (host(a) for a in t.velocity(g, P.sigma, 16, vf.FP32))
    r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, 16, levels, radius=r32)
    assert rel_err(u32, v32, r.u, r.v)[0] < 1e-6
    t.close()


def test_sym_fp32_clusters_and_repeatability(vf, sym_on):
    """float32 against the oracle (1e-6) and against the one-direction kernel
    (the two differ by float32 rounding only); repeated evaluations differ at
    most by the float64 rounding of the atomically added sums."""
    P = W.clusters(60000, seed=64, sigma=0.005)
    L, p = 5, 14
    print_case("sym_fp32", n=P.n, levels=L, p=p)
    x, y, g = dev(P.x), dev(P.y), dev(P.gamma)
    t = vf.Tree(x, y, L, p_max=p)
    us, vs = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP32))
    us2, vs2 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP32))
    r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, p, L)
    assert rel_err(us, vs, r.u, r.v)[0] < 1e-6
    assert rel_err(us2, vs2, us, vs)[0] < 1e-13
    vf.set_tuning(sym=0)
    ta = vf.Tree(x, y, L, p_max=p)
    assert ta.tuning()["sym"] == 0
    ua, va = (host(a) for a in ta.velocity(g, P.sigma, p, vf.FP32))
    e_sym = rel_err(us, vs, r.u, r.v)[0]
    e_one = rel_err(ua, va, r.u, r.v)[0]
    d = rel_err(us, vs, ua, va)[0]
    print(f"float32 vs oracle: symmetric {e_sym:.3e}, one direction {e_one:.3e}; apart {d:.3e}")
    # two float32 roundings of the same sums: apart by no more than both errors
    assert d <= e_sym + e_one and e_sym < 1e-6 and e_one < 1e-6
    # a rebuild keeps the setting of the tree
    t.rebuild(x, y)
    assert t.tuning()["sym"] == 1
    ub, vb = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP32))
    assert rel_err(ub, vb, us, vs)[0] < 1e-13
    t.close(); ta.close()


def test_sym_ignored_where_it_does_not_apply(vf, sym_on):
    """32-particle tiles build a tree without it; evaluation points and the
    adaptive tree of a symmetric tree take both directions separately."""
    P = W.clusters(12000, seed=65, sigma=0.01)
    L, p = 4, 12
    print_case("sym_ignored", n=P.n, levels=L, p=p)
    x, y, g = dev(P.x), dev(P.y), dev(P.gamma)
    vf.set_tuning(tile=32)
    t32 = vf.Tree(x, y, L, p_max=p)
    assert t32.tuning()["sym"] == 0
    t32.close()
    vf.set_tuning(tile=64)
    t = vf.Tree(x, y, L, p_max=p)
    assert t.tuning()["sym"] == 1
    r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, p, L)
    u, v = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP64))
    assert rel_err(u, v, r.u, r.v)[0] < 1e-12
    # evaluation points at the particles: the one-direction path, same values
    ue, ve = (host(a) for a in t.velocity_at(g, P.sigma, p, x, y, vf.FP64))
    assert rel_err(ue, ve, r.u, r.v)[0] < 1e-12
    # adaptive tree with capacity 0 (every leaf at level L): the one-direction
    # near field, equal to the oracle
    ua, va = (host(a) for a in t.velocity_adaptive(g, P.sigma, p, 0, vf.FP64))
    assert rel_err(ua, va, r.u, r.v)[0] < 1e-12
    t.close()
