"""Distance cut-off of the near field (Section 4.1's distance a), GPU vs the
float64 oracle, through the C ABI.

The library searches the rings of leaves at Chebyshev distance 2 .. D (D <= 4,
the smallest with D w_L >= radius) and clamps the radius to 4 w_L; the oracle
takes the effective radius and tests every pair.
Tolerances (normalised by the maximum velocity, Section 5.1): float64 vs the
oracle FMM with the same radius 1e-12 (near part 1e-13); float32 vs the
oracle 1e-6.  Radius 0 is bit-identical to the paper's split.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fmm as F
from oracle import kernel as K
from oracle import quadtree as qt
from tests.gpu_util import dev, host, print_case, rel_err, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vf():
    return require_gpu()


def _w(P, levels):
    return qt.box_side(qt.root_square(P.x, P.y), levels)


@pytest.mark.parametrize("levels,radius", [(3, 0.3), (3, 10.0), (4, 0.2), (3, "auto"), (2, "auto"),
                                           (4, 0.3), (4, 0.45), (5, 10.0), (5, "auto")])
def test_cutoff_fp64_matches_oracle(vf, levels, radius):
    """2000 uniform particles with sigma = 0.08: the leaf side is 0.8 to 6
    sigma, so the rings of leaves hold many pairs closer than the radius; the
    cases take 2, 3 and 4 rings (w_L = 0.25 at L = 3, 0.125 at L = 4, 0.0625 at
    L = 5, the square being about [-1, 1]^2)."""
    P = W.uniform(2000, seed=5, sigma=0.08)
    w = _w(P, levels)
    r_lib = vf.NEAR_RADIUS_AUTO if radius == "auto" else radius
    r_eff = min(math.sqrt(76.0) * P.sigma if radius == "auto" else radius, vf.NEAR_RINGS_MAX * w)
    print_case("cutoff_fp64", levels=levels, radius=radius, r_eff=r_eff)
    t = vf.Tree(dev(P.x), dev(P.y), levels, p_max=20)
    t.set_near_radius(r_lib)
    g = dev(P.gamma)
    u, v = (host(a) for a in t.velocity(g, P.sigma, 20, vf.FP64))
    un, vn = (host(a) for a in t.velocity(g, P.sigma, 20, vf.FP64, parts=vf.PART_NEAR))
    r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, 20, levels, radius=r_eff)
    assert rel_err(u, v, r.u, r.v)[0] < 1e-12
    den = np.max(np.hypot(r.u, r.v))
    assert np.max(np.hypot(un - r.near_u, vn - r.near_v)) / den < 1e-13
    # the correction is not empty
    r0 = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, 20, levels)
    assert np.max(np.hypot(r.u - r0.u, r.v - r0.v)) / den > 1e-11


def test_cutoff_at_points_and_fp32(vf):
    P = W.config("lattice_320")
    L, p = 6, 12
    w = _w(P, L)
    root = qt.root_square(P.x, P.y)
    xe, ye = W.eval_points(600, 4, root)
    print_case("cutoff_points", levels=L)
    t = vf.Tree(dev(P.x), dev(P.y), L, p_max=p)
    t.set_near_radius(vf.NEAR_RADIUS_AUTO)
    g = dev(P.gamma)
    u, v = (host(a) for a in t.velocity_at(g, P.sigma, p, dev(xe), dev(ye), vf.FP64))
    r = F.fmm_velocity_at(P.x, P.y, P.gamma, P.sigma, p, L, xe, ye,
                          radius=min(math.sqrt(76.0) * P.sigma, vf.NEAR_RINGS_MAX * w))
    assert rel_err(u, v, r.u, r.v)[0] < 1e-12
    u32, v32 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP32))
    idx = W.sample_targets(P.n, 500, 6)
    r32 = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, p, L, targets=idx,
                         radius=min(6.0 * P.sigma, vf.NEAR_RINGS_MAX * w))
    assert rel_err(u32[idx], v32[idx], r32.u, r32.v)[0] < 1e-6


def test_radius_zero_is_bit_identical(vf):
    P = W.config("lattice_320")
    t = vf.Tree(dev(P.x), dev(P.y), 5, p_max=12)
    g = dev(P.gamma)
    u0, v0 = (host(a) for a in t.velocity(g, P.sigma, 12, vf.FP32))
    t.set_near_radius(vf.NEAR_RADIUS_AUTO)
    t.set_near_radius(0.0)
    u1, v1 = (host(a) for a in t.velocity(g, P.sigma, 12, vf.FP32))
    assert np.array_equal(u0, u1) and np.array_equal(v0, v1)
    with pytest.raises(vf.VfmmError):
        t.set_near_radius(float("nan"))


def test_clusters_full_size_deeper_tree(vf):
    """N = 2^20 clustered particles one level deeper than the paper's split
    allows (L = 7: leaf side 4.3 sigma), p = 14, FP32, automatic radius
    (6 sigma): 256 sampled targets against the oracle FMM with the same
    radius (float64 path, 1e-12) and the oracle direct sum (FP32 path, 1e-6);
    without the cut-off the same tree misses 1e-6."""
    P = W.config("clusters_1m")
    L, p = 7, 14
    w = _w(P, L)
    print_case("clusters_1m_cutoff", n=P.n, levels=L, p=p)
    t = vf.Tree(dev(P.x), dev(P.y), L, p_max=p)
    g = dev(P.gamma)
    tg = W.sample_targets(P.n, 256, seed=31)
    ud, vd = K.direct_velocity(P.x, P.y, P.gamma, P.sigma, targets=tg)
    u0, v0 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP32))
    e_paper = rel_err(u0[tg], v0[tg], ud, vd)[0]
    t.set_near_radius(vf.NEAR_RADIUS_AUTO)
    u32, v32 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP32))
    u64, v64 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP64))
    r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, p, L, targets=tg,
                       radius=min(math.sqrt(76.0) * P.sigma, vf.NEAR_RINGS_MAX * w))
    assert rel_err(u64[tg], v64[tg], r.u, r.v)[0] < 1e-12
    e32 = rel_err(u32[tg], v32[tg], ud, vd)[0]
    print(f"clusters_1m L7 p14 fp32: paper split {e_paper:.3e}, with cut-off {e32:.3e}")
    assert e32 < 1e-6 < e_paper


def test_clusters_full_size_benchmark_configuration(vf):
    """The configuration the benchmark times on N = 2^20 clustered particles:
    p = 14, L = 7, FP32, radius sigma sqrt(2 ln 1e6) (where one pair's kernel
    difference equals the 1e-6 tolerance), the autotuned near-field launch
    shape; 256 sampled targets against the oracle FMM with that radius (float64
    path 1e-12, FP32 path 1e-6) and the oracle direct sum (FP32 path, 1e-6)."""
    from paper_0809_1810_amd import autotune as AT
    P = W.config("clusters_1m")
    L, p = 7, 14
    radius = P.sigma * math.sqrt(2.0 * math.log(1e6))
    assert radius < 2 * _w(P, L)  # not clamped
    saved = vf.get_tuning()
    AT.apply_for(P.n, L, cutoff=True)
    try:
        print_case("clusters_1m_bench_config", n=P.n, levels=L, p=p, radius=radius,
                   tuning=vf.get_tuning())
        t = vf.Tree(dev(P.x), dev(P.y), L, p_max=p)
        t.set_near_radius(radius)
        g = dev(P.gamma)
        u32, v32 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP32))
        u64, v64 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP64))
        t.close()
    finally:
        vf.set_tuning(**saved)
    tg = W.sample_targets(P.n, 256, seed=32)
    r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, p, L, targets=tg, radius=radius)
    assert rel_err(u64[tg], v64[tg], r.u, r.v)[0] < 1e-12
    assert rel_err(u32[tg], v32[tg], r.u, r.v)[0] < 1e-6
    ud, vd = K.direct_velocity(P.x, P.y, P.gamma, P.sigma, targets=tg)
    e32 = rel_err(u32[tg], v32[tg], ud, vd)[0]
    print(f"clusters_1m benchmark configuration: fp32 vs direct {e32:.3e}")
    assert e32 < 1e-6


@pytest.mark.parametrize("tile,waves", [(32, 2), (16, 4)])
def test_cutoff_on_every_tile_shape(vf, tile, waves):
    """The distance cut-off with two and four lanes per target (each source
    sub-stream tests its ring sources pair by pair): FP64 against the oracle
    FMM with the same radius (1e-12), FP32 within FP32 rounding of the
    64-target shape.  4000 uniform particles, L = 4 (leaf side
    2.5 sigma), radius 2.5 leaf sides: three rings of leaves."""
    P = W.uniform(4000, seed=21, sigma=0.05)
    L, p = 4, 16
    radius = 2.5 * _w(P, L)
    print_case("cutoff_tile_shape", tile=tile, waves=waves, radius=radius)
    g = dev(P.gamma)
    saved = vf.get_tuning()
    try:
        vf.set_tuning(tile=64, waves=4)
        t0 = vf.Tree(dev(P.x), dev(P.y), L, p_max=p)
        t0.set_near_radius(radius)
        u0, v0 = (host(a) for a in t0.velocity(g, P.sigma, p, vf.FP32))
        t0.close()
        vf.set_tuning(tile=tile, waves=waves)
        t = vf.Tree(dev(P.x), dev(P.y), L, p_max=p)
        t.set_near_radius(radius)
        u64, v64 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP64))
        u32, v32 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP32))
        t.close()
    finally:
        vf.set_tuning(**saved)
    r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, p, L, radius=radius)
    assert rel_err(u64, v64, r.u, r.v)[0] < 1e-12
    assert rel_err(u32, v32, u0, v0)[0] < 1e-6
    r0 = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, p, L)
    den = np.max(np.hypot(r.u, r.v))
    assert np.max(np.hypot(r.u - r0.u, r.v - r0.v)) / den > 1e-9  # the rings matter here
