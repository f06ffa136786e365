"""FMM at separate evaluation points (eq. 8), the direct sum there and the error
field (Section 5), GPU vs the float64 oracle, through the C ABI.

Tolerances (normalised by the maximum velocity, Section 5.1): float64 FMM vs
the oracle FMM at the same (p, L) 1e-12; float64 direct vs the oracle direct
1e-13; float32 FMM vs the oracle's float64 FMM 1e-6.  The error field agrees
with the oracle's log10 map to 1e-12 where it is above the -300 floor and
exactly at the floor.  Points outside the root square are NaN on both sides.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fmm as F
from oracle import kernel as K
from oracle import metrics as M
from oracle import quadtree as qt
from tests.gpu_util import dev, host, print_case, rel_err, require_gpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vf():
    return require_gpu()


def _points(P, k, seed, extra=True):
    root = qt.root_square(P.x, P.y)
    xe, ye = W.eval_points(k, seed, root)
    if extra:
        x0, y0, s = root
        # on particles, on leaf edges of every level, on the root's edges, outside
        ex = [P.x[5], P.x[17], x0 + 0.5 * s, x0 + 0.25 * s, x0 + s, x0, x0 + s * (1 + 1e-9), x0 - 1.0]
        ey = [P.y[5], P.y[17], y0 + 0.5 * s, y0 + 0.75 * s, y0 + s, y0 + 0.3 * s, y0, y0]
        xe = np.concatenate([xe, ex]); ye = np.concatenate([ye, ey])
    return root, xe, ye


def _cmp_nan(a, b):
    na, nb = np.isnan(a), np.isnan(b)
    assert np.array_equal(na, nb)
    return ~na


@pytest.mark.parametrize("p,levels", [(12, 3), (20, 4), (6, 2)])
def test_velocity_at_matches_oracle(vf, p, levels):
    P = W.config("uniform_1k")
    _, xe, ye = _points(P, 700, seed=p)
    print_case("velocity_at", p=p, levels=levels, n_targets=len(xe))
    t = vf.Tree(dev(P.x), dev(P.y), levels, p_max=p)
    g, xt, yt = dev(P.gamma), dev(xe), dev(ye)
    u, v = (host(a) for a in t.velocity_at(g, P.sigma, p, xt, yt, vf.FP64))
    un, vn = (host(a) for a in t.velocity_at(g, P.sigma, p, xt, yt, vf.FP64, parts=vf.PART_NEAR))
    uf, vf_ = (host(a) for a in t.velocity_at(g, P.sigma, p, xt, yt, vf.FP64, parts=vf.PART_FAR))
    u32, v32 = (host(a) for a in t.velocity_at(g, P.sigma, p, xt, yt, vf.FP32))
    r = F.fmm_velocity_at(P.x, P.y, P.gamma, P.sigma, p, levels, xe, ye)
    ok = _cmp_nan(u, r.u)
    _cmp_nan(u32, r.u)
    assert ok.sum() == len(xe) - 2
    assert rel_err(u[ok], v[ok], r.u[ok], r.v[ok])[0] < 1e-12
    den = np.max(np.hypot(r.u[ok], r.v[ok]))
    assert np.max(np.hypot(un - r.near_u, vn - r.near_v)[ok]) / den < 1e-13
    assert np.max(np.hypot(uf - r.far_u, vf_ - r.far_v)[ok]) / den < 1e-12
    assert rel_err(u32[ok], v32[ok], r.u[ok], r.v[ok])[0] < 1e-6


def test_velocity_at_particles_equals_velocity(vf):
    """At the particles' own positions, in their order, the evaluation-point
    path reproduces the particle path bit for bit (same sort, same tiles)."""
    P = W.config("lattice_320")
    L, p = 5, 12
    print_case("at_particles", n=P.n)
    x, y, g = dev(P.x), dev(P.y), dev(P.gamma)
    saved = vf.get_tuning()
    try:
        vf.set_tuning(sym=0)  # both paths one direction per pair: the same sums
        t = vf.Tree(x, y, L, p_max=p)
        for prec in (vf.FP64, vf.FP32, vf.M2L_BF16):
            u0, v0 = (host(a) for a in t.velocity(g, P.sigma, p, prec))
            u1, v1 = (host(a) for a in t.velocity_at(g, P.sigma, p, x, y, prec))
            assert np.array_equal(u0, u1) and np.array_equal(v0, v1), prec
        # a subset in a shuffled order: float64 agrees to rounding
        idx = np.random.default_rng(4).permutation(P.n)[:5000]
        u0, v0 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP64))
        u1, v1 = (host(a) for a in t.velocity_at(g, P.sigma, p, dev(P.x[idx]), dev(P.y[idx]),
                                                 vf.FP64))
        assert rel_err(u1, v1, u0[idx], v0[idx])[0] < 1e-15
        # a tree with the symmetric near field: its particle path sums the
        # same pairs in another order, the points keep one direction per pair
        vf.set_tuning(tile=64, sym=1)
        ts = vf.Tree(x, y, L, p_max=p)
        u0, v0 = (host(a) for a in ts.velocity(g, P.sigma, p, vf.FP64))
        u1, v1 = (host(a) for a in ts.velocity_at(g, P.sigma, p, x, y, vf.FP64))
        assert rel_err(u1, v1, u0, v0)[0] < 1e-14
    finally:
        vf.set_tuning(**saved)


def test_section52_single_source_on_lattice(vf):
    """Section 5.2: the unit source at the domain centre, the 94 x 94 lattice as
    evaluation points (p = 20, L = 4), against the oracle."""
    P = W.paper_single_source(8836)
    side = P.meta["side"]
    dom = (-side / 2, -side / 2, side)
    print_case("section52")
    t = vf.Tree(dev(P.x[:1]), dev(P.y[:1]), 4, p_max=20, domain=dom)
    u, v = (host(a) for a in t.velocity_at(dev(P.gamma[:1]), P.sigma, 20, dev(P.x[1:]),
                                           dev(P.y[1:]), vf.FP64))
    r = F.fmm_velocity_at(P.x[:1], P.y[:1], P.gamma[:1], P.sigma, 20, 4, P.x[1:], P.y[1:],
                          domain=dom)
    assert rel_err(u, v, r.u, r.v)[0] < 1e-12


def test_direct_velocity_at_matches_oracle(vf):
    P = W.config("uniform_1k")
    _, xe, ye = _points(P, 900, seed=9, extra=False)
    xe = np.concatenate([xe, P.x[:3]]); ye = np.concatenate([ye, P.y[:3]])
    print_case("direct_at", n_targets=len(xe))
    u, v = (host(a) for a in vf.direct_velocity_at(dev(P.x), dev(P.y), dev(P.gamma), P.sigma,
                                                    dev(xe), dev(ye)))
    ur, vr = K.direct_velocity_at(xe, ye, P.x, P.y, P.gamma, P.sigma)
    assert rel_err(u, v, ur, vr)[0] < 1e-13
    # at the particles themselves it equals the particle direct sum (self term zero)
    ud, vd = K.direct_velocity(P.x, P.y, P.gamma, P.sigma, targets=np.arange(3))
    assert rel_err(u[-3:], v[-3:], ud, vd)[0] < 1e-13


def test_error_field_matches_oracle(vf):
    rng = np.random.default_rng(8)
    n = 3000
    ur = rng.normal(size=n); vr = rng.normal(size=n)
    u = ur + rng.normal(size=n) * 10.0 ** rng.uniform(-14, -2, n)
    v = vr.copy()
    u[:10] = ur[:10]; v[:10] = vr[:10]           # exact agreement: floor
    u[10] = np.nan                                 # NaN propagates
    print_case("error_field", n=n)
    f = host(vf.error_field(dev(u), dev(v), dev(ur), dev(vr)))
    m = M.log10_error_map(u, v, ur, vr)
    assert np.isnan(f[10]) and np.isnan(m[10])
    keep = np.ones(n, bool); keep[10] = False
    assert np.all(f[:10] == -300.0) and np.all(m[:10] == -300.0)
    assert np.max(np.abs(f[keep] - m[keep])) < 1e-12


def test_edge_cases(vf):
    P = W.config("uniform_1k")
    t = vf.Tree(dev(P.x), dev(P.y), 3, p_max=8)
    g = dev(P.gamma)
    e = torch.empty(0, dtype=torch.float64, device="cuda")
    u, v = t.velocity_at(g, P.sigma, 8, e, e, vf.FP64)
    assert u.numel() == 0
    root = qt.root_square(P.x, P.y)
    # one point; all points outside; many points in one leaf (several tiles)
    cases = {
        "single": (np.array([0.1]), np.array([-0.2])),
        "outside": (np.array([root[0] - 1, root[0] + 2 * root[2]]), np.array([0.0, 0.0])),
        "one_leaf": (0.3 + 1e-3 * np.arange(300) / 300, np.full(300, 0.31)),
    }
    for name, (xe, ye) in cases.items():
        print_case("edge", case=name)
        u, v = (host(a) for a in t.velocity_at(g, P.sigma, 8, dev(xe), dev(ye), vf.FP64))
        r = F.fmm_velocity_at(P.x, P.y, P.gamma, P.sigma, 8, 3, xe, ye)
        ok = _cmp_nan(u, r.u)
        if ok.any():
            assert rel_err(u[ok], v[ok], r.u[ok], r.v[ok])[0] < 1e-12
    with pytest.raises(vf.VfmmError):
        small = torch.empty(256, dtype=torch.uint8, device="cuda")
        t.velocity_at(g, P.sigma, 8, dev(np.zeros(100)), dev(np.zeros(100)), vf.FP64,
                      workspace=small)


def test_clusters_full_size_lattice_sampled(vf):
    """N = 2^20 clustered particles at the benchmark's tuned configuration
    (p = 14, L = 6, FP32) evaluated on a 1024^2 lattice covering the root
    square; 256 sampled points against the oracle FMM (float64 path to 1e-12)
    and the oracle direct sum (FP32 path to 1e-6)."""
    P = W.config("clusters_1m")
    L, p = 6, 14
    root = qt.root_square(P.x, P.y)
    xe, ye = W.eval_lattice(1024, root)
    print_case("clusters_1m_lattice", n=P.n, n_targets=len(xe), levels=L, p=p)
    t = vf.Tree(dev(P.x), dev(P.y), L, p_max=p)
    g, xt, yt = dev(P.gamma), dev(xe), dev(ye)
    u32, v32 = (host(a) for a in t.velocity_at(g, P.sigma, p, xt, yt, vf.FP32))
    u64, v64 = (host(a) for a in t.velocity_at(g, P.sigma, p, xt, yt, vf.FP64))
    assert np.isfinite(u32).all() and np.isfinite(u64).all()
    sel = W.sample_targets(len(xe), 256, seed=5)
    r = F.fmm_velocity_at(P.x, P.y, P.gamma, P.sigma, p, L, xe[sel], ye[sel])
    assert rel_err(u64[sel], v64[sel], r.u, r.v)[0] < 1e-12
    ud, vd = K.direct_velocity_at(xe[sel], ye[sel], P.x, P.y, P.gamma, P.sigma)
    e32 = rel_err(u32[sel], v32[sel], ud, vd)[0]
    e64 = rel_err(u64[sel], v64[sel], ud, vd)[0]
    print(f"clusters_1m on 1024^2 lattice: fp32 vs direct {e32:.3e}, fp64 vs direct {e64:.3e}")
    assert e32 < 1e-6
