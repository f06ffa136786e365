"""Per-tree launch shapes and the opt-in finiteness check, through the C ABI.

* Two trees built under different process-wide tuning settings keep their own
  near-field launch shapes (tile size, waves per workgroup) whatever the
  settings are when they are evaluated; both match the float64 oracle.
* vfmm_tree_set_check_finite: finite inputs pass; a NaN or infinite
  circulation, a NaN position, or an evaluation point outside the root square
  (whose velocity is NaN by definition) give VFMM_ERR_NONFINITE; the check is
  refused on a stream under graph capture, and off again it lets the same
  evaluation through.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fmm as F
from tests.gpu_util import dev, host, print_case, rel_err, require_gpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vf():
    return require_gpu()


def test_two_trees_keep_their_own_launch_shape(vf):
    P = W.clusters(40000, seed=41, sigma=0.01)
    L, p = 5, 10
    print_case("per-tree tuning", n=P.n, levels=L, p=p)
    old = vf.get_tuning()
    x, y, g = dev(P.x), dev(P.y), dev(P.gamma)
    try:
        vf.set_tuning(tile=16, waves=8, m2l=0)
        ta = vf.Tree(x, y, L, p_max=p)
        vf.set_tuning(tile=64, waves=1, m2l=2)
        tb = vf.Tree(x, y, L, p_max=p)
        vf.set_tuning(tile=32, waves=2, m2l=1)  # neither tree follows later settings
        assert ta.tuning() == {"tile": 16, "waves": 8, "m2l": 0, "sym": 0}
        assert tb.tuning() == {"tile": 64, "waves": 1, "m2l": 2, "sym": 0}
        r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, p, L)
        for t in (ta, tb, ta):
            u, v = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP64))
            assert rel_err(u, v, r.u, r.v)[0] < 1e-12
        ta.rebuild(x, y)  # a rebuild keeps the tree's shape
        assert ta.tuning() == {"tile": 16, "waves": 8, "m2l": 0, "sym": 0}
        ta.close(); tb.close()
    finally:
        vf.set_tuning(**old)


def _nonfinite(vf, fn):
    with pytest.raises(vf.VfmmError) as ei:
        fn()
        torch.cuda.synchronize()
    assert ei.value.status == vf.vfmm.ERR_NONFINITE, ei.value
    return str(ei.value)


def test_finiteness_check(vf):
    P = W.uniform(5000, seed=42, sigma=0.02)
    L, p = 4, 10
    print_case("finiteness check", n=P.n, levels=L, p=p)
    x, y, g = dev(P.x), dev(P.y), dev(P.gamma)
    t = vf.Tree(x, y, L, p_max=p)
    t.set_check_finite(True)
    # finite: passes, result as without the check
    u, v = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP32))
    r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, p, L)
    assert rel_err(u, v, r.u, r.v)[0] < 1e-6
    for bad in (math.nan, math.inf, -math.inf):
        gb = g.clone()
        gb[1234] = bad
        msg = _nonfinite(vf, lambda: t.velocity(gb, P.sigma, p, vf.FP32))
        assert "1 non-finite input" in msg, msg
    # a NaN position: the tree built on it holds a NaN coordinate
    xb = x.clone()
    xb[77] = math.nan
    tn = vf.Tree(xb, y, L, p_max=p)
    tn.set_check_finite(True)
    _nonfinite(vf, lambda: tn.velocity(g, P.sigma, p, vf.FP64))
    tn.close()
    # separate evaluation points: one outside the root square gets NaN
    xt = dev(np.array([0.1, 0.2, 50.0])); yt = dev(np.array([0.0, 0.1, 0.0]))
    msg = _nonfinite(vf, lambda: t.velocity_at(g, P.sigma, p, xt, yt, vf.FP64))
    assert "2 non-finite velocity" in msg, msg
    ui, vi = (host(a) for a in t.velocity_at(g, P.sigma, p, xt[:2].contiguous(),
                                             yt[:2].contiguous(), vf.FP64))
    assert np.all(np.isfinite(ui)) and np.all(np.isfinite(vi))
    # refused under graph capture (it synchronises); allowed once switched off
    s = torch.cuda.Stream()
    uo = torch.empty(P.n, dtype=torch.float64, device="cuda"); vo = torch.empty_like(uo)
    graph = torch.cuda.CUDAGraph()
    with pytest.raises(vf.VfmmError) as ei:
        with torch.cuda.graph(graph, stream=s):
            t.velocity(g, P.sigma, p, vf.FP32, out=(uo, vo))
    assert ei.value.status == vf.vfmm.ERR_INVALID_ARG
    torch.cuda.synchronize()
    t.set_check_finite(False)
    gb = g.clone()
    gb[0] = math.nan
    un, vn = (host(a) for a in t.velocity(gb, P.sigma, p, vf.FP32))  # no check: no error
    assert np.isnan(un).any()
    t.close()
