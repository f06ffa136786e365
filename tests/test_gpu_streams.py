"""Ordering of an evaluation whose expansion sweeps run on the tree's own
stream, concurrently with the near field on the caller's stream, through the
C ABI.

* Back-to-back evaluations on a non-default stream with no host
  synchronisation between them (circulations changed in place between calls,
  results copied on the same stream) give the results of separate,
  synchronised evaluations; the sum is checked against the float64 oracle.
* Phase timing records 8 phases; a far-only evaluation skips the near-field
  phases.
* The far part alone of a tree without far field (L < 2) is zeros.
* Rebuild + evaluation captured into a graph replay like eager calls, also
  with the symmetric near field (its float64 sums cleared inside each replay).
"""
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


def test_back_to_back_calls_on_a_stream(vf):
    P = W.clusters(30000, seed=12, sigma=0.01)
    L, p = 5, 12
    print_case("streams_back_to_back", n=P.n, levels=L, p=p)
    t = vf.Tree(dev(P.x), dev(P.y), L, p_max=p)
    g = dev(P.gamma)
    ref = [host(a).copy() for a in t.velocity(g, P.sigma, p, vf.FP32)]
    s = torch.cuda.Stream()
    u = torch.empty(P.n, dtype=torch.float64, device="cuda")
    v = torch.empty_like(u)
    outs = []
    with torch.cuda.stream(s):
        for k in range(6):
            t.velocity(g, P.sigma, p, vf.FP32, out=(u, v))
            outs.append((u.clone(), v.clone()))
            g.mul_(-1.0)  # the next call must see the new circulations
    s.synchronize()
    for k, (uk, vk) in enumerate(outs):
        sign = 1.0 if k % 2 == 0 else -1.0
        assert np.array_equal(host(uk), sign * ref[0]) and np.array_equal(host(vk), sign * ref[1]), k
    r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, p, L)
    assert rel_err(ref[0], ref[1], r.u, r.v)[0] < 1e-6
    t.close()


def test_phase_timing(vf):
    P = W.uniform(20000, seed=13, sigma=0.01)
    t = vf.Tree(dev(P.x), dev(P.y), 5, p_max=10)
    g = dev(P.gamma)
    t.velocity(g, P.sigma, 10, vf.FP32)
    t.enable_timing(3)
    for _ in range(2):
        t.velocity(g, P.sigma, 10, vf.FP32)
    t.velocity(g, P.sigma, 10, vf.FP32, parts=vf.PART_FAR)
    ph = t.read_timing()
    assert len(ph) == 3 and all(len(x) == vf.N_PHASES == 8 for x in ph)
    assert all(val >= 0.0 for x in ph for val in x.values())
    assert ph[0]["p2p"] > 0.0 and ph[0]["l2p"] > 0.0 and ph[0]["m2l_l2l"] > 0.0
    assert ph[2]["p2p"] < 0.02 and ph[2]["p2p_sched"] < 0.02  # skipped: begin and end together
    t.close()


def test_far_part_of_a_shallow_tree_is_zero(vf):
    P = W.uniform(500, seed=14, sigma=0.05)
    t = vf.Tree(dev(P.x), dev(P.y), 1, p_max=8)
    u = torch.full((P.n,), float("nan"), dtype=torch.float64, device="cuda")
    v = torch.full_like(u, float("nan"))
    t.velocity(dev(P.gamma), P.sigma, 8, vf.FP32, parts=vf.PART_FAR, out=(u, v))
    assert np.all(host(u) == 0.0) and np.all(host(v) == 0.0)
    t.close()


def test_graph_capture_of_rebuild_and_velocity(vf):
    """The fork / join of the two streams is captured into a graph; every replay
    (eager work and synchronisation between replays) equals the eager result,
    also after the inputs change in place."""
    P = W.clusters(40000, seed=15, sigma=0.01)
    L, p = 5, 12
    print_case("streams_graph", n=P.n, levels=L, p=p)
    x, y, g = dev(P.x), dev(P.y), dev(P.gamma)
    t = vf.Tree(x, y, L, p_max=p)
    u = torch.empty(P.n, dtype=torch.float64, device="cuda")
    v = torch.empty_like(u)

    def step():
        t.rebuild(x, y)
        t.velocity(g, P.sigma, p, vf.FP32, out=(u, v))

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        step()
    torch.cuda.current_stream().wait_stream(s)
    eager = (host(u).copy(), host(v).copy())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        step()
    for rep in range(3):
        u.zero_()
        v.fill_(1.0)
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(u), eager[0]) and np.array_equal(host(v), eager[1]), rep
    # new positions and circulations, same buffers: replay = eager evaluation
    x.add_(1e-3)
    g.mul_(-0.5)
    graph.replay()
    torch.cuda.synchronize()
    got = (host(u).copy(), host(v).copy())
    step()
    assert np.array_equal(got[0], host(u)) and np.array_equal(got[1], host(v))
    t.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_capture_with_symmetric_near_field(vf, prec):
    """The symmetric near field inside a captured rebuild + evaluation: its
    float64 sums are cleared by a kernel of the schedule in every replay, so
    replays (with eager work and synchronisation between them, and after the
    circulations change in place) equal an eager evaluation to the rounding of
    those atomic sums (1e-13 of the maximum velocity in FP64, 1e-6 in FP32),
    and the FP64 result matches the oracle FMM on sampled targets to 1e-12."""
    P = W.clusters(60000, seed=16, sigma=0.005)
    L, p = 5, 12
    pr = vf.FP64 if prec == "fp64" else vf.FP32
    print_case("streams_graph_sym", n=P.n, levels=L, p=p, prec=prec)
    saved = vf.get_tuning()
    try:
        vf.set_tuning(tile=64, waves=1, sym=1)
        x, y, g = dev(P.x), dev(P.y), dev(P.gamma)
        t = vf.Tree(x, y, L, p_max=p)
        assert t.tuning()["sym"] == 1
        u = torch.empty(P.n, dtype=torch.float64, device="cuda")
        v = torch.empty_like(u)

        def step():
            t.rebuild(x, y)
            t.velocity(g, P.sigma, p, pr, out=(u, v))

        step()
        torch.cuda.synchronize()
        eager = (host(u).copy(), host(v).copy())
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            step()
        den = np.max(np.hypot(*eager))
        tol = 1e-13 if prec == "fp64" else 1e-6
        for rep in range(3):
            u.fill_(float("nan"))
            graph.replay()
            torch.cuda.synchronize()
            d = np.max(np.hypot(host(u) - eager[0], host(v) - eager[1])) / den
            assert d < tol, (rep, d)
        g.mul_(-0.5)
        graph.replay()
        torch.cuda.synchronize()
        got = (host(u).copy(), host(v).copy())
        step()
        torch.cuda.synchronize()
        d = np.max(np.hypot(got[0] - host(u), got[1] - host(v))) / np.max(np.hypot(host(u), host(v)))
        assert d < tol, d
        if prec == "fp64":
            tg = W.sample_targets(P.n, 64, seed=3)
            r = F.fmm_velocity(P.x, P.y, -0.5 * P.gamma, P.sigma, p, L, targets=tg)
            assert rel_err(got[0][tg], got[1][tg], r.u, r.v)[0] < 1e-12
        t.close()
    finally:
        vf.set_tuning(**saved)
