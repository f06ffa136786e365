"""Batched evaluation of uneven instances (vfmm_batch_*), through the C ABI.

Each instance is checked against the float64 oracle FMM at its own (p, levels)
(FP32 near field and, for p <= 16, FP32 expansions: 1e-6 of the maximum
velocity) and against the single-tree evaluation.  Graph replay must reproduce
eager runs bit for bit, also after the inputs change between replays (the
program's own work and synchronisations run between the replays).
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


def _instances(count, seed, n_range, levels=(2, 4)):
    insts = W.batch_instances(count, seed=seed, n_range=n_range, level_range=levels)
    out = []
    for P, p, L in insts:
        out.append(dict(P=P, x=dev(P.x), y=dev(P.y), gamma=dev(P.gamma), sigma=P.sigma, p=p, levels=L))
    return out


def test_batched_matches_oracle_and_single(vf):
    insts = _instances(10, seed=40, n_range=(300, 3000))
    # edge cases: single particle, no far field
    P1 = W.uniform(1, seed=1); P2 = W.uniform(500, seed=2, sigma=0.05)
    insts.append(dict(P=P1, x=dev(P1.x), y=dev(P1.y), gamma=dev(P1.gamma), sigma=0.02, p=5, levels=0))
    insts.append(dict(P=P2, x=dev(P2.x), y=dev(P2.y), gamma=dev(P2.gamma), sigma=0.05, p=8, levels=1))
    b = vf.Batch(insts)
    b.run()
    for i, d in enumerate(insts):
        P = d["P"]
        print_case("batched", i=i, n=P.n, p=d["p"], levels=d["levels"])
        u, v = host(b.u[i]), host(b.v[i])
        r = F.fmm_velocity(P.x, P.y, P.gamma, d["sigma"], d["p"], d["levels"])
        if np.max(np.hypot(r.u, r.v)) == 0:
            assert np.all(u == 0) and np.all(v == 0)
            continue
        assert rel_err(u, v, r.u, r.v)[0] < 1e-6
        t = vf.Tree(d["x"], d["y"], d["levels"], p_max=d["p"])
        us, vs = (host(a) for a in t.velocity(d["gamma"], d["sigma"], d["p"], vf.FP32))
        assert rel_err(u, v, us, vs)[0] < 1e-6


def test_graph_replay_matches_eager(vf):
    insts = _instances(24, seed=41, n_range=(2000, 20000), levels=(3, 6))
    b = vf.Batch(insts)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.run(use_graph=False)
        s.synchronize()
        eager = [(host(u).copy(), host(v).copy()) for u, v in zip(b.u, b.v)]
        for rep in range(3):
            for u in b.u:
                u.zero_()
            b.run(use_graph=True)
            s.synchronize()
            for i, (u, v) in enumerate(zip(b.u, b.v)):
                assert np.array_equal(host(u), eager[i][0]) and np.array_equal(host(v), eager[i][1]), (rep, i)
        # change the circulations in place: the replay must use the new values
        for d in insts:
            d["gamma"].mul_(-2.0)
        b.run(use_graph=True)
        s.synchronize()
        for i, (u, v) in enumerate(zip(b.u, b.v)):
            assert np.allclose(host(u), -2.0 * eager[i][0], rtol=1e-6, atol=1e-9 * np.abs(eager[i][0]).max())
        b.run(use_graph=False)
        s.synchronize()
        eager2 = [host(u).copy() for u in b.u]
        b.run(use_graph=True)
        s.synchronize()
        for i, u in enumerate(b.u):
            assert np.array_equal(host(u), eager2[i])


def test_batch_rejects_bad_instances(vf):
    P = W.uniform(100, seed=3)
    bad = [dict(x=dev(P.x), y=dev(P.y), gamma=dev(P.gamma), sigma=0.02, p=30, levels=3)]
    with pytest.raises(vf.VfmmError):
        vf.Batch(bad)
    bad[0]["p"] = 8; bad[0]["levels"] = 7
    with pytest.raises(vf.VfmmError):
        vf.Batch(bad)


def test_one_call_batched_equals_plan_and_run(vf):
    """vfmm_fmm_velocity_batched (plan, run, release in one call) gives the same
    bits as vfmm_batch_create + vfmm_batch_run."""
    insts = _instances(12, seed=43, n_range=(500, 6000), levels=(2, 5))
    b = vf.Batch(insts)
    b.run()
    ref = [(host(u).copy(), host(v).copy()) for u, v in zip(b.u, b.v)]
    for u in b.u:
        u.zero_()
    torch.cuda.synchronize()
    b.run_oneshot()
    for i, (u, v) in enumerate(zip(b.u, b.v)):
        assert np.array_equal(host(u), ref[i][0]) and np.array_equal(host(v), ref[i][1]), i


def test_full_sweep_batch_against_oracle(vf):
    """The parameter-sweep batch at its own size: 256 instances (N log-uniform in
    [2048, 65536], uniform or lattice, p in 5..20, L in 3..6; 4.9M particles)
    evaluated as one batch.  Every instance is compared with the float64 oracle
    FMM at its own (p, L) on 64 sampled targets, to 1e-6 of the sample's
    maximum velocity; the 64 instances with p > 16 take float64 shifts around
    a float32 M2L."""
    insts = _instances(256, seed=4, n_range=(2048, 65536), levels=(3, 6))
    b = vf.Batch(insts)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b.run(use_graph=True)  # graph replay, as the sweep is timed
    s.synchronize()
    worst = {False: 0.0, True: 0.0}
    for i, d in enumerate(insts):
        P = d["P"]
        if i % 32 == 0:
            print_case("batch_c4", i=i, n=P.n, p=d["p"], levels=d["levels"])
        tg = W.sample_targets(P.n, 64, seed=1000 + i)
        r = F.fmm_velocity(P.x, P.y, P.gamma, d["sigma"], d["p"], d["levels"], targets=tg)
        u, v = host(b.u[i]), host(b.v[i])
        e = rel_err(u[tg], v[tg], r.u, r.v)[0]
        worst[d["p"] > 16] = max(worst[d["p"] > 16], e)
        assert e < 1e-6, (i, P.n, d["p"], d["levels"], e)
    print("worst e_max: p <= 16 %.2e, p > 16 %.2e" % (worst[False], worst[True]))
    assert sum(d["p"] > 16 for d in insts) == 64
    b.close()


def test_substitution_floor_per_instance(vf):
    """vfmm_batch_substitution_bounds: per instance, the kernel-substitution
    floor of its bounding square (the oracle's root side) at its levels and
    sigma.  An instance whose leaves are narrower than sigma gets a floor above
    1, and its error against the direct sum (eq. 7) is indeed large, while an
    instance with leaves of 5 sigma or more has a negligible floor and meets
    the float32 bar against the direct sum."""
    from oracle import kernel as K
    from oracle import quadtree as Q
    Pw = W.uniform(3000, seed=51, sigma=0.01)   # root ~2, L=3: leaves ~25 sigma
    Pn = W.uniform(3000, seed=52, sigma=0.05)   # L=6: leaves ~0.6 sigma
    insts = [dict(P=Pw, p=16, levels=3), dict(P=Pn, p=12, levels=6)]
    for d in insts:
        P = d["P"]
        d.update(x=dev(P.x), y=dev(P.y), gamma=dev(P.gamma), sigma=P.sigma)
    b = vf.Batch(insts)
    with pytest.raises(vf.VfmmError):
        b.substitution_bounds()  # no run yet
    b.run()
    bounds = b.substitution_bounds()
    errs = []
    for i, d in enumerate(insts):
        P = d["P"]
        S = Q.root_square(P.x, P.y, None)[2]
        expect = vf.substitution_bound(S, d["levels"], P.sigma)[1]
        print_case("substitution floor", i=i, n=P.n, levels=d["levels"], bound=bounds[i])
        assert bounds[i] == pytest.approx(expect, rel=1e-14)
        ud, vd = K.direct_velocity(P.x, P.y, P.gamma, P.sigma)
        errs.append(rel_err(host(b.u[i]), host(b.v[i]), ud, vd)[0])
    assert bounds[0] < 1e-100 and errs[0] < 1e-6
    assert bounds[1] > 1.0 and errs[1] > 1e-3


def test_batched_symmetric_near_field(vf):
    """A batch planned with the symmetric near field (VFMM_TUNE_P2P_SYMMETRIC):
    every instance against the oracle FMM at its own (p, levels) (1e-6 of the
    maximum velocity), against the one-direction batch (within the two float32
    roundings), and graph replays against eager runs (the float64 atomic sums
    vary in order: 1e-13)."""
    insts = _instances(16, seed=47, n_range=(300, 12000), levels=(2, 5))
    P2 = W.clusters(9000, seed=48, sigma=0.004)  # several tiles per leaf
    insts.append(dict(P=P2, x=dev(P2.x), y=dev(P2.y), gamma=dev(P2.gamma), sigma=P2.sigma, p=12,
                      levels=3))
    saved = vf.get_tuning()
    try:
        vf.set_tuning(sym=0)
        b0 = vf.Batch(insts)
        vf.set_tuning(sym=1)
        b1 = vf.Batch(insts)
    finally:
        vf.set_tuning(**saved)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        b0.run()
        b1.run()
        s.synchronize()
        eager = [(host(b1.u[i]).copy(), host(b1.v[i]).copy()) for i in range(len(insts))]
        b1.run(use_graph=True)
        s.synchronize()
    for i, d in enumerate(insts):
        P = d["P"]
        print_case("batched_sym", i=i, n=P.n, p=d["p"], levels=d["levels"])
        u1, v1 = host(b1.u[i]), host(b1.v[i])
        u0, v0 = host(b0.u[i]), host(b0.v[i])
        r = F.fmm_velocity(P.x, P.y, P.gamma, d["sigma"], d["p"], d["levels"])
        e1 = rel_err(u1, v1, r.u, r.v)[0]
        e0 = rel_err(u0, v0, r.u, r.v)[0]
        assert e1 < 1e-6
        assert rel_err(u1, v1, u0, v0)[0] <= e0 + e1 + 1e-12
        assert rel_err(u1, v1, *eager[i])[0] < 1e-13
