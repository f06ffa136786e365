"""Selector network kernels vs the float64 oracle, through the C ABI.

Tolerances: with float32 activations (bf16 = 0) forward outputs and gradients
match the oracle to 1e-5 relative (norm-wise); with bfloat16 weights, inputs
and activations to 2e-2; one Adam step to 1e-6.  Training is deterministic
(bit-identical parameters from two runs).
"""
import numpy as np
import pytest

import workloads as W
from oracle import mlp as OM
from tests.gpu_util import dev, host, print_case, require_gpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vf():
    return require_gpu()


def _bf16(a):
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float32).numpy().astype(np.float64)


def _case(seed, B):
    rng = np.random.default_rng(seed)
    theta = OM.init_params(seed).astype(np.float32).astype(np.float64)
    X = rng.normal(size=(B, 10)).astype(np.float32).astype(np.float64)
    T = rng.normal(size=B).astype(np.float32).astype(np.float64)
    return theta, X, T


@pytest.mark.parametrize("B", [1, 31, 32, 100, 257])
def test_forward_matches_oracle(vf, B):
    print_case("mlp_forward", B=B)
    theta, X, _ = _case(1, B)
    y32 = host(vf.mlp_forward(dev(theta, torch.float32), dev(X, torch.float32), bf16=False))
    yr, _ = OM.forward(theta, X)
    assert np.max(np.abs(y32 - yr)) <= 1e-5 * max(1.0, np.max(np.abs(yr)))
    yb = host(vf.mlp_forward(dev(theta, torch.float32), dev(X, torch.float32), bf16=True))
    assert np.max(np.abs(yb - yr)) <= 2e-2 * max(1.0, np.max(np.abs(yr)))


@pytest.mark.parametrize("B", [7, 64, 200])
def test_gradient_matches_oracle(vf, B):
    print_case("mlp_gradient", B=B)
    theta, X, T = _case(2, B)
    g_ref = OM.gradient(theta, X, T)
    l_ref = OM.loss(theta, X, T)
    tr = vf.MlpTrainer(dev(theta, torch.float32), B)
    g32, l32 = (host(a) for a in tr.gradient(dev(X, torch.float32), dev(T, torch.float32), bf16=False))
    assert np.linalg.norm(g32 - g_ref) <= 1e-5 * np.linalg.norm(g_ref)
    assert abs(l32[0] - l_ref) <= 1e-5 * l_ref
    gb, lb = (host(a) for a in tr.gradient(dev(X, torch.float32), dev(T, torch.float32), bf16=True))
    # bf16 reference: the oracle evaluated at bf16-rounded weights and inputs
    g_rb = OM.gradient(_bf16(theta), _bf16(X), T)
    assert np.linalg.norm(gb - g_rb) <= 2e-2 * np.linalg.norm(g_rb)
    assert np.linalg.norm(gb - g_ref) <= 5e-2 * np.linalg.norm(g_ref)


def test_adam_step_matches_oracle(vf):
    theta, X, T = _case(3, 64)
    tr = vf.MlpTrainer(dev(theta, torch.float32), 64)
    g = host(tr.gradient(dev(X, torch.float32), dev(T, torch.float32), bf16=False)[0]).astype(np.float64)
    tr.adam(1e-3)
    th1 = host(tr.params)
    ref, m, v = OM.adam_step(theta, np.zeros_like(theta), np.zeros_like(theta), g, 1, 1e-3)
    assert np.max(np.abs(th1 - ref)) <= 1e-6
    tr.gradient(dev(X, torch.float32), dev(T, torch.float32), bf16=False)
    g2 = host(tr.grad).astype(np.float64)
    tr.adam(1e-3)
    ref2, _, _ = OM.adam_step(ref, m, v, g2, 2, 1e-3)
    assert np.max(np.abs(host(tr.params) - ref2)) <= 2e-6


def test_training_is_deterministic_and_learns(vf):
    rng = np.random.default_rng(5)
    X = rng.normal(size=(512, 10)).astype(np.float32)
    T = (np.sin(X[:, 0]) + 0.5 * X[:, 1] * X[:, 2]).astype(np.float32)
    outs = []
    for _ in range(2):
        tr = vf.MlpTrainer(dev(OM.init_params(0), torch.float32), 128)
        Xd, Td = dev(X), dev(T)
        l0 = None
        for step in range(200):
            s = (step % 4) * 128
            loss = tr.step(Xd[s:s + 128].contiguous(), Td[s:s + 128].contiguous(), 3e-3)
            if l0 is None:
                l0 = float(host(loss)[0])
        outs.append(host(tr.params))
        yv = host(vf.mlp_forward(tr.params, Xd))
        assert np.mean((yv - T) ** 2) < 0.2 * l0
    assert np.array_equal(outs[0], outs[1])


def test_particle_stats_and_features(vf):
    P = W.clusters(5000, seed=7)
    print_case("stats", n=P.n)
    st = vf.particle_stats(dev(P.x), dev(P.y), dev(P.gamma))
    g = P.gamma
    ref = [P.x.sum(), (P.x ** 2).sum(), P.y.sum(), (P.y ** 2).sum(), g.sum(), (g ** 2).sum(),
           np.abs(g).sum(), np.abs(g).max(), P.x.min(), P.x.max(), P.y.min(), P.y.max()]
    assert np.allclose(st, ref, rtol=1e-12, atol=1e-12)
    from oracle import quadtree as qt
    side = qt.root_square(P.x, P.y)[2]
    for p, L in ((4, 2), (12, 5), (20, 7)):
        for radius in (0.0, -1.0, 5.26 * P.sigma):
            f = vf.selector_features(st, P.n, P.sigma, p, L, radius)
            fr = OM.features(P.x, P.y, P.gamma, P.sigma, p, L, side, radius)
            assert np.allclose(f, fr, rtol=1e-6, atol=1e-6)


def _time_eval(vf, x, y, g, sigma, p, L, prec, reps=3, radius=0.0):
    times = []
    for _ in range(reps + 1):
        e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        t = vf.Tree(x, y, L, p_max=p)
        t.set_near_radius(radius)
        t.velocity(g, sigma, p, prec)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
        t.close()
    return float(np.median(times[1:]))


def test_selector_gain_over_conservative_choice(vf):
    """Held-out instances (a seed the training data did not use): the learned
    choice, audited by the direct sum, always meets tol = 1e-6 and costs less
    in total than the conservative float64 evaluation (p = 20, deepest level
    with leaf side >= 8 sigma) that one would run without the network.  The
    network's own share of the gain is isolated by timing the conservative
    (p, L) in float32 as well: the same arithmetic, only the parameters
    differ."""
    from paper_0809_1810_amd import selector as S
    weights = S.load_weights()
    rng = np.random.default_rng(12345)
    tol = 1e-6
    t_sel = t_cons = t_cons32 = 0.0
    chosen = 0
    for i in range(12):
        P = S.random_instance(rng, (2 ** 13, 2 ** 17))
        x, y, g = dev(P.x), dev(P.y), dev(P.gamma)
        r = S.select_and_audit(x, y, g, P.sigma, tol, weights=weights, n_audit=2048, seed=i)
        print_case("selector", i=i, n=P.n, kind=P.meta["kind"],
                   **{k: r[k] for k in ("p", "levels", "radius", "fallback", "precision")},
                   emax=f"{r['audit_emax']:.2e}")
        assert r["audit_emax"] <= tol
        prec = vf.FP32 if r["precision"] == "fp32" else vf.FP64
        t_sel += _time_eval(vf, x, y, g, P.sigma, r["p"], r["levels"], prec, radius=r["radius"])
        probe = vf.Tree(x, y, 0, p_max=1)
        side = float(probe.arrays()[0][2].item())
        pc, Lc = S.conservative_choice(side, P.sigma, P.n)
        t_cons += _time_eval(vf, x, y, g, P.sigma, pc, Lc, vf.FP64)
        t_cons32 += _time_eval(vf, x, y, g, P.sigma, pc, Lc, vf.FP32)
        chosen += not r["fallback"]
    print(f"selected total {t_sel:.2f} ms vs conservative FP64 {t_cons:.2f} ms and conservative "
          f"FP32 {t_cons32:.2f} ms; network choices {chosen}/12")
    assert chosen >= 6
    assert t_sel < 0.7 * t_cons
    assert t_sel < t_cons32  # the parameters alone, at equal precision


def test_selection_on_the_2048_lattice(vf):
    """The selection workload at its own size: the Lamb-Oseen pair on a 2048^2
    lattice (N = 4,194,304), tol = 1e-6, audited by the FP64 direct sum on 8192
    sampled targets; the chosen evaluation is also checked against the oracle
    direct sum on 32 other targets."""
    from paper_0809_1810_amd import selector as S
    from oracle import kernel as K
    P = W.config("lattice_2048")
    x, y, g = dev(P.x), dev(P.y), dev(P.gamma)
    r = S.select_and_audit(x, y, g, P.sigma, 1e-6, weights=S.load_weights(), n_audit=8192, seed=7)
    print_case("selector_lattice_2048", n=P.n,
               **{k: r[k] for k in ("p", "levels", "radius", "fallback", "precision")},
               emax=f"{r['audit_emax']:.2e}")
    assert r["audit_emax"] <= 1e-6
    prec = vf.FP32 if r["precision"] == "fp32" else vf.FP64
    t = vf.Tree(x, y, r["levels"], p_max=r["p"])
    t.set_near_radius(r["radius"])
    u, v = (host(a) for a in t.velocity(g, P.sigma, r["p"], prec))
    t.close()
    tg = W.sample_targets(P.n, 32, seed=8)
    ud, vd = K.direct_velocity(P.x, P.y, P.gamma, P.sigma, targets=tg)
    # normalised by the largest velocity of the whole field (the audit's
    # denominator comes from its own 8192 targets)
    umax = float(np.max(np.hypot(u, v)))
    assert float(np.max(np.hypot(u[tg] - ud, v[tg] - vd))) / umax <= 1e-6
