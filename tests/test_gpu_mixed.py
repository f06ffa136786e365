"""Reduced-precision evaluations (FP32 / BF16 / FP16 M2L on the matrix cores).

Compared with the float64 GPU evaluation at the same (p, levels), which isolates
rounding, and with the float64 oracle.  Tolerances:

* FP32 (scaled coefficients, FP32 matrix instructions): local expansions within
  1e-5 of the largest coefficient of their level, velocities within 1e-6 of
  the maximum velocity;
* BF16 / FP16 inputs with FP32 accumulation: measured error bars, bounded by
  the input rounding (2^-8 and 2^-11 relative) times the far-field share of the
  velocity; checked loosely and for ordering FP32 < FP16 < BF16.
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


@pytest.mark.parametrize("p,levels", [(3, 3), (12, 5), (17, 4), (40, 3)])
def test_fp32_mfma_locals_match_fp64(vf, p, levels):
    P = W.uniform(20000, seed=31, sigma=0.005)
    print_case("mfma_locals", p=p, levels=levels)
    t = vf.Tree(dev(P.x), dev(P.y), levels, p_max=p)
    g = dev(P.gamma)
    t.velocity(g, P.sigma, p, vf.FP64)
    le64 = [host(t.expansions(1, l, p)) for l in range(2, levels + 1)]
    me64 = [host(t.expansions(0, l, p)) for l in range(2, levels + 1)]
    u32, v32 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP32))
    le32 = [host(t.expansions(1, l, p)) for l in range(2, levels + 1)]
    me32 = [host(t.expansions(0, l, p)) for l in range(2, levels + 1)]
    for a, b in zip(me32, me64):
        assert np.max(np.abs(a - b)) <= 1e-5 * np.max(np.abs(b))
    for a, b in zip(le32, le64):
        assert np.max(np.abs(a - b)) <= 1e-5 * np.max(np.abs(b))
    u64, v64 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP64))
    assert rel_err(u32, v32, u64, v64)[0] < 1e-6


def test_reduced_precision_error_bars(vf):
    P = W.config("lattice_320")
    L, p = 5, 12
    print_case("bf16_fp16", n=P.n, levels=L, p=p)
    t = vf.Tree(dev(P.x), dev(P.y), L, p_max=p)
    g = dev(P.gamma)
    u64, v64 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP64))
    fu, fv = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP64, parts=vf.PART_FAR))
    far_share = np.max(np.hypot(fu, fv)) / np.max(np.hypot(u64, v64))
    errs = {}
    for name, prec in (("fp32", vf.FP32), ("fp16", vf.M2L_FP16), ("bf16", vf.M2L_BF16)):
        u, v = (host(a) for a in t.velocity(g, P.sigma, p, prec))
        errs[name] = rel_err(u, v, u64, v64)
    print("far share", far_share, {k: f"max {e[0]:.2e} rms {e[1]:.2e}" for k, e in errs.items()})
    assert errs["fp32"][0] < 1e-6
    assert errs["fp32"][0] < errs["fp16"][0] < errs["bf16"][0]
    assert errs["fp16"][0] < 30 * 2.0 ** -11 * far_share
    assert errs["bf16"][0] < 30 * 2.0 ** -8 * far_share
    # against the oracle too (same p, L)
    r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, p, L, targets=W.sample_targets(P.n, 300, 1))
    u32, v32 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP32))
    assert rel_err(u32[r.targets], v32[r.targets], r.u, r.v)[0] < 1e-6


def test_mode_switching_keeps_tables_consistent(vf):
    P = W.uniform(5000, seed=5, sigma=0.01)
    t = vf.Tree(dev(P.x), dev(P.y), 4, p_max=16)
    g = dev(P.gamma)
    ref = {}
    for prec in (vf.FP32, vf.M2L_BF16, vf.M2L_FP16):
        ref[prec] = [host(a) for a in t.velocity(g, P.sigma, 10, prec)]
    # interleave orders and modes: every repeat must reproduce bit for bit
    for p in (16, 10):
        for prec in (vf.M2L_FP16, vf.FP32, vf.M2L_BF16):
            out = [host(a) for a in t.velocity(g, P.sigma, p, prec)]
            if p == 10:
                assert np.array_equal(out[0], ref[prec][0]) and np.array_equal(out[1], ref[prec][1])


def test_mixed_precision_full_size_clusters(vf):
    """The mixed-precision configuration at its own size: N = 2^20 clustered
    particles, L = 7, p = 12, the paper's split, M2L in FP32, FP16 and BF16 on
    the matrix cores (FP32 accumulation) with FP32 near field.  Error bars
    against the FP64 FMM at the same (p, L) over all particles and against the
    FP64 direct sum on 4096 sampled targets; the 16-bit formats' error is bounded
    by their rounding of the far field's inputs."""
    P = W.config("clusters_1m")
    L, p = 7, 12
    print_case("mixed_full_size", n=P.n, levels=L, p=p)
    t = vf.Tree(dev(P.x), dev(P.y), L, p_max=p)
    g = dev(P.gamma)
    u64, v64 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP64))
    fu, fv = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP64, parts=vf.PART_FAR))
    far_share = np.max(np.hypot(fu, fv)) / np.max(np.hypot(u64, v64))
    tg = torch.from_numpy(W.sample_targets(P.n, 4096, seed=3)).cuda()
    ud, vd = (host(a) for a in vf.direct_velocity(dev(P.x), dev(P.y), g, P.sigma, targets=tg))
    tgh = tg.cpu().numpy()
    errs = {}
    for name, prec in (("fp32", vf.FP32), ("fp16", vf.M2L_FP16), ("bf16", vf.M2L_BF16)):
        u, v = (host(a) for a in t.velocity(g, P.sigma, p, prec))
        errs[name] = (rel_err(u, v, u64, v64), rel_err(u[tgh], v[tgh], ud, vd))
    t.close()
    print("far share", far_share, {k: f"vs FMM64 max {e[0][0]:.2e} rms {e[0][1]:.2e}; "
                                      f"vs direct max {e[1][0]:.2e} rms {e[1][1]:.2e}"
                                   for k, e in errs.items()})
    assert errs["fp32"][0][0] < 1e-6
    assert errs["fp32"][0][0] < errs["fp16"][0][0] < errs["bf16"][0][0]
    assert errs["fp16"][0][0] < 30 * 2.0 ** -11 * far_share
    assert errs["bf16"][0][0] < 30 * 2.0 ** -8 * far_share


@pytest.mark.parametrize("name,levels,p,ntg", [("lattice_320", 5, 12, 2000),
                                               ("clusters_1m", 7, 12, 4096)])
def test_16bit_m2l_against_oracle(vf, name, levels, p, ntg):
    """BF16 / FP16 M2L against the float64 oracle FMM at the same (p, L) on
    sampled targets, with per-result bars on the maximum and RMS error as a
    fraction of the far field's share of the velocity: the input rounding
    unit (2^-8 BF16, 2^-11 FP16) summed over up to 27 interaction-list
    contributions per level, about 4e-3 (BF16) and 4e-4 (FP16) at most and a
    third of that in RMS.  FP32 stays within 1e-6."""
    P = W.config(name)
    print_case("16bit_vs_oracle", workload=name, levels=levels, p=p, targets=ntg)
    tg = W.sample_targets(P.n, ntg, seed=17)
    r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, p, levels, targets=tg)
    den = np.max(np.hypot(r.u, r.v))
    far_share = np.max(np.hypot(r.far_u, r.far_v)) / den
    t = vf.Tree(dev(P.x), dev(P.y), levels, p_max=p)
    g = dev(P.gamma)
    errs = {}
    for nm, prec in (("fp32", vf.FP32), ("fp16", vf.M2L_FP16), ("bf16", vf.M2L_BF16)):
        u, v = (host(a) for a in t.velocity(g, P.sigma, p, prec))
        errs[nm] = rel_err(u[tg], v[tg], r.u, r.v)
    t.close()
    print("far share", far_share,
          {k: f"max {e[0]:.2e} rms {e[1]:.2e} (of far share: {e[0] / far_share:.2e}, "
              f"{e[1] / far_share:.2e})" for k, e in errs.items()})
    assert errs["fp32"][0] < 1e-6
    assert errs["fp16"][0] <= 4e-4 * far_share and errs["fp16"][1] <= 1.4e-4 * far_share
    assert errs["bf16"][0] <= 4e-3 * far_share and errs["bf16"][1] <= 1.4e-3 * far_share


@pytest.mark.parametrize("prec_name", ["fp32", "bf16"])
@pytest.mark.parametrize("p,levels", [(17, 4), (24, 5), (40, 3)])
def test_high_order_shifts_in_fp64(vf, prec_name, p, levels):
    """For p > 16 the reduced-precision evaluation runs P2M, M2M and L2L in
    float64 (M2L stays on the float32 / 16-bit matrix cores): its multipoles
    are those of the float64 evaluation bit for bit, its locals differ only by
    the M2L rounding, and the velocity matches the oracle FMM.  At p <= 16 the
    multipoles are float32."""
    P = W.clusters(30000, seed=33, sigma=0.004)
    prec = vf.PRECISIONS[prec_name]
    print_case("shift64", p=p, levels=levels, precision=prec_name)
    t = vf.Tree(dev(P.x), dev(P.y), levels, p_max=p)
    g = dev(P.gamma)
    t.velocity(g, P.sigma, p, vf.FP64)
    me64 = [host(t.expansions(0, l, p)) for l in range(2, levels + 1)]
    le64 = [host(t.expansions(1, l, p)) for l in range(2, levels + 1)]
    u, v = (host(a) for a in t.velocity(g, P.sigma, p, prec))
    me = [host(t.expansions(0, l, p)) for l in range(2, levels + 1)]
    le = [host(t.expansions(1, l, p)) for l in range(2, levels + 1)]
    for a, b in zip(me, me64):
        assert np.array_equal(a, b)
    bar = 2e-6 if prec_name == "fp32" else 2e-2
    for a, b in zip(le, le64):
        assert np.max(np.abs(a - b)) <= bar * np.max(np.abs(b))
    if prec_name == "fp32":
        tg = W.sample_targets(P.n, 300, seed=p)
        r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, p, levels, targets=tg)
        assert rel_err(u[tg], v[tg], r.u, r.v)[0] < 1e-6
        # at p = 16 the multipoles are float32: not the float64 ones
        t.velocity(g, P.sigma, 16, vf.FP64)
        m16 = host(t.expansions(0, levels, 16))
        t.velocity(g, P.sigma, 16, vf.FP32)
        assert not np.array_equal(host(t.expansions(0, levels, 16)), m16)
    t.close()


@pytest.mark.parametrize("p,levels", [(3, 2), (8, 5), (12, 7), (14, 6), (16, 8)])
def test_m2l_tile_variants_agree(vf, p, levels):
    """The FP32 matrix-core M2L tiles (operands in registers; sources staged in
    LDS with 4 or 8 waves) give the same local expansions up to float32
    summation order, every level (tiles of one row and of several class rows,
    levels 2 .. 8), and the float64 locals within 1e-5 of each level's
    largest coefficient."""
    P = W.clusters(60000, seed=71, n_clusters=5, sigma=0.003)
    print_case("m2l_tiles", p=p, levels=levels)
    old = vf.get_tuning()
    x, y, g = dev(P.x), dev(P.y), dev(P.gamma)
    les = {}
    try:
        for mode in (0, 1, 2):
            vf.set_tuning(m2l=mode)
            t = vf.Tree(x, y, levels, p_max=p)
            assert t.tuning()["m2l"] == mode
            t.velocity(g, P.sigma, p, vf.FP32, parts=vf.PART_FAR)
            les[mode] = [host(t.expansions(1, l, p)) for l in range(2, levels + 1)]
            if mode == 0:
                t.velocity(g, P.sigma, p, vf.FP64, parts=vf.PART_FAR)
                les[64] = [host(t.expansions(1, l, p)) for l in range(2, levels + 1)]
            t.close()
    finally:
        vf.set_tuning(**old)
    for mode in (1, 2):
        for a, b, c in zip(les[mode], les[0], les[64]):
            scale = np.max(np.abs(c))
            assert np.max(np.abs(a - b)) <= 2e-6 * scale
            assert np.max(np.abs(a - c)) <= 1e-5 * scale
