"""Error metrics on the GPU (Section 5.1) against the oracle's definition.

vfmm_error_metrics reduces max |dW|, sum |dW|^2 and max |W_ref| over the
points; the binding turns them into (e_max, e_rms, max |W_ref|).  The oracle
(oracle.metrics.errors) is the plain NumPy definition.  Checked: several sizes
around the reduction's block and grid boundaries, a zero reference (absolute
errors, denominator 1), one element, and non-finite values, which must reach
the result (a NaN or an infinity anywhere makes e_max non-finite) instead of
being dropped by the maximum.
"""
import math

import numpy as np
import pytest

from gpu_util import dev, print_case, require_gpu
from oracle import metrics as M

pytestmark = pytest.mark.gpu


def _fields(n, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    ur = rng.normal(size=n) * scale
    vr = rng.normal(size=n) * scale
    u = ur + rng.normal(size=n) * 1e-7 * scale
    v = vr + rng.normal(size=n) * 1e-7 * scale
    return u, v, ur, vr


def _gpu(u, v, ur, vr):
    vf = require_gpu()
    return vf.error_metrics(dev(u), dev(v), dev(ur), dev(vr))


@pytest.mark.parametrize("n", [1, 2, 255, 256, 257, 65536, 131071, 512 * 256 + 1, 1_000_003])
def test_metrics_match_oracle(n):
    print_case("metrics", n=n)
    u, v, ur, vr = _fields(n, seed=n)
    em, er, den = _gpu(u, v, ur, vr)
    om, orr, oden = M.errors(u, v, ur, vr)
    # maxima are exact up to the last bit of hypot; the sum of squares is
    # reassociated by the reduction tree
    assert abs(den - oden) <= 1e-15 * oden
    assert abs(em - om) <= 1e-14 * om
    assert abs(er - orr) <= 1e-13 * orr


def test_metrics_zero_reference_is_absolute():
    print_case("metrics zero reference")
    n = 1000
    rng = np.random.default_rng(5)
    u = rng.normal(size=n); v = rng.normal(size=n)
    z = np.zeros(n)
    em, er, den = _gpu(u, v, z, z)
    om, orr, oden = M.errors(u, v, z, z)
    assert den == 1.0 and oden == 1.0
    assert abs(em - om) <= 1e-15 * om and abs(er - orr) <= 1e-13 * orr
    # identical fields: exactly zero error
    em, er, _ = _gpu(u, v, u, v)
    assert em == 0.0 and er == 0.0


def test_metrics_single_element():
    print_case("metrics single element")
    em, er, den = _gpu(np.array([3.0]), np.array([4.0]), np.array([0.0]), np.array([1.0]))
    # |dW| = |(3, 3)| = 3 sqrt 2, |W_ref| = 1
    assert den == 1.0
    assert abs(em - 3.0 * math.sqrt(2.0)) <= 1e-15 * em
    assert abs(er - 3.0 * math.sqrt(2.0)) <= 1e-15 * er
    assert M.errors([3.0], [4.0], [0.0], [1.0])[0] == pytest.approx(em, rel=1e-15)


@pytest.mark.parametrize("where", ["u", "v", "u_ref", "v_ref"])
@pytest.mark.parametrize("pos", [0, 777, 131071, 300_000 - 1])
def test_metrics_nan_propagates(where, pos):
    print_case("metrics nan", where=where, pos=pos)
    u, v, ur, vr = _fields(300_000, seed=11)
    arrs = {"u": u, "v": v, "u_ref": ur, "v_ref": vr}
    arrs[where][pos] = np.nan
    em, er, den = _gpu(u, v, ur, vr)
    om, orr, oden = M.errors(u, v, ur, vr)
    assert math.isnan(om) and math.isnan(orr)
    assert math.isnan(em), em
    assert math.isnan(er), er
    if where in ("u_ref", "v_ref"):
        assert math.isnan(den) and math.isnan(oden)
    else:
        assert den == oden


def test_metrics_infinity_propagates():
    print_case("metrics inf")
    u, v, ur, vr = _fields(50_000, seed=12)
    u[49_999] = np.inf
    em, er, den = _gpu(u, v, ur, vr)
    om, orr, _ = M.errors(u, v, ur, vr)
    assert math.isinf(om) and math.isinf(em) and math.isinf(er)


def test_error_field_matches_oracle_map():
    """Per-point log10 error field (Section 5 maps) against the oracle's map."""
    print_case("error field")
    vf = require_gpu()
    u, v, ur, vr = _fields(70_001, seed=13)
    u[5] = ur[5]; v[5] = vr[5]  # exact agreement: floored at -300
    f = vf.error_field(dev(u), dev(v), dev(ur), dev(vr)).cpu().numpy()
    ref = M.log10_error_map(u, v, ur, vr)
    assert f[5] == -300.0 and ref[5] == -300.0
    assert np.max(np.abs(f - ref)) <= 1e-13
