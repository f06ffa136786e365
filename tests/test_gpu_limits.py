"""The largest tree depth and expansion order the library accepts, GPU vs the
float64 oracle on sampled targets, through the C ABI.

* L = 12 (4^12 = 16.8M leaves, 6 GB of workspace at p = 8) on 20,000 clustered
  particles: most leaves are empty, the particles sit in a few hundred
  thousand of them.
* p = 40 on the 320^2 lattice at L = 5.

Tolerances (normalised by the maximum velocity, Section 5.1): float64 1e-12,
float32 1e-6 against the oracle FMM with the same (p, L).
"""
import numpy as np
import pytest

import workloads as W
from oracle import fmm as F
from tests.gpu_util import dev, host, print_case, rel_err, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vf():
    return require_gpu()


def _check(vf, P, L, p, ntg, seed):
    tg = W.sample_targets(P.n, ntg, seed=seed)
    r = F.fmm_velocity(P.x, P.y, P.gamma, P.sigma, p, L, targets=tg)
    t = vf.Tree(dev(P.x), dev(P.y), L, p_max=p)
    g = dev(P.gamma)
    u, v = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP64))
    e64 = rel_err(u[tg], v[tg], r.u, r.v)[0]
    u32, v32 = (host(a) for a in t.velocity(g, P.sigma, p, vf.FP32))
    e32 = rel_err(u32[tg], v32[tg], r.u, r.v)[0]
    t.close()
    print(f"L={L} p={p}: fp64 {e64:.2e}, fp32 {e32:.2e}")
    assert e64 < 1e-12 and e32 < 1e-6


def test_deepest_tree(vf):
    P = W.clusters(20000, seed=21, sigma=1e-4)
    print_case("limits_levels", n=P.n, levels=12, p=8)
    _check(vf, P, 12, 8, 150, 4)


def test_highest_order(vf):
    P = W.config("lattice_320")
    print_case("limits_order", n=P.n, levels=5, p=40)
    _check(vf, P, 5, 40, 200, 5)
