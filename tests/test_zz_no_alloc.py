"""vfmm_error_metrics_noalloc (the library's own device array for the partial
sums, no scratch argument) against vfmm_error_metrics (caller's scratch),
through the C ABI: two calls in a row, the second with a smaller input, must
each give the values of the entry point with a scratch buffer; the metrics
agree with the oracle's definition as well.
"""
import ctypes as C

import numpy as np
import pytest

from oracle import metrics as M
from tests.gpu_util import dev, print_case, require_gpu

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _fields(n, seed):
    rng = np.random.default_rng(seed)
    ur = rng.normal(size=n); vr = rng.normal(size=n)
    return ur + 1e-6 * rng.normal(size=n), vr + 1e-6 * rng.normal(size=n), ur, vr


def _raw(lib, fn, arrays, n, out, scratch=None):
    args = [a.data_ptr() for a in arrays] + [n]
    if scratch is not None:
        args.append(scratch.data_ptr())
    args += [out.data_ptr(), C.c_void_p(torch.cuda.current_stream().cuda_stream)]
    assert fn(*args) == 0, lib.vfmm_last_error()
    torch.cuda.synchronize()
    return out.cpu().numpy().copy()


def test_noalloc_metrics_match_scratch_entry_point():
    vf = require_gpu()
    lib = vf.lib()
    scratch = torch.empty(int(lib.vfmm_metrics_scratch_bytes()), dtype=torch.uint8, device="cuda")
    out_a = torch.empty(3, dtype=torch.float64, device="cuda")
    out_b = torch.empty(3, dtype=torch.float64, device="cuda")
    # the second call is smaller: fewer blocks write partial sums, and what the
    # first call left in the library's array must not leak into the result
    for n, seed in ((1_000_003, 1), (3_001, 2), (1, 3)):
        print_case("noalloc metrics", n=n)
        u, v, ur, vr = _fields(n, seed)
        arrays = [dev(u), dev(v), dev(ur), dev(vr)]
        ref = _raw(lib, lib.vfmm_error_metrics, arrays, n, out_a, scratch)
        got = _raw(lib, lib.vfmm_error_metrics_noalloc, arrays, n, out_b)
        assert np.array_equal(got, ref), (n, got, ref)  # same kernels, same order: same bits
        om, orr, oden = M.errors(u, v, ur, vr)
        den = got[2] if got[2] > 0 else 1.0
        assert abs(got[0] / den - om) <= 1e-14 * om
        assert abs(np.sqrt(got[1] / n) / den - orr) <= 1e-13 * orr
    # argument errors are reported before any device work
    f = C.c_void_p(256)
    assert lib.vfmm_error_metrics_noalloc(None, f, f, f, 10, f, None) == vf.vfmm.ERR_INVALID_ARG
    assert lib.vfmm_error_metrics_noalloc(f, f, f, f, 0, f, None) == vf.vfmm.ERR_INVALID_ARG
