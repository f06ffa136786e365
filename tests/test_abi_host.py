"""Host-side checks of the C ABI (no GPU needed, no kernel launched).

The library must load, export every function the public header declares, and
reject invalid arguments on the host with the documented status codes before
any device call.
"""
import ctypes as C
import os
import subprocess

import pytest

import paper_0809_1810_amd as vf
from paper_0809_1810_amd import vfmm as B


def _lib():
    try:
        return vf.lib()
    except vf.VfmmUnavailable:
        pytest.skip("libvfmm.so not built (python -m paper_0809_1810_amd.build)")


def test_exports_every_header_symbol():
    _lib()
    declared = set(vf.header_symbols())
    assert len(declared) >= 16
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert declared <= exported, declared - exported
    assert set(B._SIGS) == declared  # the binding covers exactly the header


def test_header_constants_match_the_binding():
    import re
    text = open(B.HEADER_PATH).read()
    consts = dict(re.findall(r"#define\s+(VFMM_[A-Z0-9_]+)\s+\(?(-?[0-9.]+)\)?", text))
    assert int(consts["VFMM_N_PHASES"]) == vf.N_PHASES == len(vf.PHASES)
    assert int(consts["VFMM_PART_NEAR"]) == vf.PART_NEAR and int(consts["VFMM_PART_FAR"]) == vf.PART_FAR
    assert float(consts["VFMM_NEAR_RADIUS_AUTO"]) == vf.NEAR_RADIUS_AUTO
    assert int(consts["VFMM_NEAR_RINGS_MAX"]) == vf.NEAR_RINGS_MAX
    for name in ("FP64", "FP32", "M2L_BF16", "M2L_FP16"):
        assert int(consts["VFMM_" + name]) == getattr(vf, name)


def test_workspace_bytes_host_only():
    l = _lib()
    b = C.c_size_t(0)
    assert l.vfmm_workspace_bytes(1 << 20, 6, 20, C.byref(b)) == 0
    small = C.c_size_t(0)
    assert l.vfmm_workspace_bytes(1000, 3, 10, C.byref(small)) == 0
    assert 0 < small.value < b.value
    # grows with p and levels
    b2 = C.c_size_t(0)
    assert l.vfmm_workspace_bytes(1 << 20, 6, 40, C.byref(b2)) == 0 and b2.value > b.value


@pytest.mark.parametrize("args,status", [
    ((0, 3, 10), B.ERR_INVALID_ARG),
    ((10, -1, 10), B.ERR_INVALID_ARG),
    ((10, 13, 10), B.ERR_INVALID_ARG),
    ((10, 3, 0), B.ERR_INVALID_ARG),
    ((10, 3, 41), B.ERR_INVALID_ARG),
])
def test_workspace_bytes_validation(args, status):
    l = _lib()
    assert l.vfmm_workspace_bytes(*args, C.byref(C.c_size_t())) == status
    assert len(l.vfmm_last_error()) > 0


def test_build_tree_rejects_before_device_work():
    l = _lib()
    h = C.c_void_p(0)
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    # null positions
    assert l.vfmm_build_tree(None, None, 10, 3, None, 10, fake, 1 << 30, None, C.byref(h)) == B.ERR_INVALID_ARG
    # workspace too small
    assert l.vfmm_build_tree(fake, fake, 10, 3, None, 10, fake, 16, None, C.byref(h)) == B.ERR_WORKSPACE
    # misaligned workspace
    assert l.vfmm_build_tree(fake, fake, 10, 3, None, 10, C.c_void_p(0x1001), 1 << 30, None,
                             C.byref(h)) == B.ERR_WORKSPACE
    # bad domain side
    dom = (C.c_double * 3)(0.0, 0.0, -1.0)
    assert l.vfmm_build_tree(fake, fake, 10, 3, dom, 10, fake, 1 << 30, None, C.byref(h)) == B.ERR_INVALID_ARG
    assert h.value is None
    # null tree handles
    assert l.vfmm_fmm_velocity(None, fake, 0.1, 5, 0, fake, fake, None) == B.ERR_INVALID_ARG
    assert l.vfmm_tree_enable_timing(None, 4) == B.ERR_INVALID_ARG
    assert l.vfmm_direct_velocity(fake, fake, fake, 10, -1.0, None, 10, fake, fake, None) == B.ERR_INVALID_ARG
    assert l.vfmm_direct_velocity(fake, fake, fake, 10, 0.1, None, 5, fake, fake, None) == B.ERR_INVALID_ARG
    l.vfmm_tree_destroy(None)  # ignored


def test_status_strings():
    l = _lib()
    names = {}
    for s in (0, -1, -2, -3, -4, -5, -6, -99):
        names[s] = l.vfmm_status_string(s).decode()
        assert len(names[s]) > 0
    # every documented status has its own name
    assert len({names[s] for s in (0, -1, -2, -3, -4, -5, -6)}) == 7
    assert names[-99] == "unknown status"
    assert "memory" in names[B.ERR_OUT_OF_MEMORY] and "finite" in names[B.ERR_NONFINITE]
    assert l.vfmm_version() >= 100


def test_status_codes_match_the_header():
    import re
    text = open(B.HEADER_PATH).read()
    consts = dict(re.findall(r"#define\s+(VFMM_(?:OK|ERR_[A-Z_]+))\s+\(?(-?[0-9]+)\)?", text))
    for name in ("INVALID_ARG", "OUT_OF_MEMORY", "HIP", "UNSUPPORTED", "NONFINITE", "WORKSPACE"):
        assert int(consts["VFMM_ERR_" + name]) == getattr(B, "ERR_" + name)
    assert int(consts["VFMM_OK"]) == B.OK


def test_tree_settings_reject_null_tree():
    l = _lib()
    assert l.vfmm_tree_set_check_finite(None, 1) == B.ERR_INVALID_ARG
    assert l.vfmm_tree_get_tuning(None, B.TUNE_P2P_TILE) == -1
    assert l.vfmm_tree_get_tuning(None, B.TUNE_P2P_WAVES) == -1
    # process-wide settings: validated, read back
    old = (l.vfmm_get_tuning(B.TUNE_P2P_TILE), l.vfmm_get_tuning(B.TUNE_P2P_WAVES))
    assert l.vfmm_set_tuning(B.TUNE_P2P_TILE, 48) == B.ERR_INVALID_ARG
    assert l.vfmm_set_tuning(B.TUNE_P2P_WAVES, 3) == B.ERR_INVALID_ARG
    assert l.vfmm_set_tuning(99, 1) == B.ERR_INVALID_ARG
    assert l.vfmm_get_tuning(99) == -1
    assert (l.vfmm_get_tuning(B.TUNE_P2P_TILE), l.vfmm_get_tuning(B.TUNE_P2P_WAVES)) == old


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(vf.VfmmUnavailable):
        B.lib()


def test_selector_features_host_function_matches_oracle():
    """vfmm_selector_features is pure host code: compare with the oracle definition."""
    _lib()
    import numpy as np

    import workloads as W
    from oracle import mlp as OM
    from oracle import quadtree as qt
    P = W.clusters(3000, seed=2)
    g = P.gamma
    st = [P.x.sum(), (P.x ** 2).sum(), P.y.sum(), (P.y ** 2).sum(), g.sum(), (g ** 2).sum(),
          np.abs(g).sum(), np.abs(g).max(), P.x.min(), P.x.max(), P.y.min(), P.y.max()]
    side = qt.root_square(P.x, P.y)[2]
    for p, L in ((4, 2), (9, 4), (20, 8)):
        for radius in (0.0, -1.0, 5.26 * P.sigma, 1e3):
            f = vf.selector_features(st, P.n, P.sigma, p, L, radius)
            fr = OM.features(P.x, P.y, g, P.sigma, p, L, side, radius)
            assert np.allclose(f, fr, rtol=1e-6, atol=1e-6), (radius, f, fr)


def test_evaluation_point_calls_reject_before_device_work():
    l = _lib()
    b = C.c_size_t(0)
    assert l.vfmm_targets_workspace_bytes(1000, 5, C.byref(b)) == 0 and b.value > 0
    b0 = C.c_size_t(1)
    assert l.vfmm_targets_workspace_bytes(0, 5, C.byref(b0)) == 0
    assert l.vfmm_targets_workspace_bytes(-1, 5, C.byref(b)) == B.ERR_INVALID_ARG
    assert l.vfmm_targets_workspace_bytes(10, 13, C.byref(b)) == B.ERR_INVALID_ARG
    fake = C.c_void_p(0x1000)
    assert l.vfmm_fmm_velocity_at(None, fake, 0.1, 5, 0, 3, fake, fake, 10, fake, 1 << 30, fake,
                                  fake, None) == B.ERR_INVALID_ARG
    assert l.vfmm_direct_velocity_at(fake, fake, fake, 10, 0.1, fake, fake, -1, fake, fake,
                                     None) == B.ERR_INVALID_ARG
    assert l.vfmm_direct_velocity_at(fake, fake, fake, 10, 0.0, fake, fake, 5, fake, fake,
                                     None) == B.ERR_INVALID_ARG
    assert l.vfmm_direct_velocity_at(fake, fake, fake, 10, 0.1, None, fake, 5, fake, fake,
                                     None) == B.ERR_INVALID_ARG
    # nothing to do: no device access
    assert l.vfmm_direct_velocity_at(fake, fake, fake, 10, 0.1, None, None, 0, None, None, None) == 0
    assert l.vfmm_error_field(fake, fake, fake, fake, 4, None, fake, None) == B.ERR_INVALID_ARG
    assert l.vfmm_error_field(fake, fake, fake, fake, -1, fake, fake, None) == B.ERR_INVALID_ARG
    assert l.vfmm_error_field(fake, fake, fake, fake, 0, fake, fake, None) == 0


def test_advect_calls_reject_before_device_work():
    l = _lib()
    b = C.c_size_t(0)
    assert l.vfmm_advect_workspace_bytes(1000, C.byref(b)) == 0 and b.value >= 6 * 8000
    assert l.vfmm_advect_workspace_bytes(0, C.byref(b)) == B.ERR_INVALID_ARG
    fake = C.c_void_p(0x1000)
    assert l.vfmm_advect(None, fake, fake, fake, 0.1, 5, 0, 0.01, 1, fake, 1 << 30,
                         None) == B.ERR_INVALID_ARG
    assert l.vfmm_tree_set_near_radius(None, 0.1) == B.ERR_INVALID_ARG


def test_one_call_entry_points_reject_before_device_work():
    lib = _lib()
    fake = C.c_void_p(256)  # never dereferenced: the checks fail first
    assert lib.vfmm_fmm_velocity_oneshot(None, fake, fake, 10, 0.1, 5, 3, 1, fake, fake, fake,
                                         1 << 20, None) == -1
    assert lib.vfmm_fmm_velocity_oneshot(fake, fake, fake, 0, 0.1, 5, 3, 1, fake, fake, fake,
                                         1 << 20, None) == -1
    assert lib.vfmm_fmm_velocity_batched(None, 1, fake, 1 << 20, None) == -1
    arr = (B.Instance * 1)()
    assert lib.vfmm_fmm_velocity_batched(arr, 0, fake, 1 << 20, None) == -1


def test_selection_struct_layout_matches_the_header(tmp_path):
    """The ctypes mirrors of vfmm_audit_step / vfmm_selection have the C layout
    (a C compiler prints sizeof and offsetof of every field)."""
    import shutil
    cc = shutil.which("cc") or shutil.which("gcc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = [f for f, _ in B.Selection._fields_]
    sfields = [f for f, _ in B.AuditStep._fields_]
    src = tmp_path / "probe.c"
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{B.HEADER_PATH}"',
             'int main(void) {',
             '  printf("%zu %zu\\n", sizeof(vfmm_selection), sizeof(vfmm_audit_step));']
    lines += [f'  printf("%zu\\n", offsetof(vfmm_selection, {f}));' for f in fields]
    lines += [f'  printf("%zu\\n", offsetof(vfmm_audit_step, {f}));' for f in sfields]
    lines += ['  return 0;', '}']
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    subprocess.run([cc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    vals = [int(v) for v in out]
    assert vals[0] == C.sizeof(B.Selection) and vals[1] == C.sizeof(B.AuditStep)
    got = [getattr(B.Selection, f).offset for f in fields] + [getattr(B.AuditStep, f).offset for f in sfields]
    assert vals[2:] == got


def test_select_and_audit_rejects_before_device_work():
    l = _lib()
    b = C.c_size_t(0)
    assert l.vfmm_select_audit_workspace_bytes(1 << 20, 4096, 0, C.byref(b)) == 0 and b.value > 0
    b7 = C.c_size_t(0)
    assert l.vfmm_select_audit_workspace_bytes(1 << 20, 4096, 7, C.byref(b7)) == 0
    assert 0 < b7.value < b.value  # sized for the deepest tree allowed
    assert l.vfmm_select_audit_workspace_bytes(0, 1, 0, C.byref(b)) == B.ERR_INVALID_ARG
    assert l.vfmm_select_audit_workspace_bytes(100, 101, 0, C.byref(b)) == B.ERR_INVALID_ARG
    assert l.vfmm_select_audit_workspace_bytes(100, 10, 13, C.byref(b)) == B.ERR_INVALID_ARG
    f = C.c_void_p(256)
    fm = (C.c_float * 10)(*([0.0] * 10)); fs = (C.c_float * 10)(*([1.0] * 10))
    out = B.Selection()

    def call(**kw):
        a = dict(x=f, n=1000, sigma=0.01, tol=1e-6, targets=f, nt=100, flags=3, slack=0.8,
                 reps=3, ws=f, wsb=1 << 40, out=C.byref(out))
        a.update(kw)
        return l.vfmm_select_and_audit(a["x"], f, f, a["n"], a["sigma"], a["tol"], f, fm, fs, 0.3,
                                       a["targets"], a["nt"], None, None, a["flags"], a["slack"],
                                       a["reps"], 0, a["ws"], a["wsb"], a["out"], None)
    assert call(x=None) == B.ERR_INVALID_ARG
    assert call(out=None) == B.ERR_INVALID_ARG
    assert call(n=0) == B.ERR_INVALID_ARG
    assert call(sigma=-1.0) == B.ERR_INVALID_ARG
    assert call(tol=0.0) == B.ERR_INVALID_ARG
    assert call(slack=1.5) == B.ERR_INVALID_ARG
    assert call(flags=8) == B.ERR_INVALID_ARG
    assert call(targets=None) == B.ERR_INVALID_ARG
    assert call(nt=1001) == B.ERR_INVALID_ARG
    assert call(reps=0) == B.ERR_INVALID_ARG
    assert call(ws=C.c_void_p(257)) == B.ERR_WORKSPACE
    assert call(wsb=16) == B.ERR_WORKSPACE


@pytest.mark.parametrize("sig", [0.05, 0.03])
def test_substitution_bound_host_function(sig):
    """vfmm_substitution_bound against the kernels of the oracle: at the
    returned distance d, |K' - K_sigma| / |K_sigma| evaluated from eq. 6 and
    eq. 15 directly (the difference of the two cancels to a relative accuracy
    of about 1e-16 / bound); d follows the leaf side, the clamped near radius
    and the automatic radius of each precision."""
    import math

    import numpy as np

    from oracle import kernel as K
    _lib()
    S, L = 2.0, 5
    w = S / 2 ** L
    cases = [
        (0.0, vf.FP64, w),                       # the paper's split
        (0.5 * w, vf.FP32, w),                    # a radius below w_L changes nothing
        (2.5 * w, vf.FP32, 2.5 * w),
        (9.0 * w, vf.FP64, 4.0 * w),              # clamped to 4 leaf sides
        (vf.NEAR_RADIUS_AUTO, vf.FP32, max(w, min(6.0 * sig, 4 * w))),
        (vf.NEAR_RADIUS_AUTO, vf.M2L_BF16, max(w, min(6.0 * sig, 4 * w))),
        (vf.NEAR_RADIUS_AUTO, vf.FP64, max(w, min(math.sqrt(76.0) * sig, 4 * w))),
    ]
    for radius, prec, d_expect in cases:
        d, b = vf.substitution_bound(S, L, sig, radius, prec)
        assert d == pytest.approx(d_expect, rel=1e-15), (radius, prec)
        for ang in (0.0, 0.7, 2.0):
            dx, dy = d * math.cos(ang), d * math.sin(ang)
            ks = np.array(K.singular_kernel(dx, dy))
            kr = np.array(K.regularized_kernel(dx, dy, sig))
            ref = np.linalg.norm(ks - kr) / np.linalg.norm(kr)
            assert b == pytest.approx(ref, rel=1e-12 + 1e-15 / b), (radius, prec, ang)


def test_substitution_bound_limits_and_errors():
    l = _lib()
    # leaves narrower than sigma: the floor exceeds the kernel itself
    assert vf.substitution_bound(1.0, 8, 0.01)[1] > 1.0
    # leaves of 10 sigma: below any float64 tolerance
    assert vf.substitution_bound(1.0, 4, 0.00625)[1] < 1e-20
    out = C.c_double(0.0)
    for args in ((0.0, 3, 0.1, 0.0, 0), (1.0, -1, 0.1, 0.0, 0), (1.0, 13, 0.1, 0.0, 0),
                 (1.0, 3, 0.0, 0.0, 0), (1.0, 3, 0.1, float("nan"), 0), (1.0, 3, 0.1, 0.0, 7),
                 (float("inf"), 3, 0.1, 0.0, 0)):
        assert l.vfmm_substitution_bound(*args, None, C.byref(out)) == B.ERR_INVALID_ARG, args
    assert l.vfmm_substitution_bound(1.0, 3, 0.1, 0.0, 0, None, None) == B.ERR_INVALID_ARG
    assert l.vfmm_batch_substitution_bounds(None, C.byref(out)) == B.ERR_INVALID_ARG
