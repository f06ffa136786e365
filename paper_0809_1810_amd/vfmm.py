"""Python binding of ``libvfmm.so`` (the C ABI declared in ``include/vfmm.h``).

Argument marshalling only: every step of the computation runs in the HIP
library.  PyTorch supplies device memory (float64 CUDA tensors, the workspace)
and the current stream.  If the library has not been built, every entry point
raises ``VfmmUnavailable``: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libvfmm.so")
HEADER_PATH = os.path.join(os.path.dirname(HERE), "include", "vfmm.h")

FP64, FP32, M2L_BF16, M2L_FP16 = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": M2L_BF16, "fp16": M2L_FP16}
PART_NEAR, PART_FAR, PART_ALL = 1, 2, 3
MAX_P, MAX_LEVELS = 40, 12

OK = 0
ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_HIP, ERR_UNSUPPORTED, ERR_NONFINITE, ERR_WORKSPACE = (
    -1, -2, -3, -4, -5, -6)


class VfmmUnavailable(ImportError):
    """The HIP library is missing (not built)."""


class VfmmError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where} failed with status {status}: {detail}")
        self.status = status


_lib = None

_SIGS = {
    "vfmm_version": (C.c_int32, []),
    "vfmm_status_string": (C.c_char_p, [C.c_int32]),
    "vfmm_last_error": (C.c_char_p, []),
    "vfmm_workspace_bytes": (C.c_int32, [C.c_int64, C.c_int32, C.c_int32, C.POINTER(C.c_size_t)]),
    "vfmm_build_tree": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                    C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "vfmm_fmm_velocity": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_int32,
                                      C.c_void_p, C.c_void_p, C.c_void_p]),
    "vfmm_fmm_velocity_oneshot": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                              C.c_double, C.c_int32, C.c_int32, C.c_int32,
                                              C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                              C.c_void_p]),
    "vfmm_fmm_velocity_batched": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t,
                                              C.c_void_p]),
    "vfmm_fmm_velocity_parts": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                            C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                            C.c_void_p]),
    "vfmm_direct_velocity": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                         C.c_double, C.c_void_p, C.c_int64, C.c_void_p,
                                         C.c_void_p, C.c_void_p]),
    "vfmm_targets_workspace_bytes": (C.c_int32, [C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]),
    "vfmm_fmm_velocity_at": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_int32,
                                         C.c_int32, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                         C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vfmm_adaptive_workspace_bytes": (C.c_int32, [C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]),
    "vfmm_fmm_velocity_adaptive": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_double, C.c_int32,
                                               C.c_int32, C.c_int32, C.c_int64, C.c_void_p,
                                               C.c_size_t, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vfmm_direct_velocity_at": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                            C.c_double, C.c_void_p, C.c_void_p, C.c_int64,
                                            C.c_void_p, C.c_void_p, C.c_void_p]),
    "vfmm_error_field": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                     C.c_void_p, C.c_void_p, C.c_void_p]),
    "vfmm_metrics_scratch_bytes": (C.c_size_t, []),
    "vfmm_error_metrics": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                       C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vfmm_error_metrics_noalloc": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                               C.c_int64, C.c_void_p, C.c_void_p]),
    "vfmm_tree_arrays": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vfmm_tree_expansions": (C.c_int32, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]),
    "vfmm_tree_destroy": (None, [C.c_void_p]),
    "vfmm_tree_rebuild": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "vfmm_tree_enable_timing": (C.c_int32, [C.c_void_p, C.c_int32]),
    "vfmm_tree_set_near_radius": (C.c_int32, [C.c_void_p, C.c_double]),
    "vfmm_substitution_bound": (C.c_int32, [C.c_double, C.c_int32, C.c_double, C.c_double,
                                            C.c_int32, C.POINTER(C.c_double),
                                            C.POINTER(C.c_double)]),
    "vfmm_advect_workspace_bytes": (C.c_int32, [C.c_int64, C.POINTER(C.c_size_t)]),
    "vfmm_advect": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_double,
                                C.c_int32, C.c_int32, C.c_double, C.c_int32, C.c_void_p,
                                C.c_size_t, C.c_void_p]),
    "vfmm_tree_read_timing": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "vfmm_mlp_scratch_bytes": (C.c_size_t, [C.c_int64]),
    "vfmm_mlp_forward": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p,
                                     C.c_void_p]),
    "vfmm_mlp_gradient": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "vfmm_mlp_adam": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32,
                                  C.c_float, C.c_void_p]),
    "vfmm_batch_workspace_bytes": (C.c_int32, [C.c_void_p, C.c_int32, C.POINTER(C.c_size_t)]),
    "vfmm_batch_create": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t,
                                      C.POINTER(C.c_void_p)]),
    "vfmm_batch_run": (C.c_int32, [C.c_void_p, C.c_int32, C.c_void_p]),
    "vfmm_batch_destroy": (None, [C.c_void_p]),
    "vfmm_batch_substitution_bounds": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double)]),
    "vfmm_set_tuning": (C.c_int32, [C.c_int32, C.c_int32]),
    "vfmm_get_tuning": (C.c_int32, [C.c_int32]),
    "vfmm_tree_get_tuning": (C.c_int32, [C.c_void_p, C.c_int32]),
    "vfmm_tree_set_check_finite": (C.c_int32, [C.c_void_p, C.c_int32]),
    "vfmm_select_scratch_bytes": (C.c_size_t, [C.c_int64]),
    "vfmm_particle_stats": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p,
                                        C.c_size_t, C.POINTER(C.c_double), C.c_void_p]),
    "vfmm_selector_features": (C.c_int32, [C.POINTER(C.c_double), C.c_int64, C.c_double, C.c_int32,
                                           C.c_int32, C.c_double, C.POINTER(C.c_float)]),
    "vfmm_select_audit_workspace_bytes": (C.c_int32, [C.c_int64, C.c_int64, C.c_int32,
                                                      C.POINTER(C.c_size_t)]),
    "vfmm_select_and_audit": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                          C.c_double, C.c_double, C.c_void_p,
                                          C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_double,
                                          C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                          C.c_int32, C.c_double, C.c_int32, C.c_int32,
                                          C.c_void_p, C.c_size_t, C.c_void_p, C.c_void_p]),
    "vfmm_select_params": (C.c_int32, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_double,
                                       C.c_double, C.c_void_p, C.POINTER(C.c_float),
                                       C.POINTER(C.c_float), C.c_double, C.c_void_p, C.c_size_t,
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double),
                                       C.POINTER(C.c_int32), C.c_void_p]),
}

NEAR_RADIUS_AUTO = -1.0
NEAR_RINGS_MAX = 4  # the cut-off radius is clamped to NEAR_RINGS_MAX leaf sides
MLP_PARAMS = 4929
N_FEATURES = 10


class Instance(C.Structure):
    """Mirror of ``vfmm_instance``."""
    _fields_ = [("x", C.c_void_p), ("y", C.c_void_p), ("gamma", C.c_void_p), ("u", C.c_void_p),
                ("v", C.c_void_p), ("n", C.c_int64), ("sigma", C.c_double), ("p", C.c_int32),
                ("levels", C.c_int32)]

TUNE_P2P_TILE, TUNE_P2P_WAVES, TUNE_M2L_TILE, TUNE_P2P_SYMMETRIC = 1, 2, 3, 4

SELECT_AUDIT, SELECT_CUTOFF = 1, 2
SELECT_TRAIL_MAX = 16


class AuditStep(C.Structure):
    """Mirror of ``vfmm_audit_step``."""
    _fields_ = [("p", C.c_int32), ("levels", C.c_int32), ("precision", C.c_int32),
                ("near_radius", C.c_double), ("emax", C.c_double), ("ms", C.c_double)]


class Selection(C.Structure):
    """Mirror of ``vfmm_selection``."""
    _fields_ = [("p", C.c_int32), ("levels", C.c_int32), ("precision", C.c_int32),
                ("near_radius", C.c_double), ("used_fallback", C.c_int32),
                ("network_p", C.c_int32), ("network_levels", C.c_int32),
                ("network_fallback", C.c_int32), ("network_radius", C.c_double),
                ("predicted_log10", C.c_double),
                ("audit_emax", C.c_double), ("n_steps", C.c_int32),
                ("steps", AuditStep * SELECT_TRAIL_MAX)]

N_PHASES = 8
PHASES = ("gather", "tables", "p2m", "m2m", "m2l_l2l", "p2p_sched", "p2p", "l2p")


def header_symbols(path: str = HEADER_PATH):
    """Function names declared in the public header."""
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vfmm_[a-z0-9_]+)\s*\(", text)))


def lib():
    """The loaded library (raises VfmmUnavailable when it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise VfmmUnavailable(f"{LIB_PATH} is missing; build it with "
                                  "`python -m paper_0809_1810_amd.build`")
        l = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def _check(status: int, where: str):
    if status != OK:
        detail = lib().vfmm_last_error().decode(errors="replace")
        raise VfmmError(status, where, detail)


def _torch():
    import torch
    return torch


def _stream():
    return _torch().cuda.current_stream().cuda_stream


def _dev_f64(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise TypeError(f"{name} must be a CUDA float64 tensor")
    if not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous")
    return t


def workspace_bytes(n: int, levels: int, p_max: int) -> int:
    b = C.c_size_t(0)
    _check(lib().vfmm_workspace_bytes(int(n), int(levels), int(p_max), C.byref(b)),
           "vfmm_workspace_bytes")
    return int(b.value)


def targets_workspace_bytes(n_targets: int, levels: int) -> int:
    b = C.c_size_t(0)
    _check(lib().vfmm_targets_workspace_bytes(int(n_targets), int(levels), C.byref(b)),
           "vfmm_targets_workspace_bytes")
    return int(b.value)


class Tree:
    """A quadtree over device-resident particles, with its workspace."""

    def __init__(self, x, y, levels: int, p_max: int = MAX_P, domain=None, workspace=None):
        torch = _torch()
        x = _dev_f64(x, "x"); y = _dev_f64(y, "y")
        if x.shape != y.shape or x.dim() != 1:
            raise ValueError("x and y must be 1-D tensors of equal length")
        self.n = int(x.shape[0])
        self.levels = int(levels)
        self.p_max = int(p_max)
        nbytes = workspace_bytes(self.n, self.levels, self.p_max)
        if workspace is None:
            workspace = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
        self.workspace = workspace
        self.device = x.device
        dom = None
        if domain is not None:
            dom = (C.c_double * 3)(*[float(d) for d in domain])
        h = C.c_void_p(0)
        _check(lib().vfmm_build_tree(x.data_ptr(), y.data_ptr(), self.n, self.levels, dom,
                                     self.p_max, workspace.data_ptr(),
                                     workspace.numel() * workspace.element_size(), _stream(),
                                     C.byref(h)), "vfmm_build_tree")
        self._h = h
        self._keep = (x, y)

    def velocity(self, gamma, sigma: float, p: int, precision=FP64, parts=PART_ALL, out=None):
        torch = _torch()
        gamma = _dev_f64(gamma, "gamma")
        if gamma.shape[0] != self.n:
            raise ValueError("gamma has the wrong length")
        precision = PRECISIONS.get(precision, precision)
        if out is None:
            u = torch.empty(self.n, dtype=torch.float64, device=self.device)
            v = torch.empty(self.n, dtype=torch.float64, device=self.device)
        else:
            u, v = out
        _check(lib().vfmm_fmm_velocity_parts(self._h, gamma.data_ptr(), float(sigma), int(p),
                                             int(precision), int(parts), u.data_ptr(),
                                             v.data_ptr(), _stream()), "vfmm_fmm_velocity")
        return u, v

    def velocity_at(self, gamma, sigma: float, p: int, xt, yt, precision=FP64, parts=PART_ALL,
                    out=None, workspace=None):
        """FMM velocity at separate evaluation points (xt, yt); NaN outside the root square."""
        torch = _torch()
        gamma = _dev_f64(gamma, "gamma")
        xt = _dev_f64(xt, "xt"); yt = _dev_f64(yt, "yt")
        if gamma.shape[0] != self.n:
            raise ValueError("gamma has the wrong length")
        if xt.shape != yt.shape or xt.dim() != 1:
            raise ValueError("xt and yt must be 1-D tensors of equal length")
        nt = int(xt.shape[0])
        precision = PRECISIONS.get(precision, precision)
        if out is None:
            u = torch.empty(nt, dtype=torch.float64, device=self.device)
            v = torch.empty(nt, dtype=torch.float64, device=self.device)
        else:
            u, v = out
        if workspace is None:
            workspace = torch.empty(max(1, targets_workspace_bytes(nt, self.levels)),
                                    dtype=torch.uint8, device=self.device)
        _check(lib().vfmm_fmm_velocity_at(self._h, gamma.data_ptr(), float(sigma), int(p),
                                          int(precision), int(parts), xt.data_ptr(), yt.data_ptr(),
                                          nt, workspace.data_ptr(),
                                          workspace.numel() * workspace.element_size(),
                                          u.data_ptr(), v.data_ptr(), _stream()),
               "vfmm_fmm_velocity_at")
        return u, v

    def velocity_adaptive(self, gamma, sigma: float, p: int, leaf_capacity: int, precision=FP64,
                          parts=PART_ALL, out=None, workspace=None):
        """FMM velocity on the adaptive tree whose leaves hold at most
        ``leaf_capacity`` particles above this tree's leaf level."""
        torch = _torch()
        gamma = _dev_f64(gamma, "gamma")
        if gamma.shape[0] != self.n:
            raise ValueError("gamma has the wrong length")
        precision = PRECISIONS.get(precision, precision)
        if out is None:
            u = torch.empty(self.n, dtype=torch.float64, device=self.device)
            v = torch.empty(self.n, dtype=torch.float64, device=self.device)
        else:
            u, v = out
        if workspace is None:
            b = C.c_size_t(0)
            _check(lib().vfmm_adaptive_workspace_bytes(self.n, self.levels, C.byref(b)),
                   "vfmm_adaptive_workspace_bytes")
            workspace = torch.empty(int(b.value), dtype=torch.uint8, device=self.device)
        self._adaptive_ws = workspace
        _check(lib().vfmm_fmm_velocity_adaptive(self._h, gamma.data_ptr(), float(sigma), int(p),
                                                int(precision), int(parts), int(leaf_capacity),
                                                workspace.data_ptr(),
                                                workspace.numel() * workspace.element_size(),
                                                u.data_ptr(), v.data_ptr(), _stream()),
               "vfmm_fmm_velocity_adaptive")
        return u, v

    def rebuild(self, x, y, domain=None):
        """Rebuild in place for new positions (same n, levels, workspace)."""
        x = _dev_f64(x, "x"); y = _dev_f64(y, "y")
        if int(x.shape[0]) != self.n or int(y.shape[0]) != self.n:
            raise ValueError("rebuild needs the same number of particles")
        dom = None if domain is None else (C.c_double * 3)(*[float(d) for d in domain])
        _check(lib().vfmm_tree_rebuild(self._h, x.data_ptr(), y.data_ptr(), dom, _stream()),
               "vfmm_tree_rebuild")
        self._keep = (x, y)

    def advect(self, x, y, gamma, sigma: float, p: int, dt: float, steps: int, precision=FP64,
               workspace=None):
        """Advance the positions x, y (device float64, in place) by `steps` Heun
        steps with the FMM velocity (eq. 5); rebuilds this tree at every stage."""
        torch = _torch()
        x = _dev_f64(x, "x"); y = _dev_f64(y, "y"); gamma = _dev_f64(gamma, "gamma")
        if int(x.shape[0]) != self.n or int(y.shape[0]) != self.n or int(gamma.shape[0]) != self.n:
            raise ValueError("x, y and gamma must have the tree's length")
        precision = PRECISIONS.get(precision, precision)
        if workspace is None:
            b = C.c_size_t(0)
            _check(lib().vfmm_advect_workspace_bytes(self.n, C.byref(b)), "vfmm_advect_workspace_bytes")
            workspace = torch.empty(int(b.value), dtype=torch.uint8, device=self.device)
        _check(lib().vfmm_advect(self._h, x.data_ptr(), y.data_ptr(), gamma.data_ptr(), float(sigma),
                                 int(p), int(precision), float(dt), int(steps), workspace.data_ptr(),
                                 workspace.numel() * workspace.element_size(), _stream()),
               "vfmm_advect")
        self._keep = (x, y)
        return x, y

    def set_near_radius(self, radius: float):
        """Distance cut-off of the near field for later evaluations: 0 = the
        paper's split, > 0 = min(radius, NEAR_RINGS_MAX w_L), NEAR_RADIUS_AUTO =
        automatic (6 sigma in FP32, sqrt(76) sigma in FP64, same clamp)."""
        _check(lib().vfmm_tree_set_near_radius(self._h, float(radius)), "vfmm_tree_set_near_radius")
        self.near_radius = float(radius)

    def set_check_finite(self, enable: bool = True):
        """Opt-in finiteness check of later evaluations (raises VfmmError with
        status ERR_NONFINITE when an input or output holds NaN or infinity)."""
        _check(lib().vfmm_tree_set_check_finite(self._h, 1 if enable else 0),
               "vfmm_tree_set_check_finite")

    def tuning(self):
        """The launch shapes this tree was built with: {tile, waves, m2l, sym}."""
        return {"tile": int(lib().vfmm_tree_get_tuning(self._h, TUNE_P2P_TILE)),
                "waves": int(lib().vfmm_tree_get_tuning(self._h, TUNE_P2P_WAVES)),
                "m2l": int(lib().vfmm_tree_get_tuning(self._h, TUNE_M2L_TILE)),
                "sym": int(lib().vfmm_tree_get_tuning(self._h, TUNE_P2P_SYMMETRIC))}

    def enable_timing(self, max_calls: int):
        _check(lib().vfmm_tree_enable_timing(self._h, int(max_calls)), "vfmm_tree_enable_timing")
        self._tslots = int(max_calls)

    def read_timing(self):
        """List of per-call dicts {phase: ms} for the recorded calls (synchronises)."""
        slots = max(1, getattr(self, "_tslots", 1))
        buf = (C.c_double * (slots * N_PHASES))()
        n = C.c_int32(0)
        _check(lib().vfmm_tree_read_timing(self._h, buf, C.byref(n)), "vfmm_tree_read_timing")
        return [{PHASES[k]: buf[c * N_PHASES + k] for k in range(N_PHASES)} for c in range(n.value)]

    def arrays(self):
        """(root[4], perm[n], leaf_start[4^L + 1]) as device tensors."""
        torch = _torch()
        root = torch.empty(4, dtype=torch.float64, device=self.device)
        perm = torch.empty(self.n, dtype=torch.int32, device=self.device)
        ls = torch.empty((1 << (2 * self.levels)) + 1, dtype=torch.int32, device=self.device)
        _check(lib().vfmm_tree_arrays(self._h, root.data_ptr(), perm.data_ptr(), ls.data_ptr(),
                                      _stream()), "vfmm_tree_arrays")
        return root, perm, ls

    def expansions(self, kind: int, level: int, p: int):
        """Scaled ME (kind 0) or LE (kind 1) coefficients of `level`: complex [4^level, p]."""
        torch = _torch()
        nb = 1 << (2 * level)
        dst = torch.empty(nb * p * 2, dtype=torch.float64, device=self.device)
        _check(lib().vfmm_tree_expansions(self._h, int(kind), int(level), dst.data_ptr(),
                                          _stream()), "vfmm_tree_expansions")
        return torch.view_as_complex(dst.view(nb, p, 2))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().vfmm_tree_destroy(self._h)
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_tree(x, y, levels: int, p_max: int = MAX_P, domain=None) -> Tree:
    return Tree(x, y, levels, p_max, domain)


def fmm_velocity(x, y, gamma, sigma: float, p: int, levels: int, precision=FP64, domain=None):
    """One-shot: build the tree and evaluate the FMM velocity."""
    t = Tree(x, y, levels, p_max=p, domain=domain)
    return t.velocity(gamma, sigma, p, precision)


def fmm_velocity_oneshot(x, y, gamma, sigma: float, p: int, levels: int, precision=FP64,
                         out=None):
    """vfmm_fmm_velocity_oneshot: tree build + evaluation in one library call
    (bounding-square root); the workspace is allocated here, by the caller."""
    torch = _torch()
    x = _dev_f64(x, "x"); y = _dev_f64(y, "y"); gamma = _dev_f64(gamma, "gamma")
    n = int(x.shape[0])
    precision = PRECISIONS.get(precision, precision)
    nb = C.c_size_t(0)
    _check(lib().vfmm_workspace_bytes(n, int(levels), int(p), C.byref(nb)), "vfmm_workspace_bytes")
    ws = torch.empty(int(nb.value), dtype=torch.uint8, device=x.device)
    if out is None:
        u = torch.empty(n, dtype=torch.float64, device=x.device)
        v = torch.empty(n, dtype=torch.float64, device=x.device)
    else:
        u, v = out
    _check(lib().vfmm_fmm_velocity_oneshot(x.data_ptr(), y.data_ptr(), gamma.data_ptr(), n,
                                           float(sigma), int(p), int(levels), int(precision),
                                           u.data_ptr(), v.data_ptr(), ws.data_ptr(), ws.numel(),
                                           _stream()), "vfmm_fmm_velocity_oneshot")
    return u, v  # ws is freed on the current stream, after the call's work


def direct_velocity(x, y, gamma, sigma: float, targets=None, out=None):
    torch = _torch()
    x = _dev_f64(x, "x"); y = _dev_f64(y, "y"); gamma = _dev_f64(gamma, "gamma")
    n = int(x.shape[0])
    if targets is not None:
        if not targets.is_cuda or targets.dtype != torch.int64 or not targets.is_contiguous():
            raise TypeError("targets must be a contiguous CUDA int64 tensor")
        nt = int(targets.shape[0]); tp = targets.data_ptr()
    else:
        nt = n; tp = None
    if out is None:
        u = torch.empty(nt, dtype=torch.float64, device=x.device)
        v = torch.empty(nt, dtype=torch.float64, device=x.device)
    else:
        u, v = out
    _check(lib().vfmm_direct_velocity(x.data_ptr(), y.data_ptr(), gamma.data_ptr(), n,
                                      float(sigma), tp, nt, u.data_ptr(), v.data_ptr(), _stream()),
           "vfmm_direct_velocity")
    return u, v


def direct_velocity_at(x, y, gamma, sigma: float, xt, yt, out=None):
    """Float64 direct sum (eq. 8) at separate evaluation points."""
    torch = _torch()
    x = _dev_f64(x, "x"); y = _dev_f64(y, "y"); gamma = _dev_f64(gamma, "gamma")
    xt = _dev_f64(xt, "xt"); yt = _dev_f64(yt, "yt")
    nt = int(xt.shape[0])
    if out is None:
        u = torch.empty(nt, dtype=torch.float64, device=x.device)
        v = torch.empty(nt, dtype=torch.float64, device=x.device)
    else:
        u, v = out
    _check(lib().vfmm_direct_velocity_at(x.data_ptr(), y.data_ptr(), gamma.data_ptr(),
                                         int(x.shape[0]), float(sigma), xt.data_ptr(),
                                         yt.data_ptr(), nt, u.data_ptr(), v.data_ptr(), _stream()),
           "vfmm_direct_velocity_at")
    return u, v


def error_field(u, v, u_ref, v_ref):
    """Per-point log10(|dW| / max|W_ref|) (device tensor), floored at -300."""
    torch = _torch()
    for t, nme in ((u, "u"), (v, "v"), (u_ref, "u_ref"), (v_ref, "v_ref")):
        _dev_f64(t, nme)
    n = int(u.shape[0])
    scratch = torch.empty(int(lib().vfmm_metrics_scratch_bytes()), dtype=torch.uint8,
                          device=u.device)
    met = torch.empty(3, dtype=torch.float64, device=u.device)
    out = torch.empty(n, dtype=torch.float64, device=u.device)
    if n == 0:
        return out
    _check(lib().vfmm_error_metrics(u.data_ptr(), v.data_ptr(), u_ref.data_ptr(),
                                    v_ref.data_ptr(), n, scratch.data_ptr(), met.data_ptr(),
                                    _stream()), "vfmm_error_metrics")
    _check(lib().vfmm_error_field(u.data_ptr(), v.data_ptr(), u_ref.data_ptr(), v_ref.data_ptr(),
                                  n, met.data_ptr(), out.data_ptr(), _stream()),
           "vfmm_error_field")
    return out


def error_metrics(u, v, u_ref, v_ref):
    """(e_max, e_rms, max|W_ref|) computed on the GPU (synchronises)."""
    torch = _torch()
    for t, nme in ((u, "u"), (v, "v"), (u_ref, "u_ref"), (v_ref, "v_ref")):
        _dev_f64(t, nme)
    n = int(u.shape[0])
    scratch = torch.empty(int(lib().vfmm_metrics_scratch_bytes()), dtype=torch.uint8,
                          device=u.device)
    out = torch.empty(3, dtype=torch.float64, device=u.device)
    _check(lib().vfmm_error_metrics(u.data_ptr(), v.data_ptr(), u_ref.data_ptr(),
                                    v_ref.data_ptr(), n, scratch.data_ptr(), out.data_ptr(),
                                    _stream()), "vfmm_error_metrics")
    mx, ss, den = out.cpu().tolist()
    if den == 0.0:  # an all-zero reference: absolute errors (a NaN maximum stays NaN)
        den = 1.0
    return mx / den, math.sqrt(ss / n) / den, den


def error_metrics_noalloc(u, v, u_ref, v_ref, out):
    """vfmm_error_metrics_noalloc: raw (max |dW|, sum |dW|^2, max |W_ref|) into the
    caller's device float64 tensor ``out`` (3 entries), asynchronously, with no
    scratch argument (the library's own device array holds the partial sums)."""
    for t, nme in ((u, "u"), (v, "v"), (u_ref, "u_ref"), (v_ref, "v_ref"), (out, "out")):
        _dev_f64(t, nme)
    if out.numel() < 3:
        raise ValueError("out needs 3 entries")
    _check(lib().vfmm_error_metrics_noalloc(u.data_ptr(), v.data_ptr(), u_ref.data_ptr(),
                                            v_ref.data_ptr(), int(u.shape[0]), out.data_ptr(),
                                            _stream()), "vfmm_error_metrics_noalloc")
    return out


def substitution_bound(root_side, levels, sigma, near_radius=0.0, precision=FP64):
    """vfmm_substitution_bound (host only): (d, bound) with d the distance below
    which every pair is summed with the regularised kernel and bound the
    relative kernel error |K' - K_sigma| / |K_sigma| of a far pair at d."""
    d = C.c_double(0.0); b = C.c_double(0.0)
    _check(lib().vfmm_substitution_bound(float(root_side), int(levels), float(sigma),
                                         float(near_radius), int(precision), C.byref(d),
                                         C.byref(b)), "vfmm_substitution_bound")
    return d.value, b.value


# ----------------------------------------------------------------- selector network


def _dev_f32(t, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous CUDA float32 tensor")
    return t


def mlp_forward(params, x, bf16=True, out=None):
    """Network outputs for standardised features x [B, 10] (float32, device)."""
    torch = _torch()
    _dev_f32(params, "params"); _dev_f32(x, "x")
    B = int(x.shape[0])
    y = torch.empty(B, dtype=torch.float32, device=x.device) if out is None else out
    _check(lib().vfmm_mlp_forward(params.data_ptr(), int(bool(bf16)), x.data_ptr(), B, y.data_ptr(),
                                  _stream()), "vfmm_mlp_forward")
    return y


class MlpTrainer:
    """Device state for training: master params, Adam moments, gradient, scratch."""

    def __init__(self, params, max_batch):
        torch = _torch()
        self.params = _dev_f32(params, "params")
        self.m = torch.zeros_like(params); self.v = torch.zeros_like(params)
        self.grad = torch.zeros_like(params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=params.device)
        nb = int(lib().vfmm_mlp_scratch_bytes(int(max_batch)))
        self.scratch = torch.empty(nb, dtype=torch.uint8, device=params.device)
        self.max_batch = int(max_batch)
        self.step_count = 0

    def gradient(self, x, t, bf16=True):
        _dev_f32(x, "x"); _dev_f32(t, "target")
        B = int(x.shape[0])
        if B > self.max_batch:
            raise ValueError("batch larger than the trainer's scratch")
        _check(lib().vfmm_mlp_gradient(self.params.data_ptr(), int(bool(bf16)), x.data_ptr(),
                                       t.data_ptr(), B, self.grad.data_ptr(), self.loss.data_ptr(),
                                       self.scratch.data_ptr(), self.scratch.numel(), _stream()),
               "vfmm_mlp_gradient")
        return self.grad, self.loss

    def adam(self, lr):
        self.step_count += 1
        _check(lib().vfmm_mlp_adam(self.params.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                                   self.grad.data_ptr(), self.step_count, float(lr), _stream()),
               "vfmm_mlp_adam")

    def step(self, x, t, lr, bf16=True):
        self.gradient(x, t, bf16)
        self.adam(lr)
        return self.loss


def particle_stats(x, y, gamma):
    torch = _torch()
    for t, n in ((x, "x"), (y, "y"), (gamma, "gamma")):
        _dev_f64(t, n)
    n = int(x.shape[0])
    scratch = torch.empty(int(lib().vfmm_select_scratch_bytes(n)), dtype=torch.uint8, device=x.device)
    st = (C.c_double * 12)()
    _check(lib().vfmm_particle_stats(x.data_ptr(), y.data_ptr(), gamma.data_ptr(), n,
                                     scratch.data_ptr(), scratch.numel(), st, _stream()),
           "vfmm_particle_stats")
    return list(st)


def selector_features(stats, n, sigma, p, levels, radius=0.0):
    """The ten selector features of (p, levels, near radius) (host function)."""
    st = (C.c_double * 12)(*stats)
    out = (C.c_float * N_FEATURES)()
    _check(lib().vfmm_selector_features(st, int(n), float(sigma), int(p), int(levels),
                                        float(radius), out), "vfmm_selector_features")
    return list(out)


def select_params(x, y, gamma, sigma, tol, params, feat_mean, feat_std, margin=0.3):
    """(p, levels, near radius, predicted log10 error, used_fallback) for an FP32
    evaluation."""
    torch = _torch()
    for t, nme in ((x, "x"), (y, "y"), (gamma, "gamma")):
        _dev_f64(t, nme)
    _dev_f32(params, "params")
    n = int(x.shape[0])
    scratch = torch.empty(int(lib().vfmm_select_scratch_bytes(n)), dtype=torch.uint8, device=x.device)
    fm = (C.c_float * N_FEATURES)(*[float(v) for v in feat_mean])
    fs = (C.c_float * N_FEATURES)(*[float(v) for v in feat_std])
    p = C.c_int32(0); L = C.c_int32(0); rad = C.c_double(0.0); pred = C.c_double(0.0)
    fb = C.c_int32(0)
    _check(lib().vfmm_select_params(x.data_ptr(), y.data_ptr(), gamma.data_ptr(), n, float(sigma),
                                    float(tol), params.data_ptr(), fm, fs, float(margin),
                                    scratch.data_ptr(), scratch.numel(), C.byref(p), C.byref(L),
                                    C.byref(rad), C.byref(pred), C.byref(fb), _stream()),
           "vfmm_select_params")
    return int(p.value), int(L.value), float(rad.value), float(pred.value), bool(fb.value)


def select_and_audit(x, y, gamma, sigma, tol, params, feat_mean, feat_std, margin, targets,
                     reference=None, audit=True, cutoff=True, slack=0.5, time_reps=3,
                     max_levels=0):
    """vfmm_select_and_audit: the network's (p, L), audited on ``targets`` (device
    int64 particle indices) against ``reference`` ((u, v) of the FP64 direct sum
    there, or None: computed by the call), escalated or replaced by the
    conservative FP64 choice if it fails, and with ``cutoff`` compared with
    deeper levels under the distance cut-off.  Returns the ``Selection`` struct."""
    torch = _torch()
    for t, nme in ((x, "x"), (y, "y"), (gamma, "gamma")):
        _dev_f64(t, nme)
    _dev_f32(params, "params")
    n = int(x.shape[0])
    if not isinstance(targets, torch.Tensor) or targets.dtype != torch.int64 or not targets.is_cuda:
        raise TypeError("targets must be a CUDA int64 tensor")
    nt = int(targets.shape[0])
    ur = vr = None
    if reference is not None:
        ur, vr = (_dev_f64(a, "reference") for a in reference)
    b = C.c_size_t(0)
    _check(lib().vfmm_select_audit_workspace_bytes(n, max(1, nt), int(max_levels), C.byref(b)),
           "vfmm_select_audit_workspace_bytes")
    ws = torch.empty(int(b.value), dtype=torch.uint8, device=x.device)
    fm = (C.c_float * N_FEATURES)(*[float(v) for v in feat_mean])
    fs = (C.c_float * N_FEATURES)(*[float(v) for v in feat_std])
    flags = (SELECT_AUDIT if audit else 0) | (SELECT_CUTOFF if audit and cutoff else 0)
    out = Selection()
    _check(lib().vfmm_select_and_audit(x.data_ptr(), y.data_ptr(), gamma.data_ptr(), n,
                                       float(sigma), float(tol), params.data_ptr(), fm, fs,
                                       float(margin), targets.data_ptr(), nt,
                                       ur.data_ptr() if ur is not None else None,
                                       vr.data_ptr() if vr is not None else None, flags,
                                       float(slack), int(time_reps), int(max_levels),
                                       ws.data_ptr(), ws.numel(), C.byref(out), _stream()),
           "vfmm_select_and_audit")
    return out


# ----------------------------------------------------------------- batched instances


class Batch:
    """Many independent instances evaluated together (see vfmm_batch_create).

    ``instances``: list of dicts with device float64 tensors x, y, gamma and
    sigma, p, levels.  Outputs live in ``self.u[i]``, ``self.v[i]``.
    """

    def __init__(self, instances):
        torch = _torch()
        self.inputs, self.u, self.v = [], [], []
        arr = (Instance * len(instances))()
        for i, d in enumerate(instances):
            x = _dev_f64(d["x"], "x"); y = _dev_f64(d["y"], "y"); g = _dev_f64(d["gamma"], "gamma")
            n = int(x.shape[0])
            u = torch.empty(n, dtype=torch.float64, device=x.device)
            v = torch.empty(n, dtype=torch.float64, device=x.device)
            self.inputs.append((x, y, g)); self.u.append(u); self.v.append(v)
            arr[i] = Instance(x.data_ptr(), y.data_ptr(), g.data_ptr(), u.data_ptr(), v.data_ptr(), n,
                              float(d["sigma"]), int(d["p"]), int(d["levels"]))
        self._arr = arr
        nb = C.c_size_t(0)
        _check(lib().vfmm_batch_workspace_bytes(arr, len(instances), C.byref(nb)),
               "vfmm_batch_workspace_bytes")
        self.workspace = torch.empty(int(nb.value), dtype=torch.uint8,
                                     device=self.inputs[0][0].device)
        h = C.c_void_p(0)
        _check(lib().vfmm_batch_create(arr, len(instances), self.workspace.data_ptr(),
                                       self.workspace.numel(), C.byref(h)), "vfmm_batch_create")
        self._h = h

    def run(self, use_graph=False):
        _check(lib().vfmm_batch_run(self._h, int(bool(use_graph)), _stream()), "vfmm_batch_run")

    def run_oneshot(self):
        """vfmm_fmm_velocity_batched on the same instances and workspace: plan,
        run and release in one library call (this object's plan is untouched)."""
        _check(lib().vfmm_fmm_velocity_batched(self._arr, len(self.u), self.workspace.data_ptr(),
                                               self.workspace.numel(), _stream()),
               "vfmm_fmm_velocity_batched")

    def substitution_bounds(self):
        """vfmm_batch_substitution_bounds: per-instance kernel-substitution floor
        (list of floats) for the bounding squares of the last run."""
        out = (C.c_double * len(self.u))()
        _check(lib().vfmm_batch_substitution_bounds(self._h, out), "vfmm_batch_substitution_bounds")
        return list(out)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().vfmm_batch_destroy(self._h)
            self._h = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_tuning(tile=None, waves=None, m2l=None, sym=None):
    """Launch shapes for trees built afterwards: near-field tile size (64/32/16),
    near-field waves per workgroup (1/2/4/8), FP32 matrix-core M2L tile (0/1/2),
    symmetric near field (0/1, 64-particle tiles)."""
    if tile is not None:
        _check(lib().vfmm_set_tuning(TUNE_P2P_TILE, int(tile)), "vfmm_set_tuning")
    if waves is not None:
        _check(lib().vfmm_set_tuning(TUNE_P2P_WAVES, int(waves)), "vfmm_set_tuning")
    if m2l is not None:
        _check(lib().vfmm_set_tuning(TUNE_M2L_TILE, int(m2l)), "vfmm_set_tuning")
    if sym is not None:
        _check(lib().vfmm_set_tuning(TUNE_P2P_SYMMETRIC, int(sym)), "vfmm_set_tuning")


def get_tuning():
    return {"tile": int(lib().vfmm_get_tuning(TUNE_P2P_TILE)),
            "waves": int(lib().vfmm_get_tuning(TUNE_P2P_WAVES)),
            "m2l": int(lib().vfmm_get_tuning(TUNE_M2L_TILE)),
            "sym": int(lib().vfmm_get_tuning(TUNE_P2P_SYMMETRIC))}
