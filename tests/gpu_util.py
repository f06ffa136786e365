"""Helpers shared by the GPU tests: device transfer and oracle <-> GPU conversions."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0809_1810_amd as vf
    vf.lib()  # raises if the HIP library is missing: never a silent fallback
    return vf


def dev(a, dtype=None):
    a = np.ascontiguousarray(a)
    t = torch.from_numpy(a)
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel_err(u, v, ur, vr):
    d = np.hypot(u - ur, v - vr)
    den = np.max(np.hypot(ur, vr))
    return float(np.max(d) / den), float(np.sqrt(np.mean(d * d)) / den)


def oracle_me_scaled(a, w):
    """Paper ME coefficients a_k = (-j/2pi) w^k M_k  ->  scaled M_k."""
    k = np.arange(len(a))
    return 2 * math.pi * 1j * a / w ** k


def oracle_le_scaled(b, w):
    """Paper LE coefficients b_n = (-j/2pi) w^-(n+1) L_n  ->  scaled L_n."""
    n = np.arange(len(b))
    return 2 * math.pi * 1j * b * w ** (n + 1)


def print_case(name, **kw):
    print(f"[case] {name} " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)
