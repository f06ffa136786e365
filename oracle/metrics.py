"""Error metrics (Section 5.1): errors normalised by the maximum velocity.

Test infrastructure (see ``oracle/__init__``).

The paper compares against a reference and normalises by "the maximum velocity
of the system".  Read as: with dW_i the vector difference of the two velocities
at particle i,

* e_max = max_i |dW_i| / max_i |W_i^ref|
* e_rms = sqrt(mean_i |dW_i|^2) / max_i |W_i^ref|

(pointwise relative error is ill-posed at stagnation points such as vortex
centres).  For a sampled comparison the maximum is taken over the sample.
"""
from __future__ import annotations

import numpy as np


def errors(u, v, u_ref, v_ref):
    """Returns (e_max, e_rms, max |W_ref|)."""
    u = np.asarray(u, np.float64); v = np.asarray(v, np.float64)
    u_ref = np.asarray(u_ref, np.float64); v_ref = np.asarray(v_ref, np.float64)
    d = np.hypot(u - u_ref, v - v_ref)
    den = float(np.max(np.hypot(u_ref, v_ref))) if u_ref.size else 0.0
    if den == 0.0:
        den = 1.0
    return float(np.max(d)) / den, float(np.sqrt(np.mean(d * d))) / den, den


def log10_error_map(u, v, u_ref, v_ref, floor=1e-300):
    """Per-particle log10 |dW_i| / max|W_ref| (the spatial error maps of Section 5)."""
    _, _, den = errors(u, v, u_ref, v_ref)
    d = np.hypot(np.asarray(u) - u_ref, np.asarray(v) - v_ref) / den
    return np.log10(np.maximum(d, floor))
