"""Error estimates of Section 4 (kernel substitution and expansion truncation).

Test infrastructure (see ``oracle/__init__``).

Section 4.1: the far field replaces the regularised kernel (eq. 26) by the
singular one (eq. 27).  For a single pair at distance r the two kernels differ by
exactly exp(-r^2 / 2 sigma^2) / (2 pi r) in magnitude, which decreases with r; so
for every far pair at distance >= a,

    |u_sigma - u'| <= sum_far |Gamma_j| exp(-a^2 / 2 sigma^2) / (2 pi a).

Readings: eq. 26-29 print exp(-|z| / 2 sigma^2) (taken as |z|^2, as in eq. 3,
6 and 13) and drop the 1 / (2 pi a) factor; the magnitude uses sum |Gamma_j|.
Table 1 uses the leaf box side as a, for sigma = 0.02 and total circulation 1;
its four values differ from each other exactly as log10 of the expression above
does, and all sit a constant 0.055 below it (a factor of about 0.881 that the
paper does not explain).

Section 4.2: for sources within radius r of the expansion centre and an
evaluation point y with |r / (y - x_*)| <= b (eq. 31), the truncation error of a
p-term ME is at most A b^p / (|y - x_*| (1 - b)) with A = sum |Gamma_i| / (2 pi)
(the printed derivation writes |sum Gamma_i / 2 pi| and sums |b| instead of
|b|^m; the geometric series gives b^p / (1 - b)).
"""
from __future__ import annotations

import math

import numpy as np


def pair_kernel_gap(r, sigma):
    """|K_sigma - K'| for one unit-circulation pair at distance r (eq. 6 vs eq. 27)."""
    r = np.asarray(r, np.float64)
    return np.exp(-r * r / (2.0 * sigma * sigma)) / (2.0 * math.pi * r)


def kernel_substitution_bound(a, sigma, abs_circulation):
    """Section 4.1 bound for all far pairs at distance >= a."""
    return abs_circulation * pair_kernel_gap(a, sigma)


def log10_kernel_estimate(a, sigma, circulation=1.0):
    """log10 of the Section 4.1 estimate with minimum far distance a (Table 1 form)."""
    return math.log10(circulation) - a * a / (2.0 * sigma * sigma) / math.log(10.0) \
        - math.log10(2.0 * math.pi * a)


def me_truncation_bound(abs_circulation, radius, dist, p):
    """Section 4.2: bound on the error of a p-term ME at distance ``dist``."""
    b = radius / dist
    if not b < 1.0:
        return math.inf
    a = abs_circulation / (2.0 * math.pi)
    return a * b ** p / (dist * (1.0 - b))
