"""TEST INFRASTRUCTURE ONLY -- the paper's parameter rules, written out.

Sec. 5.1: for a chosen x,y grid N_xy on side L, the spacing h = L/N_xy fixes
g_t = 1.2 h (about 3 digits, n_g = 10) or g_t = 1.4 h (about 4 digits,
n_g = 12); xi follows from eq. gt, H_E = n_g h/2 (eq. He) and the number of
Chebyshev nodes is ceil(pi Hbar/(2h)) with Hbar = H + 6 H_E the height of the
extended domain of Sec. 5.2.2. The near cutoff r_nf is the smallest r at which
the ratio of eq. rnf drops below delta.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special


def paper_rule(L: float, n_xy: int, H: float, g_w: float, four_digits: bool):
    h = L / n_xy
    g_t = (1.4 if four_digits else 1.2) * h
    n_g = 12 if four_digits else 10
    xi = 1.0 / (2.0 * math.sqrt(g_t * g_t - g_w * g_w))
    H_E = n_g * h / 2.0
    n_z = math.ceil(math.pi * (H + 6.0 * H_E) / (2.0 * h))
    return dict(h=h, g_t=g_t, n_g=n_g, xi=xi, H_E=H_E, n_sigma=H_E / g_t, Nz=n_z)


def _dG(r, g_w, xi):
    """d/dr of [erf(r/(sqrt2 g_w)) - erf(r/sqrt(2 g_w^2 + xi^-2))]/r (eq. Gnear
    without 1/(4 pi eps)); xi = 0 drops the second term."""
    def term(r, s):  # d/dr erf(r/s)/r
        if s == 0.0:
            return -1.0 / r ** 2
        return (2.0 / math.sqrt(math.pi)) * math.exp(-(r / s) ** 2) / (s * r) - math.erf(r / s) / r ** 2
    t1 = term(r, math.sqrt(2.0) * g_w)
    if xi == 0.0:
        return t1
    return t1 - term(r, math.sqrt(2.0 * g_w ** 2 + 1.0 / xi ** 2))


def r_nf(g_w: float, xi: float, delta: float) -> float:
    """Smallest r with |dG(r;g_w,xi)/dG(r;g_w,0)| < delta (eq. rnf)."""
    def ratio(r):
        return abs(_dG(r, g_w, xi) / _dG(r, g_w, 0.0))
    lo = 1e-6 / xi
    r = lo
    step = 0.01 / xi
    while ratio(r) >= delta:
        r += step
        if r > 100.0 / xi:
            raise RuntimeError("no cutoff found")
    hi = r
    lo = r - step
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        if ratio(mid) < delta:
            hi = mid
        else:
            lo = mid
    return hi
