"""Analytic 2-D homogeneous-medium response to a point source (test pin).

Test infrastructure only.  For (1/v^2) p_tt - lap p = w(t) delta(x - xs)
(Eq. 4 with the wavelet as the source term), the 2-D Green's function is
H(t - r/v) / (2 pi sqrt(t^2 - r^2/v^2)).  Convolved with w and substituted
tau = (r/v) cosh(s), the trace at distance r becomes the smooth integral

    p(r, t) = (1 / 2 pi) * int_0^{acosh(v t / r)} w(t - (r/v) cosh s) ds,

evaluated here by adaptive quadrature.  This is a closed form independent of
any finite-difference code.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import quad


def ricker_fn(fp: float, t0: float):
    def w(t):
        a = (math.pi * fp * (t - t0)) ** 2
        return (1.0 - 2.0 * a) * math.exp(-a) if t >= 0.0 else 0.0
    return w


def green_ricker_trace(r: float, v: float, times, fp: float = 15.0, t0: float | None = None):
    """p(r, t) for each t in `times` (seconds), Ricker source of peak fp."""
    if t0 is None:
        t0 = 1.5 / fp
    w = ricker_fn(fp, t0)
    out = np.zeros(len(times))
    for i, t in enumerate(times):
        if v * t <= r:
            continue
        smax = math.acosh(v * t / r)
        val, _ = quad(lambda s: w(t - (r / v) * math.cosh(s)), 0.0, smax, limit=400,
                      epsabs=1e-12, epsrel=1e-10)
        out[i] = val / (2.0 * math.pi)
    return out
