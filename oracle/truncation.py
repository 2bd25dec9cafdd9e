"""Truncation error of the support radius (paper Sect. 4), from its
definition in FP64.  TEST INFRASTRUCTURE ONLY (see the package docstring).

With K_l = 2 pi int_{-1}^{1} K(z) P_l(z) dz (Sect. 2), cutting the kernel
at radius R changes its Legendre coefficients by

    dK_l(R) = -2 pi int_R^pi K(theta) P_l(cos theta) sin theta dtheta,

and a signal of angular power spectrum C_l then sees an error of variance

    sigma^2(R) = sum_l (2l + 1) / (4 pi) dK_l(R)^2 C_l.

The integral is a composite Simpson rule on a uniform grid (the kernel
from the oracle's own evaluator, untruncated), P_l from scipy, over
[R, theta_max] for a spline (zero beyond) and [R, min(pi, 40 sigma)] for a
Gaussian (whose FP64 value is exactly zero beyond 38.6 sigma).
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special

from . import kernel


def _support_end(profile):
    if profile.kind == "gaussian":
        return min(math.pi, 40.0 * profile.fwhm / math.sqrt(8.0 * math.log(2.0)))
    return min(math.pi, float(profile.theta_max))


def tail_coefficients(profile, radius, lmax, per_period=32, min_points=20001):
    """dK_l(R) for l = 0..lmax."""
    a, b = float(radius), _support_end(profile)
    if not a < b:
        return np.zeros(lmax + 1)
    n = max(min_points, int(per_period * (b - a) * (lmax + 1) / (2 * math.pi)) + 1)
    n += (n + 1) % 2  # odd number of points: even number of Simpson intervals
    t = np.linspace(a, b, n)
    w = np.full(n, 2.0)
    w[1::2] = 4.0
    w[0] = w[-1] = 1.0
    w *= (b - a) / (n - 1) / 3.0
    f = kernel(profile, math.pi + 1.0, t) * np.sin(t) * w
    z = np.cos(t)
    return np.array([-2.0 * math.pi * np.dot(f, special.eval_legendre(l, z)) for l in range(lmax + 1)])


def truncation_variance(profile, radius, cl):
    """sigma^2(R) for the power spectrum cl[0..lmax]."""
    cl = np.asarray(cl, dtype=np.float64)
    lmax = cl.size - 1
    dk = tail_coefficients(profile, radius, lmax)
    l = np.arange(lmax + 1)
    return float(np.sum((2 * l + 1) / (4 * math.pi) * dk ** 2 * cl)), dk
