"""Closed-form 2D homogeneous solution — oracle accuracy pin, test infrastructure.

For u_tt - c^2 Lap u = w(t) delta(x - x_s) in the plane, with zero initial data,
convolving the 2D Green's function H(ct - r) / (2 pi c sqrt(c^2 t^2 - r^2)) with w
and substituting c tau = r cosh(sigma) gives

    u(r, t) = 1/(2 pi c^2) * integral_0^{arccosh(ct/r)} w(t - (r/c) cosh sigma) dsigma

for t > r/c and 0 otherwise.  The integrand is smooth, so Gauss-Legendre
quadrature (numpy's leggauss) converges quickly.
"""
from __future__ import annotations

import numpy as np


def green2d_trace(r, t, c, wavelet_fn, n_gauss=400):
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    out = np.zeros_like(t)
    xg, wg = np.polynomial.legendre.leggauss(n_gauss)
    for i, ti in enumerate(t):
        if c * ti <= r:
            continue
        smax = np.arccosh(c * ti / r)
        s = 0.5 * smax * (xg + 1.0)
        out[i] = 0.5 * smax * np.sum(wg * wavelet_fn(ti - (r / c) * np.cosh(s)))
    return out / (2.0 * np.pi * c * c)
