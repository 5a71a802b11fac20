"""Seeded P-wavespeed models, damping profiles and acquisition layouts (inputs only).

Units: km, s, km/s.  2D points are (x, z), 3D points (x, y, z), z >= 0 downward.
"""
from __future__ import annotations

import numpy as np


def homogeneous_vp(vp):
    """Constant model; returns a function of point arrays."""
    def f(*xs):
        return np.full(np.shape(xs[0]), float(vp))
    return f


def _anomaly_centres(seed, n, lo, hi):
    rng = np.random.default_rng(seed)
    centres = lo + (np.asarray(hi) - np.asarray(lo)) * rng.random((n, len(lo)))
    signs = np.where(rng.random(n) < 0.5, -1.0, 1.0)
    return centres, signs


def layered_anomaly_vp(seed, n_layers=8, vmin=1.5, vmax=4.5, depth=3.0,
                       n_anom=3, amp=0.10, radius=0.3,
                       anom_lo=(1.0, 0.5), anom_hi=(7.0, 2.5), with_anomalies=True):
    """Flat layers, vp rising linearly in layer index from vmin to vmax over ``depth``
    (the deepest layer continues below), times 1 + sum_a s_a*amp*exp(-|x-x_a|^2/r^2)
    for ``n_anom`` seeded Gaussian anomalies of sign s_a = +-1."""
    centres, signs = _anomaly_centres(seed, n_anom, np.array(anom_lo), np.array(anom_hi))
    dz = depth / n_layers

    def f(x, z):
        x = np.asarray(x, dtype=np.float64)
        z = np.asarray(z, dtype=np.float64)
        idx = np.minimum(np.floor(np.maximum(z, 0.0) / dz), n_layers - 1)
        v = vmin + (vmax - vmin) * idx / (n_layers - 1)
        if with_anomalies:
            pert = np.zeros_like(v)
            for (ax, az), s in zip(centres, signs):
                pert += s * amp * np.exp(-((x - ax) ** 2 + (z - az) ** 2) / radius ** 2)
            v = v * (1.0 + pert)
        return v
    f.centres = centres
    f.signs = signs
    return f


def layered_anomaly_vp_3d(seed, n_layers=8, vmin=1.5, vmax=4.5, depth=2.0,
                          n_anom=3, amp=0.10, radius=0.3,
                          anom_lo=(0.5, 0.5, 0.3), anom_hi=(3.5, 3.5, 1.7)):
    """3D analogue of ``layered_anomaly_vp``."""
    centres, signs = _anomaly_centres(seed, n_anom, np.array(anom_lo), np.array(anom_hi))
    dz = depth / n_layers

    def f(x, y, z):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        z = np.asarray(z, dtype=np.float64)
        idx = np.minimum(np.floor(np.maximum(z, 0.0) / dz), n_layers - 1)
        v = vmin + (vmax - vmin) * idx / (n_layers - 1)
        pert = np.zeros_like(v)
        for (ax, ay, az), s in zip(centres, signs):
            pert += s * amp * np.exp(-((x - ax) ** 2 + (y - ay) ** 2 + (z - az) ** 2) / radius ** 2)
        return v * (1.0 + pert)
    return f


def sponge_eta(x, z, x_lo, x_hi, z_hi, width, c_max, R=1e-3):
    """Quadratic damping profile eta(x) = sum_k eta_max (d_k/L)^2 in a layer of width
    L outside the physical box [x_lo, x_hi] x [0, z_hi] (left, right, bottom; the top
    is open), zero inside; eta_max = 3 c_max ln(1/R) / (2L).  This is the paper's
    quadratic damping function sigma_i, used as the trace of the damping matrix."""
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    eta_max = 3.0 * c_max * np.log(1.0 / R) / (2.0 * width)
    dx = np.maximum(x_lo - x, 0.0) + np.maximum(x - x_hi, 0.0)
    dz = np.maximum(z - z_hi, 0.0)
    return eta_max * ((dx / width) ** 2 + (dz / width) ** 2)


def pml_sigma(x, z, x_lo, x_hi, z_hi, width, c_max, R=1e-3):
    """Per-axis damping functions of the PML, sigma_x and sigma_z, each the quadratic
    sigma_max (d_k/L)^2 of the distance d_k into the layer along its axis (left and
    right layers: sigma_x; bottom layer: sigma_z; the top is open), zero inside the
    physical box; sigma_max = 3 c_max ln(1/R) / (2L).  Returns [n, 2]; their sum is
    sponge_eta."""
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    s_max = 3.0 * c_max * np.log(1.0 / R) / (2.0 * width)
    dx = np.maximum(x_lo - x, 0.0) + np.maximum(x - x_hi, 0.0)
    dz = np.maximum(z - z_hi, 0.0)
    return np.stack([s_max * (dx / width) ** 2, s_max * (dz / width) ** 2], axis=1)


def pml_sigma_3d(x, y, z, lo, hi, width, c_max, R=1e-3):
    """3D per-axis damping functions (sigma_x, sigma_y, sigma_z) on the five faces
    other than the top z = 0.  Returns [n, 3]; their sum is sponge_eta_3d."""
    s_max = 3.0 * c_max * np.log(1.0 / R) / (2.0 * width)
    d = [np.maximum(lo[0] - x, 0.0) + np.maximum(x - hi[0], 0.0),
         np.maximum(lo[1] - y, 0.0) + np.maximum(y - hi[1], 0.0),
         np.maximum(z - hi[2], 0.0)]
    return np.stack([s_max * (di / width) ** 2 for di in d], axis=1)


def sponge_eta_3d(x, y, z, lo, hi, width, c_max, R=1e-3):
    """3D version of ``sponge_eta`` on the five faces other than the top z = 0."""
    eta_max = 3.0 * c_max * np.log(1.0 / R) / (2.0 * width)
    d = [np.maximum(lo[0] - x, 0.0) + np.maximum(x - hi[0], 0.0),
         np.maximum(lo[1] - y, 0.0) + np.maximum(y - hi[1], 0.0),
         np.maximum(z - hi[2], 0.0)]
    return eta_max * sum((di / width) ** 2 for di in d)


def surface_receivers(n, x0, x1, z):
    """n receivers evenly spaced on the line z = const between x0 and x1."""
    x = np.linspace(x0, x1, n)
    return np.stack([x, np.full(n, float(z))], axis=1)


def surface_sources(n, x0, x1, z):
    return surface_receivers(n, x0, x1, z)


def grid_receivers_3d(nx, ny, lo, hi, z):
    xs = np.linspace(lo[0], hi[0], nx)
    ys = np.linspace(lo[1], hi[1], ny)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, float(z))], axis=1)
