"""The seeded synthetic workloads (inputs only: meshes, models, layouts, times).

Names describe the workload:
  homog_kmv2_c1     2D homogeneous vp=1.5 km/s, 1 km x 1 km, 40x40 squares split
                    into 3200 right triangles (h = 25 m), KMV2, one 5 Hz Ricker at
                    the centre, 100 receivers 100 m below the top, T = 0.5 s,
                    dt = 0.5 ms (1000 steps), no damping; observed data from
                    vp = 1.6 km/s.
  layered_kmv4      2D 8 km x 3 km, 8 flat layers 1.5 -> 4.5 km/s plus 3 seeded
                    +-10 % Gaussian anomalies (r = 300 m); 750 m sponge on the
                    left, right and bottom; newest-vertex-bisection graded mesh
                    with leg <= s * vp / (5 Hz * 2.5) and 15 % seeded jitter,
                    s = 0.125 -> about 150k triangles; KMV4; one 5 Hz Ricker at
                    (4.0, 0.01) km; 300 receivers at z = 0.1 km; T = 4 s at
                    0.9 x the power-iteration CFL step.  Observed data from the
                    full model, current model = layers only.
  layered_kmv4_40shots  the same with 40 shots along the surface.
  serving_meshes    three layered/anomaly meshes of about 20k, 80k, 300k cells.
  gradient_check_2d the gradient-verification problem: 1 km x 1 km physical
                    domain, upper half 4.0 km/s and lower half 1.0 km/s (initial
                    model 4.0 km/s everywhere), a 200 m absorbing layer (sponge or
                    PML) on the left, right and bottom, uniform right triangles with
                    20 m legs (8400 cells), KMV2, a 5 Hz Ricker at 0.1 km depth,
                    100 receivers at 0.9 km depth from x = 0.1 to 0.9 km, T = 1 s,
                    dt = 0.5 ms.
  gradient_check_3d its 3D analogue: 1 km cube, 200 m sponge on the five faces
                    other than the top, Kuhn tetrahedra with 20 m box edges (1.76M
                    cells), KMV2tet, source at (0.5, 0.5, 0.1), a 10 x 10 receiver
                    grid at 0.9 km depth over [0.1, 0.9]^2, T = 1 s, dt = 0.5 ms.
  layered_tet_kmv3  3D 4 x 4 x 2 km layered + anomalies, 500 m sponge on five
                    faces, Maubach-graded Kuhn tetrahedra (shortest edge below
                    s * vp / (5 Hz * 2.5), s = 0.355 -> 1.33M tetrahedra, 16.9M KMV3 DOFs),
                    KMV3tet, 40x40 receiver grid, T = 2 s.  Observed data from
                    the full model, current model = layers only.
"""
from __future__ import annotations

import functools
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from .meshes import (structured_tri, nvb_graded_tri, jitter_vertices, kuhn_tet_box,
                     graded_tet_box)
from .models import (homogeneous_vp, layered_anomaly_vp, layered_anomaly_vp_3d, sponge_eta,
                     sponge_eta_3d, surface_receivers, surface_sources, grid_receivers_3d, pml_sigma,
                     pml_sigma_3d)


@dataclass
class Workload:
    name: str
    dim: int
    degree: int
    coords: np.ndarray
    cells: np.ndarray
    vp: Callable            # current model (function of point coordinates)
    vp_obs: Callable        # model that produces the observed data
    eta: Optional[Callable]  # damping eta(x) in 1/s, or None
    sources: np.ndarray     # [n_shots, dim]
    receivers: np.ndarray   # [n_rec, dim]
    T: float
    dt: Optional[float]     # None: cfl_fraction x the power-iteration bound
    f0: float = 5.0
    t0: float = 0.2
    amp: float = 1.0
    cfl_fraction: float = 0.9
    extra: dict = field(default_factory=dict)

    @property
    def n_cells(self):
        return len(self.cells)


def steps_for(T, dt_max):
    """Number of steps and step size: dt = T / ceil(T / dt_max)."""
    nt = int(np.ceil(T / dt_max - 1e-12))
    return nt, T / nt


@functools.lru_cache(maxsize=None)
def homog_kmv2_c1():
    coords, cells = structured_tri(40, 40, 0.0, 1.0, 0.0, 1.0)
    return Workload(
        name="homog_kmv2_c1", dim=2, degree=2, coords=coords, cells=cells,
        vp=homogeneous_vp(1.5), vp_obs=homogeneous_vp(1.6), eta=None,
        sources=np.array([[0.5, 0.5]]),
        receivers=surface_receivers(100, 0.1, 0.9, 0.1),
        T=0.5, dt=5e-4)


def _layered_mesh(seed, scale, jitter_seed):
    vp = layered_anomaly_vp(seed)

    def hfun(x, z):
        return scale * vp(x, z) / (5.0 * 2.5)

    coords, cells = nvb_graded_tri(hfun, -0.75, 8.75, 0.0, 3.75, 0.25)
    coords = jitter_vertices(coords, cells, 0.15, jitter_seed)
    return coords, cells


def _sponge2d(x, z):
    return sponge_eta(x, z, 0.0, 8.0, 3.0, 0.75, c_max=4.5)


def _pml2d(x, z):
    """The same 750 m layer as a PML: per-axis damping functions whose sum is the sponge."""
    return pml_sigma(x, z, 0.0, 8.0, 3.0, 0.75, c_max=4.5)


@functools.lru_cache(maxsize=None)
def layered_kmv4(seed=7, scale=0.125, degree=4, n_shots=1):
    coords, cells = _layered_mesh(seed, scale, seed + 1000)
    if n_shots == 1:
        src = np.array([[4.0, 0.01]])
    else:
        src = surface_sources(n_shots, 0.1, 7.9, 0.01)
    return Workload(
        name="layered_kmv4" if n_shots == 1 else f"layered_kmv4_{n_shots}shots",
        dim=2, degree=degree, coords=coords, cells=cells,
        vp=layered_anomaly_vp(seed, with_anomalies=False),
        vp_obs=layered_anomaly_vp(seed), eta=_sponge2d,
        sources=src, receivers=surface_receivers(300, 0.1, 7.9, 0.1),
        T=4.0, dt=None, extra={"seed": seed, "scale": scale, "sigma": _pml2d})


# mesh scale for ~20k, ~80k and ~300k triangles
SERVING_MESHES = ((11, 0.32), (12, 0.17), (13, 0.09))


@functools.lru_cache(maxsize=None)
def serving_mesh(i):
    seed, scale = SERVING_MESHES[i]
    coords, cells = _layered_mesh(seed, scale, seed + 1000)
    return coords, cells, layered_anomaly_vp(seed, with_anomalies=False), layered_anomaly_vp(seed)


@functools.lru_cache(maxsize=None)
def small_tri(n=8, degree=2, seed=3, jitter=0.15):
    """Small jittered unit-square mesh for unit tests."""
    coords, cells = structured_tri(n, n, 0.0, 1.0, 0.0, 1.0)
    if jitter > 0:
        coords = jitter_vertices(coords, cells, jitter, seed)
    return coords, cells


@functools.lru_cache(maxsize=None)
def small_tet(n=3, seed=3, jitter=0.15):
    coords, cells = kuhn_tet_box(n, n, n, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    if jitter > 0:
        coords = jitter_vertices(coords, cells, jitter, seed)
    return coords, cells


def _sponge3d(x, y, z):
    return sponge_eta_3d(x, y, z, (0.0, 0.0, 0.0), (4.0, 4.0, 2.0), 0.5, c_max=4.5)


@functools.lru_cache(maxsize=None)
def layered_tet_kmv3(seed=21, coarse_h=0.5, scale=0.355):
    vp = layered_anomaly_vp_3d(seed)

    def hfun(x, y, z):
        return scale * vp(x, y, z) / (5.0 * 2.5)

    coords, cells = graded_tet_box(hfun, (-0.5, -0.5, 0.0), (4.5, 4.5, 2.5), coarse_h)
    coords = jitter_vertices(coords, cells, 0.15, seed + 1000)
    return Workload(
        name="layered_tet_kmv3", dim=3, degree=3, coords=coords, cells=cells,
        vp=layered_anomaly_vp_3d(seed, n_anom=0), vp_obs=vp, eta=_sponge3d,
        sources=np.array([[2.0, 2.0, 0.01]]),
        receivers=grid_receivers_3d(40, 40, (0.1, 0.1), (3.9, 3.9), 0.1),
        T=2.0, dt=None, extra={"seed": seed, "scale": scale})


def _half_space(v_top, v_bottom, depth):
    """v_top above the depth, v_bottom at and below it."""
    def f(*xs):
        return np.where(np.asarray(xs[-1], dtype=np.float64) < depth, float(v_top), float(v_bottom))
    return f


@functools.lru_cache(maxsize=None)
def gradient_check_2d(le=0.02, width=0.2):
    """The paper's 2D gradient-verification problem (a reading of its layout: the
    slow half is the lower one, between source and receivers, so the experiment is
    a transmission through the interface).  extra['sigma'](x, z) gives the PML's
    per-axis damping functions; eta is their sum (the sponge)."""
    nx, nz = int(round((1.0 + 2 * width) / le)), int(round((1.0 + width) / le))
    coords, cells = structured_tri(nx, nz, -width, 1.0 + width, 0.0, 1.0 + width)
    c_max = 4.0

    def eta(x, z):
        return sponge_eta(x, z, 0.0, 1.0, 1.0, width, c_max=c_max)

    def sigma(x, z):
        return pml_sigma(x, z, 0.0, 1.0, 1.0, width, c_max=c_max)

    return Workload(
        name="gradient_check_2d", dim=2, degree=2, coords=coords, cells=cells,
        vp=homogeneous_vp(4.0), vp_obs=_half_space(4.0, 1.0, 0.5), eta=eta,
        sources=np.array([[0.5, 0.1]]), receivers=surface_receivers(100, 0.1, 0.9, 0.9),
        T=1.0, dt=5e-4, extra={"sigma": sigma, "width": width, "le": le})


@functools.lru_cache(maxsize=None)
def gradient_check_3d(le=0.02, width=0.2):
    """The 3D analogue of gradient_check_2d (sponge on five faces)."""
    n = int(round((1.0 + 2 * width) / le))
    nzz = int(round((1.0 + width) / le))
    coords, cells = kuhn_tet_box(n, n, nzz, (-width, -width, 0.0), (1.0 + width, 1.0 + width, 1.0 + width))
    c_max = 4.0

    def eta(x, y, z):
        return sponge_eta_3d(x, y, z, (0.0, 0.0), (1.0, 1.0, 1.0), width, c_max=c_max)

    def sigma(x, y, z):
        return pml_sigma_3d(x, y, z, (0.0, 0.0), (1.0, 1.0, 1.0), width, c_max=c_max)

    return Workload(
        name="gradient_check_3d", dim=3, degree=2, coords=coords, cells=cells,
        vp=homogeneous_vp(4.0), vp_obs=_half_space(4.0, 1.0, 0.5), eta=eta,
        sources=np.array([[0.5, 0.5, 0.1]]), receivers=grid_receivers_3d(10, 10, (0.1, 0.1), (0.9, 0.9), 0.9),
        T=1.0, dt=5e-4, extra={"sigma": sigma, "width": width, "le": le})
