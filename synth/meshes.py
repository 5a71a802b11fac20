"""Seeded simplicial mesh generators (inputs only; no finite-element arithmetic).

* ``structured_tri``   — right-triangle grid, every square split along its
  (i,j)->(i+1,j+1) diagonal.
* ``nvb_graded_tri``   — waveform-adapted grading by newest-vertex bisection of a
  coarse right-triangle grid until every triangle's leg is below a local size
  h(x) (the cells-per-wavelength sizing rule of the paper's waveform-adapted mesh
  section, eq. gpwl), with conforming closure.
* ``jitter_vertices``  — seeded interior-vertex jitter that rejects moves which
  invert or degrade a cell.
* ``kuhn_tet_box`` / ``graded_tet_box`` — Kuhn (6 tets per cube) lattices, optionally
  graded by Maubach bisection, for the tetrahedral cases.

Coordinates are (x, z) in 2D and (x, y, z) in 3D, km, z >= 0 downward.
"""
from __future__ import annotations

import sys
import numpy as np


# ----------------------------------------------------------------------------- 2D
def structured_tri(nx: int, nz: int, x0: float, x1: float, z0: float, z1: float):
    """Right-triangle grid of nx*nz squares, each split along the (i,j)->(i+1,j+1)
    diagonal.  Cells list their diagonal (the newest-vertex refinement edge) first
    and the right-angle corner last.  Returns (coords[Nv,2] f64, cells[Ne,3] i32)."""
    xs = np.linspace(x0, x1, nx + 1)
    zs = np.linspace(z0, z1, nz + 1)
    X, Z = np.meshgrid(xs, zs, indexing="ij")
    coords = np.stack([X.ravel(), Z.ravel()], axis=1)
    i, j = np.meshgrid(np.arange(nx), np.arange(nz), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    v00 = i * (nz + 1) + j
    v10 = (i + 1) * (nz + 1) + j
    v11 = (i + 1) * (nz + 1) + j + 1
    v01 = i * (nz + 1) + j + 1
    t1 = np.stack([v00, v11, v10], axis=1)
    t2 = np.stack([v11, v00, v01], axis=1)
    cells = np.empty((2 * len(i), 3), dtype=np.int64)
    cells[0::2] = t1
    cells[1::2] = t2
    return coords, cells.astype(np.int32)


class _NVB2D:
    """Newest-vertex bisection with conforming closure.  A triangle (a, b, c) has
    refinement edge (a, b) and newest vertex c; bisection at the midpoint m of (a, b)
    yields (c, a, m) and (b, c, m)."""

    def __init__(self, coords, cells):
        self.V = [tuple(p) for p in np.asarray(coords, dtype=np.float64)]
        self.T = [list(map(int, t)) for t in cells]
        self.alive = [True] * len(self.T)
        self.edges = {}
        self.mid = {}
        for t in range(len(self.T)):
            self._link(t)

    @staticmethod
    def _key(a, b):
        return (a, b) if a < b else (b, a)

    def _link(self, t):
        a, b, c = self.T[t]
        for e in (self._key(a, b), self._key(b, c), self._key(c, a)):
            self.edges.setdefault(e, []).append(t)

    def _unlink(self, t):
        a, b, c = self.T[t]
        for e in (self._key(a, b), self._key(b, c), self._key(c, a)):
            lst = self.edges[e]
            lst.remove(t)
            if not lst:
                del self.edges[e]
        self.alive[t] = False

    def _add(self, tri):
        self.T.append(tri)
        self.alive.append(True)
        self._link(len(self.T) - 1)

    def _neighbor(self, key, t):
        for s in self.edges.get(key, ()):
            if s != t:
                return s
        return None

    def _midpoint(self, key):
        m = self.mid.get(key)
        if m is None:
            pa, pb = self.V[key[0]], self.V[key[1]]
            self.V.append(((pa[0] + pb[0]) * 0.5, (pa[1] + pb[1]) * 0.5))
            m = len(self.V) - 1
            self.mid[key] = m
        return m

    def bisect(self, t):
        a, b, c = self.T[t]
        key = self._key(a, b)
        while True:
            nb = self._neighbor(key, t)
            if nb is None:
                break
            na, nbv, _ = self.T[nb]
            if self._key(na, nbv) == key:
                break
            self.bisect(nb)
        m = self._midpoint(key)
        self._unlink(t)
        self._add([c, a, m])
        self._add([b, c, m])
        if nb is not None:
            na, nbv, nc = self.T[nb]
            self._unlink(nb)
            self._add([nc, na, m])
            self._add([nbv, nc, m])

    def arrays(self):
        coords = np.array(self.V, dtype=np.float64)
        cells = np.array([t for t, ok in zip(self.T, self.alive) if ok], dtype=np.int32)
        return coords, cells


def nvb_graded_tri(hfun, x0, x1, z0, z1, coarse_h, max_rounds=60):
    """Graded conforming triangle mesh of the box [x0,x1]x[z0,z1].

    Starts from a right-triangle grid with legs close to ``coarse_h`` and bisects
    (newest-vertex, with closure) every triangle whose leg exceeds ``hfun`` at its
    centroid, round after round, until none does.  ``hfun(x, z)`` takes arrays."""
    nx = max(1, int(round((x1 - x0) / coarse_h)))
    nz = max(1, int(round((z1 - z0) / coarse_h)))
    coords, cells = structured_tri(nx, nz, x0, x1, z0, z1)
    nvb = _NVB2D(coords, cells)
    old = sys.getrecursionlimit()
    sys.setrecursionlimit(max(old, 100000))
    try:
        for _ in range(max_rounds):
            ids = [t for t, ok in enumerate(nvb.alive) if ok]
            tri = np.array([nvb.T[t] for t in ids], dtype=np.int64)
            V = np.array(nvb.V)
            pa, pb, pc = V[tri[:, 0]], V[tri[:, 1]], V[tri[:, 2]]
            leg = np.linalg.norm(pa - pb, axis=1) / np.sqrt(2.0)
            cen = (pa + pb + pc) / 3.0
            h = hfun(cen[:, 0], cen[:, 1])
            marked = [ids[k] for k in np.nonzero(leg > h)[0]]
            if not marked:
                break
            for t in marked:
                if nvb.alive[t]:
                    nvb.bisect(t)
    finally:
        sys.setrecursionlimit(old)
    return nvb.arrays()


def _signed_area(coords, cells):
    p0, p1, p2 = coords[cells[:, 0]], coords[cells[:, 1]], coords[cells[:, 2]]
    return 0.5 * ((p1[:, 0] - p0[:, 0]) * (p2[:, 1] - p0[:, 1])
                  - (p1[:, 1] - p0[:, 1]) * (p2[:, 0] - p0[:, 0]))


def mesh_quality_tri(coords, cells):
    """Per-cell shape quality 4*sqrt(3)*|A| / sum(l^2) (1 for equilateral)."""
    p0, p1, p2 = coords[cells[:, 0]], coords[cells[:, 1]], coords[cells[:, 2]]
    l2 = (np.sum((p1 - p0) ** 2, 1) + np.sum((p2 - p1) ** 2, 1) + np.sum((p0 - p2) ** 2, 1))
    return 4.0 * np.sqrt(3.0) * np.abs(_signed_area(coords, cells)) / l2


def _boundary_vertices(coords, tol=1e-9):
    lo = coords.min(axis=0)
    hi = coords.max(axis=0)
    on = np.zeros(len(coords), dtype=bool)
    for d in range(coords.shape[1]):
        on |= np.abs(coords[:, d] - lo[d]) < tol
        on |= np.abs(coords[:, d] - hi[d]) < tol
    return on


def _vertex_min_edge(coords, cells):
    nv = len(coords)
    hmin = np.full(nv, np.inf)
    nvc = cells.shape[1]
    for i in range(nvc):
        for j in range(i + 1, nvc):
            a, b = cells[:, i], cells[:, j]
            le = np.linalg.norm(coords[a] - coords[b], axis=1)
            np.minimum.at(hmin, a, le)
            np.minimum.at(hmin, b, le)
    return hmin


def _signed_volume(coords, cells):
    p0 = coords[cells[:, 0]]
    a = coords[cells[:, 1]] - p0
    b = coords[cells[:, 2]] - p0
    c = coords[cells[:, 3]] - p0
    return np.einsum("ij,ij->i", a, np.cross(b, c)) / 6.0


def jitter_vertices(coords, cells, frac=0.15, seed=0, min_ratio=0.5):
    """Move every interior vertex by a seeded uniform offset in the ball of radius
    ``frac`` x (its shortest incident edge).  Moves that shrink an incident cell's
    signed measure below ``min_ratio`` of its original value (inverting or
    degrading it) are undone, repeatedly, until no cell is degraded."""
    coords = np.asarray(coords, dtype=np.float64)
    cells = np.asarray(cells)
    dim = coords.shape[1]
    rng = np.random.default_rng(seed)
    nv = len(coords)
    h = _vertex_min_edge(coords, cells)
    if dim == 2:
        r = frac * h * np.sqrt(rng.random(nv))
        th = 2.0 * np.pi * rng.random(nv)
        disp = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
        measure = _signed_area
    else:
        d = rng.normal(size=(nv, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        r = frac * h * np.cbrt(rng.random(nv))
        disp = d * r[:, None]
        measure = _signed_volume
    moving = ~_boundary_vertices(coords)
    m0 = measure(coords, cells)
    while True:
        new = coords + disp * moving[:, None]
        ratio = measure(new, cells) / m0
        bad = ratio < min_ratio
        if not bad.any():
            return new
        moving[np.unique(cells[bad].ravel())] = False


# ----------------------------------------------------------------------------- 3D
_KUHN_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def kuhn_tet_box(nx, ny, nz, lo, hi):
    """Kuhn lattice: nx*ny*nz boxes, each split into 6 tetrahedra sharing the box
    diagonal; vertex order (v000, v000+e_p0, v000+e_p0+e_p1, v111) so that Maubach
    bisection with tag 3 starts on the diagonal.  Returns (coords[Nv,3], cells[Ne,4])."""
    n = np.array([nx, ny, nz])
    axes = [np.linspace(lo[d], hi[d], n[d] + 1) for d in range(3)]
    X, Y, Z = np.meshgrid(*axes, indexing="ij")
    coords = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    strides = np.array([(ny + 1) * (nz + 1), nz + 1, 1])
    I, J, K = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    base = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    out = []
    for p in _KUHN_PERMS:
        e0 = np.zeros(3, dtype=np.int64)
        e0[p[0]] = 1
        e1 = e0.copy()
        e1[p[1]] = 1
        v0 = base @ strides
        v1 = (base + e0) @ strides
        v2 = (base + e1) @ strides
        v3 = (base + 1) @ strides
        out.append(np.stack([v0, v1, v2, v3], axis=1))
    cells = np.stack(out, axis=1).reshape(-1, 4)
    return coords, cells.astype(np.int32)


class _Maubach3D:
    """Maubach bisection of tagged tetrahedra with conforming closure.

    A tetrahedron (x0, x1, x2, x3) with tag k has refinement edge (x0, xk); with z
    its midpoint the children are (x0..x_{k-1}, z, x_{k+1}..x3) and
    (x1..xk, z, x_{k+1}..x3), both tagged k-1 (or 3 when k == 1)."""

    def __init__(self, coords, cells):
        self.V = [tuple(p) for p in np.asarray(coords, dtype=np.float64)]
        self.T = [list(map(int, t)) for t in cells]
        self.tag = [3] * len(self.T)
        self.alive = [True] * len(self.T)
        self.edges = {}
        self.mid = {}
        for t in range(len(self.T)):
            self._link(t)

    @staticmethod
    def _key(a, b):
        return (a, b) if a < b else (b, a)

    def _tet_edges(self, t):
        v = self.T[t]
        return [self._key(v[i], v[j]) for i in range(4) for j in range(i + 1, 4)]

    def _link(self, t):
        for e in self._tet_edges(t):
            self.edges.setdefault(e, set()).add(t)

    def _unlink(self, t):
        for e in self._tet_edges(t):
            s = self.edges[e]
            s.discard(t)
            if not s:
                del self.edges[e]
        self.alive[t] = False

    def _refedge(self, t):
        v = self.T[t]
        return self._key(v[0], v[self.tag[t]])

    def _midpoint(self, key):
        m = self.mid.get(key)
        if m is None:
            pa, pb = self.V[key[0]], self.V[key[1]]
            self.V.append(tuple((pa[i] + pb[i]) * 0.5 for i in range(3)))
            m = len(self.V) - 1
            self.mid[key] = m
        return m

    def _split(self, t, m):
        v = self.T[t]
        k = self.tag[t]
        c1 = v[:k] + [m] + v[k + 1:]
        c2 = v[1:k + 1] + [m] + v[k + 1:]
        nk = k - 1 if k > 1 else 3
        self._unlink(t)
        for c in (c1, c2):
            self.T.append(c)
            self.tag.append(nk)
            self.alive.append(True)
            self._link(len(self.T) - 1)

    def bisect(self, t):
        key = self._refedge(t)
        while True:
            ring = list(self.edges.get(key, ()))
            pending = [s for s in ring if self._refedge(s) != key]
            if not pending:
                break
            self.bisect(pending[0])
        m = self._midpoint(key)
        for s in list(self.edges.get(key, ())):
            self._split(s, m)

    def arrays(self):
        coords = np.array(self.V, dtype=np.float64)
        cells = np.array([t for t, ok in zip(self.T, self.alive) if ok], dtype=np.int32)
        return coords, cells


def graded_tet_box(hfun, lo, hi, coarse_h, max_rounds=60):
    """Graded conforming tetrahedral mesh of a box: a Kuhn lattice of cubes near
    ``coarse_h`` refined by Maubach bisection until every tetrahedron's shortest
    edge is below ``hfun`` at its centroid."""
    n = [max(1, int(round((hi[d] - lo[d]) / coarse_h))) for d in range(3)]
    coords, cells = kuhn_tet_box(n[0], n[1], n[2], lo, hi)
    mb = _Maubach3D(coords, cells)
    old = sys.getrecursionlimit()
    sys.setrecursionlimit(max(old, 100000))
    try:
        for _ in range(max_rounds):
            ids = [t for t, ok in enumerate(mb.alive) if ok]
            tet = np.array([mb.T[t] for t in ids], dtype=np.int64)
            V = np.array(mb.V)
            P = V[tet]
            emin = np.full(len(ids), np.inf)
            for i in range(4):
                for j in range(i + 1, 4):
                    emin = np.minimum(emin, np.linalg.norm(P[:, i] - P[:, j], axis=1))
            cen = P.mean(axis=1)
            h = hfun(cen[:, 0], cen[:, 1], cen[:, 2])
            marked = [ids[k] for k in np.nonzero(emin > h)[0]]
            if not marked:
                break
            for t in marked:
                if mb.alive[t]:
                    mb.bisect(t)
    finally:
        sys.setrecursionlimit(old)
    return mb.arrays()
