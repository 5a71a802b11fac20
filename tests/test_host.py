"""CPU tests of the HIP library's host side through the C ABI (no GPU calls):
the library loads and exports every declared symbol, its element tables, DOF
numbering, lumped mass, boundary mass and Gershgorin bound agree with the oracle's
independent construction, and its scheduling invariants and error codes hold."""
import os
import re

import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_2108_10946_amd import kmvwave as K
from paper_2108_10946_amd.api import Mesh
from oracle.elements import kmv_element
from oracle.fem import Discretization
from oracle import solver
from synth import configs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ALL = [(2, 1), (2, 2), (2, 3), (2, 4), (2, 5), (3, 1), (3, 2), (3, 3)]


def header_symbols():
    txt = open(os.path.join(ROOT, "include", "kmvwave.h")).read()
    return sorted(set(re.findall(r"\b(kmv_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = K.lib()
    declared = header_symbols()
    assert sorted(K.DECLARED) == declared
    for name in declared:
        assert hasattr(L, name), name


def match(a, b, tol=1e-10):
    """Permutation p with a[i] == b[p[i]] (points)."""
    d, p = cKDTree(b).query(a)
    assert np.all(d < tol) and len(set(p)) == len(p)
    return p


@pytest.mark.parametrize("dk", ALL)
def test_element_tables_match_oracle(dk):
    nodes, w, D = K.kmv_element_tables(*dk)
    e = kmv_element(*dk)
    p = match(nodes, e.nodes, 1e-14)
    assert np.allclose(w, e.weights[p], rtol=0, atol=1e-16)
    # D[q, a, r] with both node indices permuted
    assert np.allclose(D, e.D[np.ix_(p, p)], rtol=0, atol=1e-10 * np.abs(e.D).max())


def test_unsupported_degree():
    with pytest.raises(K.KMVError) as ei:
        K.kmv_element_tables(2, 6)
    assert ei.value.code == K.KMV_EDEGREE
    coords, cells = configs.small_tri(3)
    with pytest.raises(K.KMVError) as ei:
        Mesh(coords, cells, 4 if False else 7)
    assert ei.value.code == K.KMV_EDEGREE


def test_bad_meshes():
    coords, cells = configs.small_tri(3)
    bad = cells.copy()
    bad[0, 0] = len(coords) + 5
    with pytest.raises(K.KMVError) as ei:
        Mesh(coords, bad, 2)
    assert ei.value.code == K.KMV_EMESH
    degen = cells.copy()
    degen[0] = [degen[0, 0], degen[0, 0], degen[0, 1]]
    with pytest.raises(K.KMVError) as ei:
        Mesh(coords, degen, 2)
    assert ei.value.code == K.KMV_EMESH
    # one GPU thread per cell in workgroups of at most 256 threads
    for pc in (-1, 257):
        with pytest.raises(K.KMVError) as ei:
            Mesh(coords, cells, 2, patch_cells=pc)
        assert ei.value.code == K.KMV_EINVAL
    assert Mesh(coords, cells, 2, patch_cells=256).patch_stats()["max_patch_cells"] <= 256


MESHES = {
    "tri": lambda: configs.small_tri(7, seed=2),
    "tet": lambda: configs.small_tet(2, seed=2),
}


@pytest.mark.parametrize("kind,k,patch", [("tri", 1, 0), ("tri", 2, 0), ("tri", 2, 20), ("tri", 3, 16),
                                          ("tri", 4, 0), ("tri", 5, 12), ("tet", 1, 0), ("tet", 2, 9),
                                          ("tet", 3, 0)])
def test_mesh_matches_oracle(kind, k, patch):
    coords, cells = MESHES[kind]()
    m = Mesh(coords, cells, k, patch_cells=patch)
    m.validate()
    d = Discretization(coords, cells, k)
    assert m.n_dofs == d.n_dofs
    x = m.dof_coords()
    p = match(x, d.dof_coords)
    # lumped mass per DOF
    assert np.allclose(m.lumped_mass(), d.lumped_mass()[p], rtol=1e-13, atol=0)
    # boundary mass per DOF (different quadratures of the same facet integrals; the
    # library keeps only DOFs whose value is above rounding, so compare with a floor)
    b_or, b = d.boundary_mass()[p], m.boundary_mass()
    assert np.allclose(b, b_or, rtol=0, atol=(1e-11 if k == 5 else 1e-13) * np.abs(b_or).max())
    assert np.count_nonzero(b) >= np.count_nonzero(np.abs(b_or) > 1e-9 * np.abs(b_or).max())
    # cell -> DOF map agrees through the coordinate matching
    cd = m.cell_dofs()
    e = kmv_element(2 if kind == "tri" else 3, k)
    nodes, _, _ = K.kmv_element_tables(e.dim, k)
    q = match(nodes, e.nodes, 1e-14)
    assert np.array_equal(p[cd], d.cell_dofs[:, q])
    # Gershgorin bound equals the oracle's assembled-matrix value
    rng = np.random.default_rng(0)
    c = 1.0 + rng.random(d.n_dofs)
    Kc = d.stiffness(c)
    dt_or = solver.cfl_dt_gershgorin(Kc, d.lumped_mass())
    assert abs(m.cfl_dt(c[p]) - dt_or) < 1e-12 * dt_or


def test_large_graded_mesh_invariants():
    """The full-size graded layered mesh (about 150k triangles) preprocesses
    with valid patch maps and gather words at degree 4."""
    w = configs.layered_kmv4()
    m = Mesh(w.coords, w.cells, 4)
    m.validate()
    assert m.n_cells == len(w.cells)
    assert 140_000 < m.n_cells < 160_000
    M = m.lumped_mass()
    area = 9.5 * 3.75
    assert abs(M.sum() - area) < 1e-10 * area


def test_server_request_checks_wavelet_size():
    """The binding refuses a per-shot wavelet array that does not hold n_shots * n_steps
    values, before it builds the request (no server or GPU is needed to reach it)."""
    xs = np.zeros((2, 1, 2))
    with pytest.raises(ValueError, match="wavelets"):
        K.kmv_server_submit(None, None, K.KMV_FP32, 1e-3, 10, np.ones(4), xs, np.zeros((1, 2)), 5.0, 0.2,
                            forward_only=True, wavelets=np.zeros(10))


def test_server_request_checks_model_sizes():
    """The binding refuses a wave speed or damping array whose length is not the mesh's
    DOF count before the library copies n_dofs values from it (host only)."""
    coords, cells = configs.small_tri(3, seed=1)
    m = Mesh(coords, cells, 2)
    xs, xr = np.array([[0.5, 0.5]]), np.array([[0.2, 0.2]])
    with pytest.raises(ValueError, match="c must hold"):
        K.kmv_server_submit(None, m.handle, K.KMV_FP32, 1e-3, 10, np.ones(m.n_dofs - 1), xs, xr, 5.0, 0.2,
                            forward_only=True)
    with pytest.raises(ValueError, match="eta must hold"):
        K.kmv_server_submit(None, m.handle, K.KMV_FP32, 1e-3, 10, np.ones(m.n_dofs), xs, xr, 5.0, 0.2,
                            eta=np.zeros(m.n_dofs + 3), forward_only=True)
