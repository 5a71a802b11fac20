"""Pins for the oracle's mesh-level operators: lumped mass, assembled stiffness,
point interpolation (appendix matrices M_u and K; sections on the spatial
discretization, time discretization (eq. spectral) and receivers/sources)."""
import numpy as np
import pytest
import scipy.linalg

from oracle.fem import Discretization
from oracle import solver
from synth import configs

TRI = [1, 2, 3, 4, 5]
TET = [1, 2, 3]


@pytest.fixture(scope="module")
def tri_discs():
    coords, cells = configs.small_tri(6, seed=5)
    return {k: Discretization(coords, cells, k) for k in TRI}


@pytest.fixture(scope="module")
def tet_discs():
    coords, cells = configs.small_tet(2, seed=5)
    return {k: Discretization(coords, cells, k) for k in TET}


def interior_dofs(disc):
    x = disc.dof_coords
    tol = 1e-9
    return np.all((x > tol) & (x < 1 - tol), axis=1)


def both(tri_discs, tet_discs):
    return list(tri_discs.items()) + [(("tet", k), d) for k, d in tet_discs.items()]


def test_dof_counts():
    """Structured 40x40 right-triangle mesh: KMV2 has 1 DOF per vertex, per edge
    and per cell: 1681 + 4880 + 3200 = 9761."""
    w = configs.homog_kmv2_c1()
    d = Discretization(w.coords, w.cells, 2)
    assert d.n_dofs == 1681 + 4880 + 3200


def test_mass_sums_to_measure(tri_discs, tet_discs):
    for _, d in both(tri_discs, tet_discs):
        assert abs(d.lumped_mass().sum() - 1.0) < 1e-13


@pytest.mark.parametrize("k", TRI)
def test_mass_integrates_polynomials(tri_discs, k):
    """sum_i M_i p(x_i) = int_Omega p for deg p <= 2k-1 (affine cells, rule exact
    to at least that degree); x^a z^b over the unit square is 1/((a+1)(b+1))."""
    d = tri_discs[k]
    M = d.lumped_mass()
    x, z = d.dof_coords[:, 0], d.dof_coords[:, 1]
    for a in range(2 * k):
        for b in range(2 * k - a):
            assert abs(M @ (x ** a * z ** b) - 1.0 / ((a + 1) * (b + 1))) < 1e-13


def test_stiffness_rowsum_symmetry(tri_discs, tet_discs):
    rng = np.random.default_rng(0)
    for _, d in both(tri_discs, tet_discs):
        c = 1.0 + rng.random(d.n_dofs)
        K = d.stiffness(c)
        scale = abs(K).max()
        assert abs(K @ np.ones(d.n_dofs)).max() < 1e-12 * scale
        assert abs(K - K.T).max() < 1e-13 * scale


@pytest.mark.parametrize("k", [1, 2, 3])
def test_stiffness_psd_one_zero_mode(tri_discs, k):
    d = tri_discs[k]
    c = np.full(d.n_dofs, 1.3)
    K = d.stiffness(c).toarray()
    ev = scipy.linalg.eigvalsh(K)
    assert abs(ev[0]) < 1e-10 * ev[-1]
    assert ev[1] > 1e-6 * ev[-1]


def test_patch_test_and_laplacian(tri_discs, tet_discs):
    """c = 1: (K p)_i = 0 for linear p, and (K |x|^2)_i = -2 dim M_i, at DOFs off
    the boundary (integration by parts, rule exact for grad phi_i . grad p)."""
    for key, d in both(tri_discs, tet_discs):
        K = d.stiffness(np.ones(d.n_dofs))
        M = d.lumped_mass()
        inner = interior_dofs(d)
        x = d.dof_coords
        lin = 0.3 + 1.7 * x[:, 0] - 0.4 * x[:, -1]
        assert abs((K @ lin)[inner]).max() < 1e-11
        quad = np.sum(x ** 2, axis=1)
        k = key if isinstance(key, int) else key[1]
        if k >= 2:
            assert np.allclose((K @ quad)[inner], -2 * d.dim * M[inner], atol=1e-11)


def test_stiffness_energy_closed_form(tri_discs):
    """u = x, c^2 = 1 + x: u.K u = int c^2 |grad x|^2 = int (1+x) = 3/2 on the unit
    square when the rule integrates c^2 exactly (k >= 1, c^2 linear)."""
    for k, d in tri_discs.items():
        x = d.dof_coords[:, 0]
        c = np.sqrt(1.0 + x)
        K = d.stiffness(c)
        assert abs(x @ (K @ x) - 1.5) < 1e-12


def test_gershgorin_bounds_power(tri_discs):
    for k, d in tri_discs.items():
        c = np.full(d.n_dofs, 1.5)
        K = d.stiffness(c)
        M = d.lumped_mass()
        rho_p = solver.power_rho(K, M, iters=2000)
        rho_ev = scipy.linalg.eigh(K.toarray(), np.diag(M), eigvals_only=True)[-1]
        assert abs(rho_p - rho_ev) < 1e-6 * rho_ev
        assert solver.gershgorin_rho(K, M) >= rho_ev * (1 - 1e-12)


def test_interpolation_reproduces_polynomials(tri_discs, tet_discs):
    rng = np.random.default_rng(4)
    for key, d in both(tri_discs, tet_discs):
        k = key if isinstance(key, int) else key[1]
        pts = 0.05 + 0.9 * rng.random((20, d.dim))
        P = d.interpolation_matrix(pts)
        x = d.dof_coords
        f = lambda y: (0.2 + y[:, 0]) ** k + (0.5 * y[:, -1]) ** k - y[:, 0] * y[:, -1] ** (k - 1)
        assert np.allclose(P @ f(x), f(pts), atol=1e-11)


def test_locate_outside_raises(tri_discs):
    with pytest.raises(ValueError):
        tri_discs[2].locate([[1.5, 0.5]])
