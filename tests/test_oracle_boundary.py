"""Oracle pins for the absorbing boundary term (the first-order condition
du/dt + c du/dn = 0 on the outer boundary; its weak form puts the boundary integral
of c phi_i phi_j in the damping matrix M_{u,1} of the appendix).

* Boundary mass b_i = integral of phi_i over the boundary: on the unit square and
  the unit cube, sum_i b_i f(x_i) must equal the boundary integral of f exactly for
  every f the element reproduces on its facets (constants and linears always,
  quadratics from k = 2): a dropped facet, a wrong facet measure or a wrong trace
  of the basis fails one of them.
* Gradient: the derivative of J through the c-dependent boundary damping, checked
  by central differences of the oracle's own J (not by its formula); the same
  check without the boundary term must fail, so the term is what makes it pass.
* Energy: with no sponge and the source off, the discrete energy is conserved
  without the term and decays with it.
* Reflection: a plane pulse meeting the boundary head-on is reflected whole by the
  Neumann boundary and almost not at all with the term (the first-order condition
  is exact at normal incidence); a damping off by a factor alpha would reflect
  |1 - alpha| / (1 + alpha), 1/3 for alpha = 2 or 1/2."""
import numpy as np
import pytest

from oracle.fem import Discretization
from oracle import solver
from synth import configs


def _tri(k):
    coords, cells = configs.small_tri(5, seed=2)
    return Discretization(coords, cells, k)


def _tet(k):
    coords, cells = configs.small_tet(2, seed=2)
    return Discretization(coords, cells, k)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_boundary_mass_integrates_the_square_boundary(k):
    d = _tri(k)
    b = d.boundary_mass()
    x, z = d.dof_coords.T
    tol = 1e-12 if k < 5 else 1e-11   # KMV5's basis has condition ~1e6
    assert abs(b.sum() - 4.0) < tol * 4
    assert abs(b @ x - 2.0) < tol * 4          # x = 1 side: 1, top and bottom: 1/2 each
    assert abs(b @ (x * z) - 1.0) < tol * 4    # linear along every side
    if k >= 2:
        assert abs(b @ x ** 2 - 5.0 / 3.0) < tol * 4
    else:
        assert abs(b @ x ** 2 - 5.0 / 3.0) > 1e-3  # trapezoid rule on P1 traces
    on = (np.minimum(x, z) < 1e-12) | (np.maximum(x, z) > 1 - 1e-12)
    # off the boundary only the rounding of basis traces that vanish there
    assert np.all(np.abs(b[~on]) < tol * b.max()) and np.all(np.abs(b[on]) > 1e-6 * b.max())


@pytest.mark.parametrize("k", [1, 2, 3])
def test_boundary_mass_integrates_the_cube_boundary(k):
    d = _tet(k)
    b = d.boundary_mass()
    x, y, z = d.dof_coords.T
    assert abs(b.sum() - 6.0) < 1e-12 * 6
    assert abs(b @ x - 3.0) < 1e-12 * 6
    if k >= 2:
        assert abs(b @ x ** 2 - 7.0 / 3.0) < 1e-12 * 6
        assert abs(b @ (y * z) - 1.5) < 1e-12 * 6
    lo, hi = d.dof_coords.min(axis=1), d.dof_coords.max(axis=1)
    on = (lo < 1e-12) | (hi > 1 - 1e-12)
    assert np.all(np.abs(b[~on]) < 1e-13 * b.max())


def _fd_case(kind):
    if kind == "tri":
        coords, cells = configs.small_tri(6, seed=3)
        d = Discretization(coords, cells, 2)
        x, z = d.dof_coords.T
        c_true, c0 = 1.5 + 0.4 * z + 0.1 * np.sin(5 * x), 1.5 + 0.4 * z
        src, f0 = [[0.5, 0.3]], 8.0
        rec = np.stack([np.linspace(0.1, 0.9, 8), np.full(8, 0.2)], axis=1)
        delta = np.exp(-(x ** 2 + (z - 0.5) ** 2) / 0.05) + 0.5 * np.exp(-((x - 0.6) ** 2 + (z - 1) ** 2) / 0.05)
    else:
        coords, cells = configs.small_tet(2, seed=3)
        d = Discretization(coords, cells, 2)
        x, y, z = d.dof_coords.T
        c_true, c0 = 1.5 + 0.3 * z + 0.1 * np.sin(4 * x), 1.5 + 0.3 * z
        src, f0 = [[0.5, 0.5, 0.4]], 6.0
        rec = np.stack([np.linspace(0.2, 0.8, 5), np.full(5, 0.5), np.full(5, 0.2)], axis=1)
        delta = np.exp(-((x - 1) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2) / 0.1)
    dt = 0.8 * solver.cfl_dt_gershgorin(d.stiffness(c_true), d.lumped_mass())
    nt = int(np.ceil(1.0 / dt))  # 1 s: the wave reaches every side
    sh = solver.Shot(d, src, rec, dt, nt, f0=f0, t0=0.1)
    return d, sh, c_true, c0, delta, dt, nt


@pytest.mark.parametrize("kind", ["tri", "tet"])
def test_boundary_term_gradient_matches_central_differences(kind):
    d, sh, c_true, c0, delta, dt, nt = _fd_case(kind)
    dobs, _ = sh.forward(c_true, absorb=True)
    J, g, _ = sh.misfit_gradient(c0, dobs, absorb=True)
    h = 1e-4
    Jp = solver.misfit(sh.forward(c0 + h * delta, absorb=True)[0], dobs)
    Jm = solver.misfit(sh.forward(c0 - h * delta, absorb=True)[0], dobs)
    fd = (Jp - Jm) / (2 * h)
    assert abs(g @ delta - fd) < 1e-7 * abs(fd)
    # the same gradient without the boundary term misses by far more
    K, M = d.stiffness(c0), d.lumped_mass()
    a = sh.damping(c0, M, None, True)
    _, states = solver.forward(K, M, a, dt, nt, solver.point_source_load(sh.s_vec, sh.wavelet), keep_states=True)
    _, g_no, _ = solver.gradient(d, c0, K, M, a, dt, sh.P, dobs, states)
    assert abs(g_no @ delta - fd) > 1e-3 * abs(fd)


@pytest.mark.parametrize("kind", ["tri", "tet"])
def test_boundary_term_dissipates_energy(kind):
    d, sh, c_true, c0, delta, dt, nt = _fd_case(kind)
    K, M = d.stiffness(c0), d.lumped_mass()
    n_off = int(np.ceil(0.45 / dt))  # the Ricker pulse (f0 >= 6 Hz, t0 = 0.1 s) is below 1e-17
    E = {}
    for absorb in (False, True):
        a = sh.damping(c0, M, None, absorb)
        _, st = solver.forward(K, M, a, dt, nt, solver.point_source_load(sh.s_vec, sh.wavelet), keep_states=True)
        # E^{n+1/2} = |u^{n+1} - u^n|_M^2 / (2 dt^2) + u^{n+1}.K u^n / 2
        E[absorb] = np.array([0.5 * (((st[n + 1] - st[n]) ** 2) * M).sum() / dt ** 2
                              + 0.5 * st[n + 1] @ (K @ st[n]) for n in range(n_off, nt)])
    assert np.ptp(E[False]) < 1e-9 * E[False][0]
    assert np.all(np.diff(E[True]) <= 1e-12 * E[True][0])
    assert E[True][-1] < 0.5 * E[True][0]


def test_boundary_term_absorbs_a_normally_incident_plane_wave():
    coords, cells = configs.structured_tri(40, 40, 0.0, 2.0, 0.0, 2.0)
    d = Discretization(coords, cells, 2)
    x, z = d.dof_coords.T
    c = np.full(d.n_dofs, 1.5)
    K, M = d.stiffness(c), d.lumped_mass()
    dt = 0.8 * solver.cfl_dt_gershgorin(K, M)
    pulse = lambda xx: np.exp(-((xx - 1.2) / 0.08) ** 2)
    u0, um1 = pulse(x), pulse(x + 1.5 * dt)  # u(x, t) = pulse(x - c t), moving to x = 2
    nt = int(np.ceil(1.0 / dt))              # out to x = 2 and back to x ~ 1.3
    band = (np.abs(z - 1.0) < 0.3) & (x < 1.6)  # away from the grazing top and bottom sides

    def reflected(alpha):
        a = None if alpha == 0 else alpha * dt * c * d.boundary_mass() / (2.0 * M)
        _, st = solver.forward(K, M, a, dt, nt, lambda n: None, u0=u0, um1=um1, keep_states=True)
        return np.abs(st[-1][band]).max()

    assert reflected(0) > 0.95          # Neumann: the pulse comes back whole
    assert reflected(1.0) < 0.08        # the boundary term: almost nothing comes back
    assert reflected(2.0) > 0.2 and reflected(0.5) > 0.2  # a wrong scale reflects ~1/3
