"""Pins for the oracle's PML (section "Forward wave simulation in a PML truncated
medium", eqs. acoustic_pml and forward2d_I/II; the appendix matrices; the
transposed scheme of eq. acoustic_pml_FEM_adj; eq. gradient).

What pins it, independently of its own formulas:
* with sigma = 0 it is the plain scheme (bitwise the solver without a PML);
* the derivative matrices: D_k 1 = 0 (the derivative of a constant), D_k x_j =
  delta_kj M (the nodal rule integrates phi_i times a constant exactly), and
  D_k + D_k^T = the boundary integral of phi_i phi_j n_k, whose row sums are the
  boundary integral of phi_i n_k (Gauss-Green);
* the discrete adjoint: <y, P U(x)> = dt^2 sum_n lam^{n+1}(y) . x^n for arbitrary
  forcing x and data y (2D and 3D), which fails for any transposition or sign slip
  in the couplings;
* the gradient: central differences of J, O(h^2), along directions inside and
  across the layer (2D and 3D);
* absorption: a plane pulse at normal incidence into a layer of width L with
  sigma_max = 3 c ln(1/R)/(2L) comes back with the continuous PML's amplitude R
  (R = 1e-3 here) up to discretisation error, a factor ~30 below the same profile
  used as a sponge, whose round trip keeps R^{1/2}, and ~1000 below Neumann;
* long runs stay bounded (2D and 3D), while the same recursion with the auxiliary
  damping at level n (the reading not taken) grows without bound.
"""
import numpy as np
import pytest

from oracle.fem import Discretization
from oracle import pml as PML
from oracle import solver
from synth import configs
from synth.meshes import structured_tri
from synth.models import pml_sigma, pml_sigma_3d


def small2d(n=8, k=2, seed=5):
    coords, cells = configs.small_tri(n, seed=seed)
    d = Discretization(coords, cells, k)
    x, z = d.dof_coords.T
    sig = pml_sigma(x, z, 0.2, 0.8, 0.75, 0.2, c_max=2.0)
    c = 1.5 + 0.3 * z + 0.1 * np.sin(4 * x)
    return d, sig, c


def small3d(n=3, k=2, seed=5):
    coords, cells = configs.small_tet(n, seed=seed)
    d = Discretization(coords, cells, k)
    x, y, z = d.dof_coords.T
    sig = pml_sigma_3d(x, y, z, (0.25, 0.25), (0.75, 0.75, 0.7), 0.25, c_max=2.0)
    c = 1.5 + 0.3 * z
    return d, sig, c


@pytest.mark.parametrize("dim", [2, 3])
def test_derivative_matrices(dim):
    d, sig, c = small2d(6, 3) if dim == 2 else small3d(2, 2)
    D = d.derivative_matrices()
    M = d.lumped_mass()
    one = np.ones(d.n_dofs)
    b = d.boundary_mass()
    for k in range(dim):
        assert np.abs(D[k] @ one).max() < 1e-13
        for j in range(dim):
            v = D[k] @ d.dof_coords[:, j]
            ref = M if j == k else np.zeros_like(M)
            assert np.abs(v - ref).max() < 1e-13 * M.max()
    # Gauss-Green on the unit square/cube: the row sums of D_k + D_k^T are the
    # boundary integral of phi_i n_k, i.e. +b_i on the face x_k = 1, -b_i on x_k = 0
    x = d.dof_coords
    for k in range(dim):
        rs = np.asarray((D[k] + D[k].T).sum(axis=1)).ravel()
        ref = np.where(np.abs(x[:, k] - 1.0) < 1e-12, b, 0.0) - np.where(np.abs(x[:, k]) < 1e-12, b, 0.0)
        corner = np.sum(np.abs(x - 0.5) > 0.5 - 1e-12, axis=1) > 1   # on two faces: b splits
        assert np.abs(rs - ref)[~corner].max() < 1e-12


def test_zero_sigma_is_the_plain_scheme():
    d, sig, c = small2d()
    K, M = d.stiffness(c), d.lumped_mass()
    dt = 0.8 * solver.cfl_dt_gershgorin(K, M)
    sh = solver.Shot(d, [[0.5, 0.4]], [[0.3, 0.3], [0.7, 0.6]], dt, 150, f0=6.0, t0=0.15)
    t0, _ = sh.forward(c)
    t1, _ = sh.forward(c, pml=np.zeros_like(sig))
    assert np.array_equal(t0, t1)


@pytest.mark.parametrize("dim", [2, 3])
def test_pml_dot_product(dim):
    d, sig, c = small2d() if dim == 2 else small3d()
    K, M = d.stiffness(c), d.lumped_mass()
    dt = 0.8 * solver.cfl_dt_gershgorin(K, M)
    pm = PML.PML(d, sig)
    a = dt * pm.tr1 / 2
    rng = np.random.default_rng(2)
    nt = 80
    rec = np.random.default_rng(3).random((4, dim))
    P = d.interpolation_matrix(rec)
    xs = rng.standard_normal((nt, d.n_dofs))
    y = rng.standard_normal((nt, P.shape[0]))
    tr, _, _ = PML.forward(pm, K, M, a, c, dt, nt, lambda n: xs[n], P=P)
    lam = PML.adjoint(pm, K, M, a, c, dt, P, y)
    lhs = float(np.sum(y * tr))
    rhs = dt * dt * sum(lam[n] @ xs[n] for n in range(nt))   # lam[n] = lam^{n+1}
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("dim", [2, 3])
def test_pml_gradient_central_differences(dim):
    d, sig, c = small2d() if dim == 2 else small3d()
    K, M = d.stiffness(c), d.lumped_mass()
    dt = 0.7 * solver.cfl_dt_gershgorin(K, M)
    nt = 120 if dim == 2 else 80
    x = d.dof_coords
    src = [[0.5, 0.3]] if dim == 2 else [[0.5, 0.5, 0.3]]
    rec = np.random.default_rng(4).random((5, dim)) * 0.6 + 0.2
    sh = solver.Shot(d, src, rec, dt, nt, f0=6.0, t0=0.15)
    c_true = c * (1.0 + 0.05 * np.exp(-np.sum((x - 0.45) ** 2, axis=1) / 0.02))
    dobs, _ = sh.forward(c_true, pml=sig)
    J, g, _ = sh.misfit_gradient(c, dobs, pml=sig)
    rng = np.random.default_rng(9)
    # a smooth direction over the whole mesh (physical domain and layer), and one
    # supported in the layer only
    dirs = [np.exp(-np.sum((x - rng.random(dim)) ** 2, axis=1) / 0.05),
            (np.abs(sig).sum(axis=1) > 0) * (1.0 + x[:, 0])]
    for ct in dirs:
        ct = ct / np.abs(ct).max()
        an = ct @ g
        fd = {}
        for h in (1e-3, 5e-4):
            Jp, _ = sh.forward(c + h * ct, pml=sig)
            Jm, _ = sh.forward(c - h * ct, pml=sig)
            fd[h] = (solver.misfit(Jp, dobs) - solver.misfit(Jm, dobs)) / (2 * h)
        e1, e2 = abs(fd[1e-3] - an), abs(fd[5e-4] - an)
        assert e2 < 1e-4 * abs(an), (fd, an)
        assert e2 < 0.3 * e1 + 1e-13 * abs(an)      # O(h^2)
        rich = (4.0 * fd[5e-4] - fd[1e-3]) / 3.0     # Richardson: the h^2 term removed
        assert abs(rich - an) < 1e-8 * abs(an), (rich, an)


def strip(nx, L, width, k=2):
    """[0, nx*h] x [0, 2h] strip of right triangles, h = 1/40 km: plane waves in x."""
    h = 0.025
    coords, cells = structured_tri(nx, 2, 0.0, nx * h, 0.0, 2 * h)
    return Discretization(coords, cells, k), h


def reflected_amplitude(kind):
    """Peak of the wave that comes back from the right-hand layer (L = 0.5 km),
    relative to the incident peak, for a Ricker plane pulse at normal incidence."""
    nx, width = 120, 0.5
    d, h = strip(nx, 3.0, width)
    x = d.dof_coords[:, 0]
    c = np.full(d.n_dofs, 1.5)
    x_pml = nx * h - width
    R = 1e-3
    smax = 3.0 * 1.5 * np.log(1.0 / R) / (2.0 * width)
    sx = smax * (np.maximum(x - x_pml, 0.0) / width) ** 2
    K, M = d.stiffness(c), d.lumped_mass()
    dt = 0.5 * solver.cfl_dt_gershgorin(K, M)
    nt = int(3.4 / dt)
    # line source at x = 0.6 km: the sum of the point sources across the strip
    zs = np.unique(d.dof_coords[:, 1])
    src = np.stack([np.full(len(zs), 0.6), zs], axis=1)
    rec = np.array([[1.0, 0.025]])
    sh = solver.Shot(d, src, rec, dt, nt, f0=4.0, t0=0.3)
    if kind == "pml":
        tr, _ = sh.forward(c, pml=np.stack([sx, np.zeros_like(sx)], axis=1))
    elif kind == "sponge":
        tr, _ = sh.forward(c, eta=sx)
    else:
        tr, _ = sh.forward(c)
    t = (np.arange(nt) + 1) * dt
    inc = np.abs(tr[t < 1.1, 0]).max()            # the direct wave passes x = 1 km by then
    ref = np.abs(tr[t > 2.0, 0]).max()            # echo from the layer (x = 3 km) after 2.3 s
    # the left end (x = 0) reflects too; its echo reaches x = 1 km at 1.07 s + the
    # direct arrival: it is inside the incident window and gone by 2 s
    return ref / inc


def test_pml_absorbs_a_plane_pulse_to_its_design_reflection():
    r_pml = reflected_amplitude("pml")
    r_sponge = reflected_amplitude("sponge")
    r_neu = reflected_amplitude("neumann")
    assert r_neu > 0.5
    # the continuous PML returns exp(-2/c int sigma dx) = R = 1e-3 at normal incidence
    # for every frequency; measured 1.010e-3 (sponge 0.100, Neumann 1.001)
    assert abs(r_pml / 1e-3 - 1.0) < 0.05
    assert r_sponge > 1e-2       # the same profile as a sponge: round trip ~ R^(1/2)
    assert r_pml < r_sponge / 10


@pytest.mark.parametrize("dim", [2, 3])
def test_long_run_stays_bounded(dim):
    """4000 steps from a random start with the layer on: the wavefield decays, no
    mode grows (the damping is scaled to sigma_max dt = 0.1, five times the
    workloads' 0.02)."""
    d, sig, c = small2d(6, 2) if dim == 2 else small3d(2, 2)
    K, M = d.stiffness(c), d.lumped_mass()
    dt = 0.8 * solver.cfl_dt_gershgorin(K, M)
    sig = sig * (0.1 / (sig.max() * dt))
    pm = PML.PML(d, sig)
    a = dt * pm.tr1 / 2
    rng = np.random.default_rng(1)
    f0 = rng.standard_normal(d.n_dofs)
    nt = 4000
    _, st, _ = PML.forward(pm, K, M, a, c, dt, nt, lambda n: f0 if n < 5 else None, keep_states=True)
    peak = max(np.abs(s).max() for s in st[:200])
    assert all(np.isfinite(s).all() for s in st)
    assert np.abs(st[-1]).max() < peak


@pytest.mark.parametrize("sdt", [0.01, 0.1, 1.0, 5.0])
def test_auxiliary_damping_centring(sdt):
    """The reading for the damping term of the first-order auxiliary rows: centred,
    (1 + s dt) p^{n+1} = (1 - s dt) p^{n-1}, both roots of the undriven recursion
    lie inside the unit circle for every s dt > 0; at level n, as the printed A_n
    places it, p^{n+1} = p^{n-1} - 2 s dt p^n has a root of modulus
    s dt + sqrt(1 + (s dt)^2) > 1, so a decaying field grows."""
    centred = np.roots([1.0 + sdt, 0.0, -(1.0 - sdt)])
    level_n = np.roots([1.0, 2.0 * sdt, -1.0])
    assert np.abs(centred).max() < 1.0
    assert np.abs(level_n).max() == pytest.approx(sdt + np.sqrt(1.0 + sdt * sdt), rel=1e-12)
    assert np.abs(level_n).max() > 1.0


def test_pml_subsampling_partitions_the_full_gradient():
    """Gradient subsampling with the PML: the mean over the r offsets of the r-scaled
    subsampled gradients is the full gradient (the pairing sum partitioned by m mod r)."""
    d, sig, c = small2d()
    K, M = d.stiffness(c), d.lumped_mass()
    dt = 0.7 * solver.cfl_dt_gershgorin(K, M)
    x = d.dof_coords
    sh = solver.Shot(d, [[0.5, 0.3]], [[0.3, 0.6], [0.7, 0.5]], dt, 90, f0=6.0, t0=0.15)
    dobs, _ = sh.forward(c * (1.0 + 0.05 * np.exp(-np.sum((x - 0.45) ** 2, axis=1) / 0.02)), pml=sig)
    _, g, _ = sh.misfit_gradient(c, dobs, pml=sig)
    gs = [sh.misfit_gradient(c, dobs, pml=sig, r=3, offset=o)[1] for o in range(3)]
    assert np.abs(sum(gs) / 3.0 - g).max() < 1e-12 * np.abs(g).max()
