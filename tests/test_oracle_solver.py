"""Pins for the oracle's time stepping, adjoint and gradient (eqs. Leapfrog,
forward3, acoustic_pml_FEM_adj, l2error, gradient3, discrete_fd/control_deriv)."""
import numpy as np
import pytest

from oracle.fem import Discretization
from oracle import solver
from oracle.green import green2d_trace
from synth import configs
from synth.meshes import structured_tri
from synth.models import sponge_eta


@pytest.fixture(scope="module")
def small():
    coords, cells = configs.small_tri(8, seed=9)
    d = Discretization(coords, cells, 3)
    rng = np.random.default_rng(7)
    c = 1.0 + 0.5 * rng.random(d.n_dofs)
    K = d.stiffness(c)
    M = d.lumped_mass()
    dt = 0.8 * 2.0 / np.sqrt(solver.power_rho(K, M, 800))
    eta = sponge_eta(d.dof_coords[:, 0], d.dof_coords[:, 1], 0.2, 0.8, 0.8, 0.2, c_max=1.5)
    return d, c, K, M, dt, eta


def energy(K, M, u_next, u, dt):
    du = (u_next - u) / dt
    return 0.5 * du @ (M * du) + 0.5 * u_next @ (K @ u)


def test_energy_conserved_without_damping(small):
    d, c, K, M, dt, _ = small
    rng = np.random.default_rng(1)
    u0 = rng.standard_normal(d.n_dofs)
    um1 = u0 + 0.01 * rng.standard_normal(d.n_dofs)
    _, states = solver.forward(K, M, None, dt, 400, lambda n: None, u0=u0, um1=um1,
                               keep_states=True)
    E = [energy(K, M, states[n + 1], states[n], dt) for n in range(len(states) - 1)]
    E0 = energy(K, M, u0, um1, dt)
    assert max(abs(e - E0) for e in E) < 1e-12 * abs(E0)


def test_damping_dissipates(small):
    d, c, K, M, dt, eta = small
    rng = np.random.default_rng(1)
    u0 = rng.standard_normal(d.n_dofs)
    _, states = solver.forward(K, M, eta * dt / 2, dt, 300, lambda n: None, u0=u0, um1=u0,
                               keep_states=True)
    E = [energy(K, M, states[n + 1], states[n], dt) for n in range(len(states) - 1)]
    assert E[-1] < E[0] and np.all(np.diff(E) <= 1e-12 * E[0])


def test_reciprocity_with_sponge(small):
    d, c, K, M, dt, eta = small
    A, B = np.array([[0.31, 0.42]]), np.array([[0.66, 0.27]])
    w = solver.ricker(np.arange(300) * dt, 8.0, 0.12)
    a = eta * dt / 2
    sA = np.asarray(d.interpolation_matrix(A).sum(0)).ravel()
    sB = np.asarray(d.interpolation_matrix(B).sum(0)).ravel()
    tAB, _ = solver.forward(K, M, a, dt, 300, solver.point_source_load(sA, w), P=d.interpolation_matrix(B))
    tBA, _ = solver.forward(K, M, a, dt, 300, solver.point_source_load(sB, w), P=d.interpolation_matrix(A))
    assert np.abs(tAB - tBA).max() < 1e-13 * np.abs(tAB).max()


def test_linearity_in_amplitude(small):
    d, c, K, M, dt, eta = small
    rec = np.random.default_rng(3).random((5, 2))
    sh = solver.Shot(d, [[0.5, 0.5]], rec, dt, 200, f0=8.0, t0=0.1)
    t1, _ = sh.forward(c, eta)
    sh2 = solver.Shot(d, [[0.5, 0.5]], rec, dt, 200, wavelet=2.5 * sh.wavelet)
    t2, _ = sh2.forward(c, eta)
    assert np.abs(t2 - 2.5 * t1).max() < 1e-13 * np.abs(t2).max()


def test_dot_product(small):
    """<y, P u(x)> = dt^2 sum_n lam^{n+1}(y) . x^n for arbitrary forcing x, data y."""
    d, c, K, M, dt, eta = small
    rng = np.random.default_rng(11)
    nt = 120
    X = rng.standard_normal((nt, d.n_dofs))
    P = d.interpolation_matrix(rng.random((7, 2)) * 0.9 + 0.05)
    Y = rng.standard_normal((nt, 7))
    a = eta * dt / 2
    tr, _ = solver.forward(K, M, a, dt, nt, lambda n: X[n], P=P)
    lam = solver.adjoint(K, M, a, dt, P, Y)
    lhs = np.sum(Y * tr)
    rhs = dt * dt * sum(lam[n] @ X[n] for n in range(nt))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_gradient_central_fd(small):
    d, c, K, M, dt, eta = small
    rng = np.random.default_rng(12)
    rec = rng.random((6, 2)) * 0.8 + 0.1
    sh = solver.Shot(d, [[0.45, 0.55]], rec, dt, 250, f0=8.0, t0=0.1)
    c_true = c * (1 + 0.05 * np.sin(3 * d.dof_coords[:, 0]))
    dobs, _ = sh.forward(c_true, eta)
    J, g, _ = sh.misfit_gradient(c, dobs, eta)
    direction = rng.standard_normal(d.n_dofs)
    errs = []
    for h in (1e-3, 1e-4, 1e-5):
        Jp = solver.misfit(sh.forward(c + h * direction, eta)[0], dobs)
        Jm = solver.misfit(sh.forward(c - h * direction, eta)[0], dobs)
        fd = (Jp - Jm) / (2 * h)
        errs.append(abs(fd - direction @ g) / abs(fd))
    # second-order convergence of the central difference towards c~ . g
    assert 50 < errs[0] / errs[1] < 200
    assert errs[2] < 1e-8
    # J vanishes at the model that produced the data
    J0, g0, _ = sh.misfit_gradient(c_true, dobs, eta)
    assert J0 == 0.0 and np.all(g0 == 0.0)


def _grad_case(small):
    d, c, K, M, dt, eta = small
    rng = np.random.default_rng(12)
    rec = rng.random((6, 2)) * 0.8 + 0.1
    sh = solver.Shot(d, [[0.45, 0.55]], rec, dt, 250, f0=8.0, t0=0.1)
    c_true = c * (1 + 0.05 * np.sin(3 * d.dof_coords[:, 0]))
    dobs, _ = sh.forward(c_true, eta)
    return sh, c, dobs, eta


def test_gradient_subsampling_partitions_the_full_gradient(small):
    """Gradient subsampling (section on gradient subsampling): the r offsets of the
    pairing steps partition the reverse steps, so the mean of the r subsampled
    gradients (each scaled by r) is the full gradient, which the central-difference
    test pins.  A wrong step selection, a dropped step or a wrong scale breaks it."""
    sh, c, dobs, eta = _grad_case(small)
    J1, g1, d1 = sh.misfit_gradient(c, dobs, eta)
    for r in (2, 3, 5):
        gs = []
        for o in range(r):
            J, g, d = sh.misfit_gradient(c, dobs, eta, r=r, offset=o)
            assert J == J1 and np.array_equal(d, d1)  # the forward and misfit are untouched
            gs.append(g)
        assert np.linalg.norm(np.mean(gs, axis=0) - g1) <= 1e-13 * np.linalg.norm(g1)
        assert np.linalg.norm(gs[0] - g1) > 1e-8 * np.linalg.norm(g1)  # a genuine subsample


def test_gradient_subsampling_follows_the_sampling_theorem(small):
    """The pairing is a product of two wavefields band-limited by the 8 Hz Ricker
    (about 20 Hz), so about 40 Hz: sampled every r dt it converges to the full sum
    once r dt is below the 12.5 ms Nyquist interval (dt = 7.1 ms here), and not far
    above it."""
    sh, c, dobs, eta = _grad_case(small)
    _, g1, _ = sh.misfit_gradient(c, dobs, eta)
    err = {r: np.linalg.norm(sh.misfit_gradient(c, dobs, eta, r=r)[1] - g1) / np.linalg.norm(g1)
           for r in (2, 3, 5)}
    assert err[2] < 1e-4 < err[3] < 1e-2 < err[5]


def test_gradient_fd_c1():
    """C1 (homogeneous KMV2, 1000 steps): central FD at h = 1e-3 along a seeded
    direction agrees with c~ . g to O(h^2)."""
    w = configs.homog_kmv2_c1()
    d = Discretization(w.coords, w.cells, 2)
    c = d.nodal_values(w.vp)
    sh = solver.Shot(d, w.sources, w.receivers, w.dt, 1000)
    dobs, _ = sh.forward(d.nodal_values(w.vp_obs))
    J, g, _ = sh.misfit_gradient(c, dobs)
    ct = np.random.default_rng(5).standard_normal(d.n_dofs)
    h = 1e-3
    fd = (solver.misfit(sh.forward(c + h * ct)[0], dobs)
          - solver.misfit(sh.forward(c - h * ct)[0], dobs)) / (2 * h)
    assert abs(fd - ct @ g) < 1e-6 * abs(fd)


def test_green_function_accuracy():
    """Homogeneous 2D: KMV traces approach the closed-form solution (receiver
    error E of eq. receiver_error_calc) and the error falls under refinement."""
    c0, f0, t0 = 1.5, 5.0, 0.15
    L = 2.0
    errs = []
    for k, n in [(2, 40), (3, 40), (3, 60)]:
        coords, cells = structured_tri(n, n, 0.0, L, 0.0, L)
        d = Discretization(coords, cells, k)
        c = np.full(d.n_dofs, c0)
        K = d.stiffness(c)
        M = d.lumped_mass()
        dt = 0.5 * 2.0 / np.sqrt(solver.gershgorin_rho(K, M))
        T = 0.72  # first reflection (from 1 km away) reaches the receivers after ~0.73 s + t0
        nt = int(T / dt)
        src = np.array([[1.0, 1.0]])
        rec = np.array([[1.4, 1.0], [1.0, 1.45], [1.3, 1.3]])
        sh = solver.Shot(d, src, rec, dt, nt, f0=f0, t0=t0)
        tr, _ = sh.forward(c)
        t = np.arange(1, nt + 1) * dt
        ref = np.stack([green2d_trace(np.linalg.norm(r - src[0]), t, c0,
                                      lambda s: solver.ricker(s, f0, t0)) for r in rec], 1)
        E = np.sqrt(np.trapezoid(np.sum((tr - ref) ** 2, 1), t) / np.trapezoid(np.sum(ref ** 2, 1), t))
        errs.append(E)
    assert errs[0] < 0.05 and errs[1] < errs[0] and errs[2] < errs[1]


def test_mms_convergence():
    """u = t^2 cos(pi x) cos(pi z) on the unit square (homogeneous Neumann), c = 1,
    lumped load M_i f(x_i, t_n).  Leapfrog is exact in time for t^2, so only the
    spatial error remains; it falls at least like h^k."""
    T, dt = 0.2, 1e-3
    for k in [2, 3]:
        errs = []
        for n in [4, 8]:
            coords, cells = structured_tri(n, n, 0.0, 1.0, 0.0, 1.0)
            d = Discretization(coords, cells, k)
            K = d.stiffness(np.ones(d.n_dofs))
            M = d.lumped_mass()
            x, z = d.dof_coords[:, 0], d.dof_coords[:, 1]
            phi = np.cos(np.pi * x) * np.cos(np.pi * z)
            nt = int(round(T / dt))
            load = lambda m: M * (2.0 + 2.0 * np.pi ** 2 * (m * dt) ** 2) * phi
            _, st = solver.forward(K, M, None, dt, nt, load, u0=np.zeros(d.n_dofs),
                                   um1=dt * dt * phi, keep_states=True)
            exact = T ** 2 * phi
            errs.append(np.sqrt(np.sum(M * (st[-1] - exact) ** 2) / np.sum(M * exact ** 2)))
        assert errs[1] < errs[0] / 2 ** k


@pytest.mark.parametrize("f0,t0,amp", [(5.0, 0.2, 1.0), (8.0, 0.1, 2.5), (12.5, 0.3, -0.7)])
def test_ricker_wavelet_pins(f0, t0, amp):
    """The oracle's wavelet against what fixes the Ricker wavelet independently of its
    formula: the peak frequency f0 of its amplitude spectrum (section on the forward
    wave simulation: the source is a Ricker wavelet of a given peak frequency), its
    value amp at the delay t0, its zero crossings at t0 +- 1/(sqrt(2) pi f0), its
    symmetry about t0, its zero mean, and its spectrum against the closed-form Fourier
    transform of the second derivative of a Gaussian."""
    dt = 1e-4
    n = int(round(4.0 / dt))
    t = t0 + (np.arange(n) - n // 2) * dt              # 4 s centred on t0: the whole wavelet
    w = solver.ricker(t, f0, t0, amp)
    # value at the delay and zero crossings
    assert solver.ricker(np.array([t0]), f0, t0, amp)[0] == pytest.approx(amp, rel=1e-15)
    tz = 1.0 / (np.sqrt(2.0) * np.pi * f0)
    z = solver.ricker(np.array([t0 - tz, t0 + tz]), f0, t0, amp)
    assert np.abs(z).max() < 1e-14 * abs(amp)
    # sign change across each zero (so they are crossings, not touch points)
    for s in (-1.0, 1.0):
        a, b = solver.ricker(np.array([t0 + s * tz * 0.99, t0 + s * tz * 1.01]), f0, t0, amp)
        assert a * b < 0
    # symmetry about t0
    tau = np.linspace(0.0, 0.5, 101)
    assert np.abs(solver.ricker(t0 + tau, f0, t0, amp) - solver.ricker(t0 - tau, f0, t0, amp)).max() \
        < 1e-15 * abs(amp)
    # zero mean (the wavelet is a second derivative of a Gaussian)
    assert abs(np.sum(w) * dt) < 1e-10 * abs(amp)
    # amplitude spectrum: peak at f0 within the frequency resolution of a padded FFT
    nfft = 1 << 20
    W = np.abs(np.fft.rfft(w, nfft)) * dt
    f = np.fft.rfftfreq(nfft, dt)
    df = f[1]
    assert abs(f[np.argmax(W)] - f0) <= df
    # closed form |W(f)| = |amp| 2 f^2 / (sqrt(pi) f0^3) exp(-f^2/f0^2) (the Fourier
    # transform of -(1/(2 pi^2 f0^2)) d^2/dt^2 exp(-pi^2 f0^2 t^2), times amp)
    ref = abs(amp) * 2.0 * f ** 2 / (np.sqrt(np.pi) * f0 ** 3) * np.exp(-(f / f0) ** 2)
    band = f < 4 * f0
    assert np.abs(W[band] - ref[band]).max() < 1e-6 * ref.max()
