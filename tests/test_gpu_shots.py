"""Shots stepped together (kmv_options.n_shots): one launch per step advances every
shot of a problem, each with its own sources and state.

A shot's arithmetic is the same as in a one-shot problem, so its traces must be
bitwise those of the one-shot problem with its sources; J and the gradient are
the fixed-order sums over the shots, equal to the sums of the one-shot results up
to float64 rounding of the sum (1e-12 relative).  The FP64 sum also matches the
oracle (1e-10, the parity bar).  Cases cover several patches per shot on a small
ragged patch size, so work items of one patch fall on different XCD runs, and both
reverse-sweep storage plans."""
import numpy as np
import pytest

from gpu_util import say, dof_map, rel_l2
from synth import configs
from synth.models import sponge_eta

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_10946_amd as kmv
    kmv.lib()


def cuda(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def case(kind):
    """Mesh, wave speeds, damping, dt, shot sources [S, 2, dim], receivers."""
    from paper_2108_10946_amd import Mesh
    rng = np.random.default_rng(17)
    if kind == "tri":
        coords, cells = configs.small_tri(10, seed=3)
        m = Mesh(coords, cells, 3, patch_cells=13)
        x = m.dof_coords()
        c_true = 1.5 + 0.5 * x[:, 1] + 0.1 * np.exp(-((x[:, 0] - 0.4) ** 2 + (x[:, 1] - 0.5) ** 2) / 0.02)
        c0 = 1.5 + 0.5 * x[:, 1]
        eta = sponge_eta(x[:, 0], x[:, 1], 0.0, 1.0, 0.8, 0.2, c_max=2.5)
        S = 5
        xs = np.stack([np.stack([[0.1 + 0.8 * rng.random(), 0.05 + 0.1 * rng.random()] for _ in range(2)])
                       for _ in range(S)])
        xr = np.stack([np.linspace(0.1, 0.9, 12), np.full(12, 0.15)], axis=1)
        nt, f0 = 300, 8.0
    else:
        coords, cells = configs.small_tet(3, seed=5)
        m = Mesh(coords, cells, 2, patch_cells=7)
        x = m.dof_coords()
        c_true = 1.5 + 0.4 * x[:, 2] + 0.1 * np.exp(-np.sum((x - 0.5) ** 2, axis=1) / 0.03)
        c0 = 1.5 + 0.4 * x[:, 2]
        eta = None
        S = 3
        xs = np.stack([np.stack([0.1 + 0.8 * rng.random(3) for _ in range(2)]) for _ in range(S)])
        xr = np.stack([np.linspace(0.15, 0.85, 8), np.full(8, 0.4), np.full(8, 0.2)], axis=1)
        nt, f0 = 120, 6.0
    dt = 0.5 * m.cfl_dt(c_true)
    return m, c_true, c0, eta, dt, nt, f0, xs, xr


def problem(m, dt, nt, prec, eta, f0, xs, xr, **kw):
    from paper_2108_10946_amd import Problem
    p = Problem(m, dt, nt, precision=prec, n_shots=len(xs) if xs.ndim == 3 else 1, **kw)
    if eta is not None:
        p.set_damping(eta)
    p.set_sources(xs, f0=f0, t0=0.1)
    p.set_receivers(xr)
    return p


@pytest.mark.parametrize("kind", ["tri", "tet"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ckpt", [0, 7])
def test_shots_equal_one_shot_problems(kind, prec, ckpt):
    m, c_true, c0, eta, dt, nt, f0, xs, xr = case(kind)
    S = len(xs)
    say(f"shots: {kind} {prec} S={S} checkpoint_every={ckpt}")
    pb = problem(m, dt, nt, prec, eta, f0, xs, xr, checkpoint_every=ckpt)
    obs = pb.forward(cuda(c_true))
    assert tuple(obs.shape) == (S, nt, len(xr))
    Jb, gb, trb = pb.misfit_gradient(cuda(c0), obs, keep_traces=True)
    Js, gs = [], []
    for s in range(S):
        p1 = problem(m, dt, nt, prec, eta, f0, xs[s], xr, checkpoint_every=ckpt)
        o1 = p1.forward(cuda(c_true))
        assert torch.equal(o1, obs[s]), f"forward traces of shot {s} differ from its one-shot problem"
        J1, g1, tr1 = p1.misfit_gradient(cuda(c0), o1, keep_traces=True)
        assert torch.equal(tr1, trb[s]), f"misfit traces of shot {s} differ"
        Js.append(J1)
        gs.append(g1.cpu().numpy())
        p1.close()
    pb.close()
    gsum = np.sum(gs, axis=0)
    say(f"  J {Jb:.12e} sum {sum(Js):.12e}; gradient rel {rel_l2(gb.cpu().numpy(), gsum):.2e}")
    assert sum(Js) > 0
    assert abs(Jb - sum(Js)) <= 1e-12 * sum(Js)
    assert rel_l2(gb.cpu().numpy(), gsum) < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_shots_adjoint_source_traces(prec):
    """Adjoint solves of several shots with their own data: each shot's source trace
    equals its one-shot problem's bitwise, and the dot-product identity holds."""
    m, c_true, c0, eta, dt, nt, f0, xs, xr = case("tri")
    S = len(xs)
    say(f"shots: adjoint source traces {prec} S={S}")
    rng = np.random.default_rng(4)
    wav = rng.standard_normal(nt)
    pb = problem(m, dt, nt, prec, eta, f0, xs, xr)
    pb.set_source_wavelet(wav)
    c = cuda(c0)
    tr = pb.forward(c)
    y = rng.standard_normal((S, nt, len(xr)))
    _, st = pb.adjoint(c, cuda(y, pb.dtype), src_trace=True)
    assert tuple(st.shape) == (S, nt, 2)
    for s in range(S):
        p1 = problem(m, dt, nt, prec, eta, f0, xs[s], xr)
        p1.set_source_wavelet(wav)
        _, st1 = p1.adjoint(c, cuda(y[s], p1.dtype), src_trace=True)
        assert torch.equal(st1, st[s]), f"source traces of shot {s} differ"
        lhs = float(np.sum(y[s] * tr[s].double().cpu().numpy()))
        rhs = dt * dt * float(np.sum(wav[:, None] * st[s].double().cpu().numpy()))
        tol = 1e-12 if prec == "fp64" else 1e-5
        assert abs(lhs - rhs) <= tol * abs(lhs)
        p1.close()
    pb.close()


def test_shots_fp64_against_oracle():
    """J and gradient of a three-shot FP64 problem against the oracle's sums."""
    from oracle.fem import Discretization
    from oracle import solver
    coords, cells = configs.small_tri(8, seed=6)
    k, nt = 3, 250
    d = Discretization(coords, cells, k)
    c_true = d.nodal_values(lambda x, z: 1.5 + 0.4 * z + 0.1 * np.sin(4 * x))
    c0 = d.nodal_values(lambda x, z: 1.5 + 0.4 * z)
    eta = d.nodal_values(lambda x, z: sponge_eta(x, z, 0.0, 1.0, 0.8, 0.2, c_max=2.5))
    dt = 0.8 * solver.cfl_dt_gershgorin(d.stiffness(c_true), d.lumped_mass())
    xs = np.array([[[0.3, 0.1]], [[0.5, 0.1]], [[0.7, 0.12]]])
    xr = np.stack([np.linspace(0.1, 0.9, 10), np.full(10, 0.2)], axis=1)
    J_or, g_or = 0.0, np.zeros(d.n_dofs)
    obs = []
    for s in range(3):
        sh = solver.Shot(d, xs[s], xr, dt, nt, f0=8.0, t0=0.1)
        dobs, _ = sh.forward(c_true, eta)
        J, g, _ = sh.misfit_gradient(c0, dobs, eta)
        J_or += J
        g_or += g
        obs.append(dobs)
    from paper_2108_10946_amd import Mesh
    m = Mesh(coords, cells, k, patch_cells=11)
    p = dof_map(m.dof_coords(), d.dof_coords)
    say("shots: three-shot FP64 problem vs oracle")
    pb = problem(m, dt, nt, "fp64", eta[p], 8.0, xs, xr, checkpoint_every=9)
    Jb, gb, _ = pb.misfit_gradient(cuda(c0[p]), cuda(np.stack(obs)))
    pb.close()
    assert abs(Jb - J_or) < 1e-10 * J_or
    assert rel_l2(gb.cpu().numpy(), g_or[p]) < 1e-10


def test_shots_argument_errors():
    from paper_2108_10946_amd import Problem
    from paper_2108_10946_amd import kmvwave as K
    m, c_true, c0, eta, dt, nt, f0, xs, xr = case("tri")
    say("shots: argument errors")
    p = Problem(m, dt, nt, precision="fp32", n_shots=2)
    assert K.kmv_problem_num_shots(p.handle) == 2
    with pytest.raises(K.KMVError) as e:
        p.set_sources(xs[0][:1], f0=f0)  # one point for two shots
    assert e.value.code == K.KMV_EINVAL
    p.set_sources(xs[:2], f0=f0)
    p.set_receivers(xr)
    with pytest.raises(ValueError):
        p.misfit_gradient(cuda(c0), torch.zeros((nt, len(xr)), device="cuda"))
    with pytest.raises(ValueError):
        p.adjoint(cuda(c0), torch.zeros((2, nt, len(xr)), device="cuda"), keep_lambda=True)
    p.close()
    with pytest.raises(K.KMVError) as e:
        Problem(m, dt, nt, precision="fp32", n_shots=2000)
    assert e.value.code == K.KMV_EINVAL


@pytest.mark.parametrize("kind", ["tri", "tet"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_per_shot_wavelets(kind, prec):
    """kmv_set_source_wavelets: each shot fires its own wavelet (here Ricker pulses
    of different delay, frequency and polarity).  Each shot's traces are bitwise those
    of a one-shot problem given that wavelet; J and the gradient are the sums (1e-12)."""
    m, c_true, c0, eta, dt, nt, f0, xs, xr = case(kind)
    S = len(xs)
    t = np.arange(nt) * dt
    rng = np.random.default_rng(29)
    waves = []
    for s in range(S):
        f, t0, sgn = f0 * rng.uniform(0.8, 1.2), rng.uniform(0.08, 0.14), rng.choice([-1.0, 1.0])
        a = (np.pi * f * (t - t0)) ** 2
        waves.append(sgn * (1 - 2 * a) * np.exp(-a))
    waves = np.stack(waves)
    say(f"shots: per-shot wavelets {kind} {prec} S={S}")
    pb = problem(m, dt, nt, prec, eta, f0, xs, xr)
    pb.set_source_wavelet(waves)
    obs = pb.forward(cuda(c_true))
    Jb, gb, trb = pb.misfit_gradient(cuda(c0), obs, keep_traces=True)
    Js, gs = [], []
    for s in range(S):
        p1 = problem(m, dt, nt, prec, eta, f0, xs[s], xr)
        p1.set_source_wavelet(waves[s])
        o1 = p1.forward(cuda(c_true))
        assert torch.equal(o1, obs[s]), f"forward traces of shot {s} differ from its one-shot problem"
        J1, g1, tr1 = p1.misfit_gradient(cuda(c0), o1, keep_traces=True)
        assert torch.equal(tr1, trb[s]), f"misfit traces of shot {s} differ"
        Js.append(J1)
        gs.append(g1.cpu().numpy())
        p1.close()
    # a shared wavelet again: every shot fires waves[0]
    pb.set_source_wavelet(waves[0])
    o_shared = pb.forward(cuda(c_true))
    p0 = problem(m, dt, nt, prec, eta, f0, xs[1], xr)
    p0.set_source_wavelet(waves[0])
    assert torch.equal(p0.forward(cuda(c_true)), o_shared[1])
    p0.close()
    with pytest.raises(ValueError):
        pb.set_source_wavelet(waves[:, :-1])
    pb.close()
    gsum = np.sum(gs, axis=0)
    assert abs(Jb - sum(Js)) <= 1e-12 * sum(Js)
    assert rel_l2(gb.cpu().numpy(), gsum) < 1e-12


def test_per_shot_wavelets_vs_oracle():
    """FP64, two shots with seeded random wavelets of their own, against the oracle
    run shot by shot with the same wavelets: J, traces and gradient to 1e-10."""
    from oracle.fem import Discretization
    from oracle import solver
    from paper_2108_10946_amd import Mesh, Problem
    from gpu_util import dof_map
    coords, cells = configs.small_tri(7, seed=8)
    k = 2
    d = Discretization(coords, cells, k)
    c_true = d.nodal_values(lambda x, z: 1.5 + 0.4 * z + 0.1 * np.sin(5 * x))
    c0 = d.nodal_values(lambda x, z: 1.5 + 0.4 * z)
    dt = 0.8 * solver.cfl_dt_gershgorin(d.stiffness(c_true), d.lumped_mass())
    nt = 150
    rng = np.random.default_rng(31)
    waves = rng.standard_normal((2, nt))
    xs = np.array([[[0.3, 0.2]], [[0.7, 0.4]]])
    xr = np.stack([np.linspace(0.1, 0.9, 6), np.full(6, 0.15)], axis=1)
    J_or, g_or, tr_or, obs = 0.0, np.zeros(d.n_dofs), [], []
    for s in range(2):
        sh = solver.Shot(d, xs[s], xr, dt, nt, wavelet=waves[s])
        dobs, _ = sh.forward(c_true)
        J, g, tr = sh.misfit_gradient(c0, dobs)
        J_or, g_or = J_or + J, g_or + g
        tr_or.append(tr)
        obs.append(dobs)
    m = Mesh(coords, cells, k, patch_cells=11)
    p = dof_map(m.dof_coords(), d.dof_coords)
    say("shots: per-shot wavelets vs oracle, fp64")
    prob = Problem(m, dt, nt, precision="fp64", n_shots=2)
    prob.set_sources(xs, f0=8.0)
    prob.set_source_wavelet(waves)
    prob.set_receivers(xr)
    J, g, tr = prob.misfit_gradient(cuda(c0[p]), cuda(np.stack(obs)), keep_traces=True)
    prob.close()
    assert abs(J - J_or) < 1e-10 * J_or
    assert rel_l2(tr.cpu().numpy(), np.stack(tr_or)) < 1e-10
    assert rel_l2(g.cpu().numpy(), g_or[p]) < 1e-10


def test_maximum_shot_count():
    """1024 shots, the most one problem takes, on a small mesh of 7-cell patches: the
    work-item mapping then deals n_patches * 1024 workgroups over the XCDs.  Sampled
    shots' traces are bitwise those of one-shot problems.  The observed data equal the
    computed traces except at the sampled shots, so every other shot's residual, and
    its gradient term, is exactly zero: J and the gradient are then the sampled shots'
    sums (1e-12 relative, the float64 order of the sum)."""
    from paper_2108_10946_amd import Mesh
    coords, cells = configs.small_tri(4, seed=3)
    m = Mesh(coords, cells, 2, patch_cells=7)
    x = m.dof_coords()
    c = 1.5 + 0.5 * x[:, 1]
    S, nt, f0 = 1024, 40, 8.0
    xs = np.stack([[[0.05 + 0.9 * s / (S - 1), 0.5]] for s in range(S)])
    xr = np.array([[0.3, 0.3], [0.6, 0.45], [0.55, 0.8]])
    dt = 0.5 * m.cfl_dt(c)
    say(f"shots: maximum shot count S={S}")
    pb = problem(m, dt, nt, "fp32", None, f0, xs, xr)
    cg = torch.as_tensor(c, dtype=torch.float64, device="cuda")
    tr = pb.forward(cg).cpu().numpy()
    assert tr.shape == (S, nt, len(xr))
    sample = [0, 1, 7, 8, 9, 511, 1016, 1023]
    rng = np.random.default_rng(3)
    obs = tr.copy()
    for s in sample:
        obs[s] += rng.standard_normal((nt, len(xr))).astype(np.float32) * 1e-3
    J, g, _ = pb.misfit_gradient(cg, torch.as_tensor(obs, device="cuda"), keep_traces=True)
    g = g.cpu().numpy()
    pb.close()
    J1, g1 = 0.0, np.zeros_like(g)
    for s in sample:
        p1 = problem(m, dt, nt, "fp32", None, f0, xs[s], xr)
        assert np.array_equal(p1.forward(cg).cpu().numpy(), tr[s])
        Js, gs, _ = p1.misfit_gradient(cg, torch.as_tensor(obs[s], device="cuda"), keep_traces=True)
        J1, g1 = J1 + Js, g1 + gs.cpu().numpy()
        p1.close()
    assert J1 > 0 and abs(J - J1) < 1e-12 * J1
    assert rel_l2(g, g1) < 1e-12
