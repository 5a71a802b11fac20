"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Tolerances (relative L2 unless stated):
  FP64 mode: 1e-12 for one stiffness apply, 1e-10 for traces, misfit and gradient
             after hundreds to a thousand steps.
  FP32 mode: 1e-5 for one apply on random data (float32 rounding of ~n_d^2 terms),
             1e-4 on traces and 1e-3 on the gradient after the full time window.
DOFs are matched by coordinates (the library and the oracle number them
independently)."""
import numpy as np
import pytest

from gpu_util import say, dof_map, rel_l2
from oracle.fem import Discretization
from oracle import solver
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


def lib_mesh(coords, cells, k, patch=0):
    from paper_2108_10946_amd import Mesh
    return Mesh(coords, cells, k, patch_cells=patch)


def cuda(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


APPLY_CASES = [("tri", k, patch) for k in (1, 2, 3, 4, 5) for patch in (0, 13)] + \
              [("tet", k, patch) for k in (1, 2, 3) for patch in (0, 7)]


@pytest.mark.parametrize("kind,k,patch", APPLY_CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stiffness_apply(kind, k, patch, prec):
    from paper_2108_10946_amd import Problem
    coords, cells = configs.small_tri(9, seed=4) if kind == "tri" else configs.small_tet(3, seed=4)
    say(f"apply {kind} k={k} patch={patch} {prec}")
    m = lib_mesh(coords, cells, k, patch)
    d = Discretization(coords, cells, k)
    p = dof_map(m.dof_coords(), d.dof_coords)
    rng = np.random.default_rng(k)
    c_or = 1.0 + rng.random(d.n_dofs)
    u_or = rng.standard_normal(d.n_dofs)
    y_or = d.stiffness(c_or) @ u_or
    prob = Problem(m, 1e-3, 4, precision=prec)
    y = prob.stiffness_apply(cuda(c_or[p]), cuda(u_or[p], prob.dtype)).double().cpu().numpy()
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert rel_l2(y, y_or[p]) < tol


@pytest.fixture(scope="module")
def c1():
    w = configs.homog_kmv2_c1()
    d = Discretization(w.coords, w.cells, 2)
    sh = solver.Shot(d, w.sources, w.receivers, w.dt, 1000)
    c_or = d.nodal_values(w.vp)
    dobs, _ = sh.forward(d.nodal_values(w.vp_obs))
    J, g, tr = sh.misfit_gradient(c_or, dobs)
    return w, d, sh, c_or, dobs, J, g, tr


def c1_problem(w, prec, **kw):
    from paper_2108_10946_amd import Problem
    m = lib_mesh(w.coords, w.cells, 2, kw.pop("patch", 0))
    prob = Problem(m, w.dt, 1000, precision=prec, **kw)
    prob.set_sources(w.sources, f0=w.f0, t0=w.t0)
    prob.set_receivers(w.receivers)
    return m, prob


def test_c1_forward_fp64(c1):
    w, d, sh, c_or, dobs, J, g, tr = c1
    say("c1 forward fp64")
    m, prob = c1_problem(w, "fp64")
    p = dof_map(m.dof_coords(), d.dof_coords)
    traces = prob.forward(cuda(d.nodal_values(w.vp_obs)[p])).cpu().numpy()
    assert rel_l2(traces, dobs) < 1e-10


@pytest.mark.parametrize("ckpt", [0, 37])
def test_c1_misfit_gradient_fp64(c1, ckpt):
    w, d, sh, c_or, dobs, J, g, tr = c1
    say(f"c1 misfit+gradient fp64 checkpoint_every={ckpt}")
    m, prob = c1_problem(w, "fp64", checkpoint_every=ckpt)
    p = dof_map(m.dof_coords(), d.dof_coords)
    Jg, gg, trg = prob.misfit_gradient(cuda(c_or[p]), cuda(dobs), keep_traces=True)
    assert abs(Jg - J) < 1e-10 * J
    assert rel_l2(trg.cpu().numpy(), tr) < 1e-10
    assert rel_l2(gg.cpu().numpy(), g[p]) < 1e-10


def test_c1_fp32_tolerances(c1):
    w, d, sh, c_or, dobs, J, g, tr = c1
    say("c1 misfit+gradient fp32")
    m, prob = c1_problem(w, "fp32")
    p = dof_map(m.dof_coords(), d.dof_coords)
    Jg, gg, trg = prob.misfit_gradient(cuda(c_or[p]), cuda(dobs), keep_traces=True)
    e_tr = rel_l2(trg.double().cpu().numpy(), tr)
    e_g = rel_l2(gg.cpu().numpy(), g[p])
    print(f"fp32 errors: traces {e_tr:.2e} gradient {e_g:.2e} J {abs(Jg - J) / J:.2e}")
    assert e_tr < 1e-4
    assert e_g < 1e-3
    assert abs(Jg - J) < 1e-3 * J


def test_c1_bitwise_determinism(c1):
    """Two runs, and store-all vs checkpoint recompute, give identical bits."""
    w, d, sh, c_or, dobs, J, g, tr = c1
    say("c1 determinism fp32")
    m, prob = c1_problem(w, "fp32")
    p = dof_map(m.dof_coords(), d.dof_coords)
    c = cuda(c_or[p])
    o = cuda(dobs, torch.float32)
    J1, g1, _ = prob.misfit_gradient(c, o)
    J2, g2, _ = prob.misfit_gradient(c, o)
    from paper_2108_10946_amd import Problem
    prob2 = Problem(m, w.dt, 1000, precision="fp32", checkpoint_every=64)
    prob2.set_sources(w.sources, f0=w.f0, t0=w.t0)
    prob2.set_receivers(w.receivers)
    J3, g3, _ = prob2.misfit_gradient(c, o)
    assert J1 == J2 == J3
    assert torch.equal(g1, g2) and torch.equal(g1, g3)


@pytest.fixture(scope="module")
def sponge_case():
    coords, cells = configs.small_tri(14, seed=8)
    d = Discretization(coords, cells, 3)
    rng = np.random.default_rng(1)
    c_true = d.nodal_values(lambda x, z: 1.5 + 0.5 * z + 0.1 * np.sin(6 * x))
    c0 = d.nodal_values(lambda x, z: 1.5 + 0.5 * z)
    eta = d.nodal_values(lambda x, z: sponge_eta(x, z, 0.15, 0.85, 0.85, 0.15, c_max=2.0))
    M = d.lumped_mass()
    dt = 0.9 * 2.0 / np.sqrt(solver.power_rho(d.stiffness(c_true), M, 300))
    nt = 400
    src = np.array([[0.5, 0.05]])
    rec = np.stack([np.linspace(0.1, 0.9, 9), np.full(9, 0.1)], 1)
    sh = solver.Shot(d, src, rec, dt, nt, f0=8.0, t0=0.12)
    dobs, _ = sh.forward(c_true, eta)
    J, g, tr = sh.misfit_gradient(c0, dobs, eta)
    return coords, cells, d, dt, nt, src, rec, c0, eta, dobs, J, g, tr


@pytest.mark.parametrize("prec,patch", [("fp64", 0), ("fp64", 11), ("fp32", 0)])
def test_sponge_kmv3_gradient(sponge_case, prec, patch):
    from paper_2108_10946_amd import Problem
    coords, cells, d, dt, nt, src, rec, c0, eta, dobs, J, g, tr = sponge_case
    say(f"sponge kmv3 {prec} patch={patch}")
    m = lib_mesh(coords, cells, 3, patch)
    p = dof_map(m.dof_coords(), d.dof_coords)
    prob = Problem(m, dt, nt, precision=prec)
    prob.set_damping(eta[p])
    prob.set_sources(src, f0=8.0, t0=0.12)
    prob.set_receivers(rec)
    Jg, gg, trg = prob.misfit_gradient(cuda(c0[p]), cuda(dobs), keep_traces=True)
    tol_t, tol_g = (1e-10, 1e-10) if prec == "fp64" else (1e-4, 1e-3)
    assert rel_l2(trg.double().cpu().numpy(), tr) < tol_t
    assert rel_l2(gg.cpu().numpy(), g[p]) < tol_g
    assert abs(Jg - J) < max(tol_t, 1e-9) * J * 10


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_dot_product(sponge_case, prec):
    """<y, P u(w)> = dt^2 sum_n w_n s . lambda^{n+1}(y), GPU path only."""
    from paper_2108_10946_amd import Problem
    coords, cells, d, dt, nt, src, rec, c0, eta, dobs, J, g, tr = sponge_case
    say(f"dot product {prec}")
    m = lib_mesh(coords, cells, 3)
    p = dof_map(m.dof_coords(), d.dof_coords)
    prob = Problem(m, dt, nt, precision=prec)
    prob.set_damping(eta[p])
    prob.set_sources(src, f0=8.0, t0=0.12)
    rng = np.random.default_rng(5)
    w = rng.standard_normal(nt)
    prob.set_source_wavelet(w)
    prob.set_receivers(rec)
    c = cuda(c0[p])
    tr_f = prob.forward(c).double().cpu().numpy()
    y = rng.standard_normal((nt, len(rec)))
    _, st = prob.adjoint(c, cuda(y, prob.dtype), src_trace=True)
    lhs = np.sum(y * tr_f)
    rhs = dt * dt * np.sum(w * st.double().cpu().numpy()[:, 0])
    tol = 1e-12 if prec == "fp64" else 1e-5
    assert abs(lhs - rhs) < tol * abs(lhs)


def test_lambda_matches_oracle(sponge_case):
    from paper_2108_10946_amd import Problem
    coords, cells, d, dt, nt, src, rec, c0, eta, dobs, J, g, tr = sponge_case
    say("adjoint fields fp64")
    m = lib_mesh(coords, cells, 3)
    p = dof_map(m.dof_coords(), d.dof_coords)
    prob = Problem(m, dt, nt, precision="fp64")
    prob.set_damping(eta[p])
    prob.set_sources(src, f0=8.0, t0=0.12)
    prob.set_receivers(rec)
    rng = np.random.default_rng(6)
    y = rng.standard_normal((nt, len(rec)))
    lam, _ = prob.adjoint(cuda(c0[p]), cuda(y), keep_lambda=True)
    K = d.stiffness(c0)
    lam_or = solver.adjoint(K, d.lumped_mass(), eta * dt / 2, dt, sh_P(d, rec), y)
    lam_np = lam.cpu().numpy()
    for mm in (1, nt // 2, nt):
        assert rel_l2(lam_np[mm - 1], lam_or[mm - 1][p]) < 1e-10
    assert np.all(lam_np[nt] == 0)


def sh_P(d, rec):
    return d.interpolation_matrix(rec)


def test_spectral_radius(sponge_case):
    from paper_2108_10946_amd import Problem
    coords, cells, d, dt, nt, src, rec, c0, eta, dobs, J, g, tr = sponge_case
    say("spectral radius")
    m = lib_mesh(coords, cells, 3)
    p = dof_map(m.dof_coords(), d.dof_coords)
    prob = Problem(m, dt, 4, precision="fp64")
    rho = prob.spectral_radius(cuda(c0[p]), iters=1500)
    rho_or = solver.power_rho(d.stiffness(c0), d.lumped_mass(), 3000)
    assert abs(rho - rho_or) < 1e-4 * rho_or


def test_outside_point_raises():
    from paper_2108_10946_amd import Problem, KMVError
    coords, cells = configs.small_tri(4)
    say("outside point")
    m = lib_mesh(coords, cells, 2)
    prob = Problem(m, 1e-3, 10)
    with pytest.raises(KMVError) as ei:
        prob.set_receivers([[2.0, 0.5]])
    assert ei.value.code == -5


@pytest.mark.parametrize("k", [2, 3])
def test_tet_gradient_fp64(k):
    from paper_2108_10946_amd import Problem
    coords, cells = configs.small_tet(4, seed=6)
    say(f"tet k={k} gradient fp64")
    d = Discretization(coords, cells, k)
    c_true = d.nodal_values(lambda x, y, z: 1.5 + 0.3 * z)
    c0 = np.full(d.n_dofs, 1.5)
    dt = 0.8 * 2.0 / np.sqrt(solver.power_rho(d.stiffness(c_true), d.lumped_mass(), 200))
    nt = 150
    src = np.array([[0.5, 0.5, 0.1]])
    rec = np.array([[0.2, 0.3, 0.8], [0.7, 0.6, 0.75], [0.5, 0.5, 0.9]])
    sh = solver.Shot(d, src, rec, dt, nt, f0=10.0, t0=0.1)
    dobs, _ = sh.forward(c_true)
    J, g, tr = sh.misfit_gradient(c0, dobs)
    m = lib_mesh(coords, cells, k)
    p = dof_map(m.dof_coords(), d.dof_coords)
    prob = Problem(m, dt, nt, precision="fp64")
    prob.set_sources(src, f0=10.0, t0=0.1)
    prob.set_receivers(rec)
    Jg, gg, trg = prob.misfit_gradient(cuda(c0[p]), cuda(dobs), keep_traces=True)
    assert rel_l2(trg.cpu().numpy(), tr) < 1e-10
    assert rel_l2(gg.cpu().numpy(), g[p]) < 1e-10
