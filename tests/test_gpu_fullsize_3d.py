"""The 3D workload at full size: layered model with anomalies on 1.33 M
Maubach-graded tetrahedra (bisection refines in discrete levels; the nearest level
to the 1.5 M of the workload), KMV3tet (16.9 M DOFs), FP32 fields with float64
accumulation, checkpointed reverse sweep.

The oracle cannot assemble this operator in reasonable time, so the full-size checks
are sampled outputs it computes one by one, rows of the stiffness apply at 640 DOFs of
every node class (stored by tests/golden/gen_apply3d_fullsize.py), and properties that
hold at any size: the dot-product identity of the adjoint and central differences of
the misfit along a smooth seeded direction, also with the absorbing boundary term on
(its damping acts at the top surface next to the source from the first steps).  Oracle
parity of the same kernels in 3D runs on small tetrahedral meshes
(test_gpu_parity.py)."""
import numpy as np
import pytest

from gpu_util import say
from synth import configs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_10946_amd as kmv
    kmv.lib()


def cuda(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


@pytest.fixture(scope="module")
def c5():
    from paper_2108_10946_amd import Mesh, Problem
    say("3D full size: generating the graded tetrahedral mesh")
    w = configs.layered_tet_kmv3()
    say(f"3D full size: {len(w.cells)} tetrahedra; building the discretisation")
    m = Mesh(w.coords, w.cells, w.degree)
    x = m.dof_coords()
    c = w.vp(x[:, 0], x[:, 1], x[:, 2])
    eta = w.eta(x[:, 0], x[:, 1], x[:, 2])
    probe = Problem(m, 1e-4, 4, precision="fp32")
    rho = probe.spectral_radius(cuda(c), iters=100)
    probe.close()
    dt = 0.7 * 2.0 / np.sqrt(rho)  # margin: 100 power iterations underestimate rho
    say(f"3D full size: {m.n_dofs} DOFs, dt = {dt * 1e3:.4f} ms")
    return w, m, x, c, eta, dt


def test_dot_product_3d(c5):
    from paper_2108_10946_amd import Problem
    w, m, x, c, eta, dt = c5
    nt = 300
    say("3D full size: dot product, FP32")
    prob = Problem(m, dt, nt, precision="fp32")
    prob.set_damping(eta)
    prob.set_sources(w.sources, f0=w.f0, t0=0.05)
    rng = np.random.default_rng(9)
    wav = rng.standard_normal(nt)
    prob.set_source_wavelet(wav)
    prob.set_receivers(w.receivers)
    cd = cuda(c)
    tr = prob.forward(cd).double().cpu().numpy()
    y = rng.standard_normal((nt, len(w.receivers)))
    _, st = prob.adjoint(cd, cuda(y, prob.dtype), src_trace=True)
    lhs = np.sum(y * tr)
    rhs = dt * dt * np.sum(wav * st.double().cpu().numpy()[:, 0])
    say(f"  lhs {lhs:.9e} rhs {rhs:.9e} rel {abs(lhs - rhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)


def test_checkpointed_gradient_central_differences_3d(c5):
    """FP32 fields, float64 gradient accumulation, checkpoints every 25 steps."""
    from paper_2108_10946_amd import Problem, fwi_misfit
    w, m, x, c, eta, dt = c5
    nt, h = 300, 1e-3
    say("3D full size: checkpointed misfit gradient vs central differences, FP32")
    prob = Problem(m, dt, nt, precision="fp32", checkpoint_every=25)
    prob.set_damping(eta)
    prob.set_sources(w.sources, f0=w.f0, t0=0.05)
    prob.set_receivers(w.receivers)
    # observed data from a model with a smooth bump under the source
    bump = np.exp(-((x[:, 0] - 2.0) ** 2 + (x[:, 1] - 2.0) ** 2 + (x[:, 2] - 0.15) ** 2) / 0.01)
    obs = prob.forward(cuda(c * (1.0 + 0.1 * bump)))
    rng = np.random.default_rng(17)
    d = np.zeros(len(x))
    for _ in range(5):
        cx, cy, cz = rng.uniform([1.5, 1.5, 0.05], [2.5, 2.5, 0.4])
        d += rng.choice([-1.0, 1.0]) * np.exp(-((x[:, 0] - cx) ** 2 + (x[:, 1] - cy) ** 2 +
                                                (x[:, 2] - cz) ** 2) / 0.02)
    d[eta > 0] = 0.0
    d /= np.abs(d).max()
    cc = cuda(c).requires_grad_(True)
    J = fwi_misfit(cc, prob, obs)
    J.backward()
    an = float(cc.grad.cpu().numpy() @ d)
    fd = (float(fwi_misfit(cuda(c + h * d), prob, obs)) - float(fwi_misfit(cuda(c - h * d), prob, obs))) / (2 * h)
    say(f"  J {float(J):.6e} fd {fd:.6e} an {an:.6e} rel {abs(fd - an) / abs(an):.2e}")
    assert prob.info()["checkpoint_every"] == 25
    assert abs(fd - an) < 1e-2 * abs(an)


def test_absorbing_boundary_3d(c5):
    """Absorbing boundary on, FP32 fields, checkpoints every 25 steps: the adjoint's
    dot-product identity, and the gradient (boundary term included) against central
    differences along a direction concentrated at the top surface near the source."""
    from paper_2108_10946_amd import Problem
    w, m, x, c, eta, dt = c5
    nt, h = 300, 1e-3
    say("3D full size: absorbing boundary, dot product and central differences, FP32")
    prob = Problem(m, dt, nt, precision="fp32", checkpoint_every=25)
    prob.set_damping(eta)
    prob.set_absorbing_boundary(True)
    prob.set_sources(w.sources, f0=w.f0, t0=0.05)
    rng = np.random.default_rng(23)
    wav = rng.standard_normal(nt)
    prob.set_source_wavelet(wav)
    prob.set_receivers(w.receivers)
    cd = cuda(c)
    tr = prob.forward(cd).double().cpu().numpy()
    y = rng.standard_normal((nt, len(w.receivers)))
    _, st = prob.adjoint(cd, cuda(y, prob.dtype), src_trace=True)
    lhs = np.sum(y * tr)
    rhs = dt * dt * np.sum(wav * st.double().cpu().numpy()[:, 0])
    say(f"  dot: lhs {lhs:.9e} rhs {rhs:.9e} rel {abs(lhs - rhs) / abs(lhs):.2e}")
    assert abs(lhs - rhs) < 1e-5 * abs(lhs)
    prob.set_sources(w.sources, f0=w.f0, t0=0.05)  # back to the Ricker wavelet
    bump = np.exp(-((x[:, 0] - 2.0) ** 2 + (x[:, 1] - 2.0) ** 2 + (x[:, 2] - 0.15) ** 2) / 0.01)
    obs = prob.forward(cuda(c * (1.0 + 0.1 * bump)))
    d = np.exp(-((x[:, 0] - 2.1) ** 2 + (x[:, 1] - 1.9) ** 2 + x[:, 2] ** 2) / 0.02)
    d[eta > 0] = 0.0
    d /= np.abs(d).max()
    J, g, _ = prob.misfit_gradient(cd, obs)
    an = float(g.cpu().numpy() @ d)
    Jp, _, _ = prob.misfit_gradient(cuda(c + h * d), obs)
    Jm, _, _ = prob.misfit_gradient(cuda(c - h * d), obs)
    fd = (Jp - Jm) / (2 * h)
    say(f"  J {J:.6e} fd {fd:.6e} an {an:.6e} rel {abs(fd - an) / abs(an):.2e}")
    prob.close()
    assert abs(fd - an) < 1e-2 * abs(an)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_apply_rows_vs_stored_oracle(c5, prec, tol):
    """Rows of the stiffness apply y = K(c) u at full size against the oracle, at 640
    sampled DOFs of every node class (vertices, edges, faces, cell interiors) stored by
    tests/golden/gen_apply3d_fullsize.py, which discretises only the cells that hold
    each sampled DOF (a row of K u needs no other).  The apply runs in the launch
    configuration of the 3D leg (256-cell patches, whose shared refs exceed the first
    batch, so the loop over the remaining refs runs).  u oscillates on the scale of the
    cells, so K u cancels no more than with random data.  Tolerances as in the small-mesh
    apply tests: FP64 1e-12, FP32 1e-5 relative L2 over the sampled rows."""
    import importlib.util
    import json
    import os
    from scipy.spatial import cKDTree
    from paper_2108_10946_amd import Problem
    w, m, x, c, eta, dt = c5
    golden = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    spec = importlib.util.spec_from_file_location("gen_apply3d_fullsize",
                                                  os.path.join(golden, "gen_apply3d_fullsize.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    with open(os.path.join(golden, "apply3d_fullsize.json")) as f:
        ref = json.load(f)
    dist, idx = cKDTree(x).query(np.array(ref["coords"]))
    assert dist.max() < 1e-9
    st = m.patch_stats()
    assert st["max_shared_refs"] > st["first_batch_refs"]
    say(f"3D full size: apply rows {prec}")
    prob = Problem(m, dt, 4, precision=prec)
    y = prob.stiffness_apply(cuda(c), cuda(gen.u_field(*x.T), prob.dtype)).double().cpu().numpy()
    prob.close()
    y_or = np.array(ref["y"])
    err = np.linalg.norm(y[idx] - y_or) / np.linalg.norm(y_or)
    say(f"  {len(idx)} rows: {err:.2e}")
    assert err < tol
