"""The paper's gradient-verification workload (section on the numerical
verification of the discrete gradient) on the GPU: 1 km x 1 km, upper half 4.0 km/s
and lower half 1.0 km/s, initial model 4.0 km/s, a 200 m absorbing layer, KMV2 on
20 m right triangles (8400 cells), T = 1 s at dt = 0.5 ms (2000 steps), and its 3D
analogue on KMV2 tetrahedra at a reduced size (140 m boxes).

* The full 2D workload against the oracle: J, traces and the gradient at 1e-10
  (FP64), with the sponge and with the PML; the 3D one likewise.
* The directional derivative d^co = c~^T M G along c~ = G masked in the layer
  (eq. control_deriv) against forward differences of J (eq. discrete_fd) at
  h = 1e-3, 1e-4, 1e-5.  The discrete gradient is the exact derivative of the
  discrete J, so in FP64 the difference falls in proportion to h (the same slope
  (d^fd - d^co)/h at every h, nothing left as h -> 0).  The paper's own table values stay parity-unpinned (other layer,
  conventions and scaling of the direction)."""
import numpy as np
import pytest

from gpu_util import say, dof_map, rel_l2
from oracle.fem import Discretization
from oracle import solver
from synth import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_10946_amd as kmv
    kmv.lib()


@pytest.fixture(scope="module")
def cache():
    return {}


def oracle(w, layer, cache):
    key = (w.name, len(w.cells), layer)
    if key in cache:
        return cache[key]
    d = Discretization(w.coords, w.cells, w.degree)
    x = d.dof_coords
    nt = int(round(w.T / w.dt))
    sh = solver.Shot(d, w.sources, w.receivers, w.dt, nt, f0=w.f0, t0=w.t0)
    c_true, c0 = w.vp_obs(*x.T), w.vp(*x.T)
    if layer == "pml":
        sig = w.extra["sigma"](*x.T)
        dobs, _ = sh.forward(c_true, pml=sig)
        J, g, tr = sh.misfit_gradient(c0, dobs, pml=sig)
    else:
        eta = w.eta(*x.T)
        dobs, _ = sh.forward(c_true, eta)
        J, g, tr = sh.misfit_gradient(c0, dobs, eta)
    cache[key] = (d, dobs, J, g, tr)
    return cache[key]


def gpu_problem(w, layer, prec):
    from paper_2108_10946_amd import Mesh, Problem
    m = Mesh(w.coords, w.cells, w.degree)
    x = m.dof_coords()
    nt = int(round(w.T / w.dt))
    prob = Problem(m, w.dt, nt, precision=prec, mem_budget=16 << 30)
    if layer == "pml":
        prob.set_pml(w.extra["sigma"](*x.T))
    else:
        prob.set_damping(w.eta(*x.T))
    prob.set_sources(w.sources, f0=w.f0, t0=w.t0)
    prob.set_receivers(w.receivers)
    return m, prob


CASES = [("2d", "sponge"), ("2d", "pml"), ("3d", "sponge"), ("3d", "pml")]


def workload(dim):
    return configs.gradient_check_2d() if dim == "2d" else configs.gradient_check_3d(le=0.14)


@pytest.mark.parametrize("dim,layer", CASES)
def test_gradient_check_workload_vs_oracle(dim, layer, cache):
    w = workload(dim)
    d, dobs, J_or, g_or, tr_or = oracle(w, layer, cache)
    say(f"gradient check: {dim} {layer} fp64 vs oracle, {len(w.cells)} cells, {d.n_dofs} DOFs")
    m, prob = gpu_problem(w, layer, "fp64")
    p = dof_map(m.dof_coords(), d.dof_coords)
    c = torch.as_tensor(w.vp(*m.dof_coords().T), dtype=torch.float64, device="cuda")
    J, g, tr = prob.misfit_gradient(c, torch.as_tensor(dobs, device="cuda"), keep_traces=True)
    prob.close()
    et, eg = rel_l2(tr.cpu().numpy(), tr_or), rel_l2(g.cpu().numpy(), g_or[p])
    say(f"  J {J:.9e} (oracle {J_or:.9e}) traces {et:.2e} gradient {eg:.2e}")
    assert abs(J - J_or) < 1e-10 * J_or and et < 1e-10 and eg < 1e-10


@pytest.mark.parametrize("dim,layer", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_directional_derivative(dim, layer, prec, cache):
    from paper_2108_10946_amd.fwi import directional_derivative_check
    w = workload(dim)
    d, dobs, _, _, _ = oracle(w, layer, cache)
    m, prob = gpu_problem(w, layer, prec)
    p = dof_map(m.dof_coords(), d.dof_coords)
    x = m.dof_coords()
    c = torch.as_tensor(w.vp(*x.T), dtype=torch.float64, device="cuda")
    obs = torch.as_tensor(dobs, dtype=prob.dtype, device="cuda")
    inside = (w.eta(*x.T) == 0.0)
    say(f"gradient check: {dim} {layer} {prec} directional derivative")
    r = directional_derivative_check(prob, c, obs, mask=inside)
    prob.close()
    say(f"  d_co {r['d_co']:.9e}  d_fd " + "  ".join(f"h={h:g}: {v:.9e} ({r['rel_err'][h]:.1e})"
                                                     for h, v in r["d_fd"].items()))
    # forward differences: d_fd(h) = d_co + a h + O(h^2) when d_co is the exact
    # derivative, so (d_fd(h) - d_co) / h is the same a at every h (first order,
    # nothing left over as h -> 0); FP32's rounding of J limits it to h = 1e-3
    e, fd, co = r["rel_err"], r["d_fd"], r["d_co"]
    slope = {h: (v - co) / h for h, v in fd.items()}
    if prec == "fp64":
        assert abs(slope[1e-4] / slope[1e-3] - 1.0) < 0.1, slope
        assert abs(slope[1e-5] / slope[1e-4] - 1.0) < 0.1, slope
        assert e[1e-5] < 1e-3
    else:
        assert e[1e-3] < 5e-2
