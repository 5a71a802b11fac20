"""The whole C2 time window against the oracle: N_t = 13,951 steps at the layered
KMV4 workload's step (T = 4 s), its layered model with the three anomalies, its
750 m sponge, source and 300 receivers, on a coarser mesh of the same model (scale
1.0 of the mesh recipe: 2,546 KMV4 triangles, 28,307 DOFs) so that the oracle's plain
FP64 recursion over the full window finishes in about two minutes.  At the full mesh
size the oracle runs a 300-step window (tests/test_gpu_fullsize.py); this file covers
the other axis, the number of steps over which FP32 rounding accumulates.

FP64: J, traces and gradient at 1e-10 relative L2.  FP32 (the bench's precision
form): traces 1e-4, gradient 1e-3, J 1e-4; the measured errors are printed."""
import numpy as np
import pytest

from gpu_util import say, dof_map, rel_l2
from oracle.fem import Discretization
from oracle import solver
from synth import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NT = 13951            # the layered KMV4 workload's steps for T = 4 s
DT = 4.0 / NT


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_10946_amd as kmv
    kmv.lib()


@pytest.fixture(scope="module")
def setup():
    w = configs.layered_kmv4(scale=1.0)
    d = Discretization(w.coords, w.cells, w.degree)
    x = d.dof_coords
    sh = solver.Shot(d, w.sources, w.receivers, DT, NT, f0=w.f0, t0=w.t0, amp=w.amp)
    return w, d, sh, w.vp_obs(*x.T), w.vp(*x.T), w.eta(*x.T)


@pytest.fixture(scope="module")
def observed(setup):
    w, d, sh, c_true, c0, eta = setup
    say(f"long window: oracle forward, {d.n_dofs} DOFs x {NT} steps")
    dobs, _ = sh.forward(c_true, eta)
    return dobs


@pytest.fixture(scope="module")
def reference(setup, observed):
    w, d, sh, c_true, c0, eta = setup
    say(f"long window: oracle misfit and gradient, {NT} steps")
    return sh.misfit_gradient(c0, observed, eta)


def gpu_problem(w, prec):
    from paper_2108_10946_amd import Mesh, Problem
    m = Mesh(w.coords, w.cells, w.degree)
    prob = Problem(m, DT, NT, precision=prec, mem_budget=16 << 30)
    prob.set_damping(w.eta(*m.dof_coords().T))
    prob.set_sources(w.sources, f0=w.f0, t0=w.t0, amp=w.amp)
    prob.set_receivers(w.receivers)
    return m, prob


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_long_window_forward(prec, setup, observed):
    w, d, sh, c_true, c0, eta = setup
    m, prob = gpu_problem(w, prec)
    p = dof_map(m.dof_coords(), d.dof_coords)
    say(f"long window: forward {prec}")
    tr = prob.forward(torch.as_tensor(c_true[p], dtype=torch.float64, device="cuda"))
    prob.status()
    prob.close()
    e = rel_l2(tr.double().cpu().numpy(), observed)
    say(f"  traces {e:.2e}")
    assert e < (1e-10 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_long_window_misfit_gradient(prec, setup, observed, reference):
    w, d, sh, c_true, c0, eta = setup
    J_or, g_or, tr_or = reference
    m, prob = gpu_problem(w, prec)
    p = dof_map(m.dof_coords(), d.dof_coords)
    say(f"long window: misfit and gradient {prec}")
    J, g, tr = prob.misfit_gradient(torch.as_tensor(c0[p], dtype=torch.float64, device="cuda"),
                                    torch.as_tensor(observed, dtype=prob.dtype, device="cuda"), keep_traces=True)
    prob.close()
    eJ = abs(J - J_or) / J_or
    et, eg = rel_l2(tr.double().cpu().numpy(), tr_or), rel_l2(g.cpu().numpy(), g_or[p])
    say(f"  J {J:.9e} (oracle {J_or:.9e}, {eJ:.1e}) traces {et:.2e} gradient {eg:.2e}")
    if prec == "fp64":
        assert eJ < 1e-10 and et < 1e-10 and eg < 1e-10
    else:
        assert eJ < 1e-4 and et < 1e-4 and eg < 1e-3
