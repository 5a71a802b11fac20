"""Misfit, traces and gradient against the oracle for every supported element
(triangles k = 1..5, tetrahedra k = 1..3), sponge damping on, with the default
patches and with small ragged ones (many patches, shared DOFs everywhere), over
0.5 s of simulated time at 0.8 x the Gershgorin step (60 to 825 steps).
Tolerances: FP64 1e-10 relative L2 on J, traces and gradient; FP32 1e-4 on the
traces and 1e-3 on the gradient."""
import numpy as np
import pytest

from gpu_util import say, dof_map, rel_l2
from oracle.fem import Discretization
from oracle import solver
from synth import configs
from synth.models import sponge_eta

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = [("tri", k) for k in (1, 2, 3, 4, 5)] + [("tet", k) for k in (1, 2, 3)]


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_10946_amd as kmv
    kmv.lib()


@pytest.fixture(scope="module")
def oracle_results():
    return {}


def oracle_case(kind, k, cache):
    if (kind, k) in cache:
        return cache[(kind, k)]
    if kind == "tri":
        coords, cells = configs.small_tri(7, seed=10 + k)
        d = Discretization(coords, cells, k)
        x, z = d.dof_coords[:, 0], d.dof_coords[:, 1]
        c_true = 1.5 + 0.4 * z + 0.15 * np.exp(-((x - 0.5) ** 2 + (z - 0.5) ** 2) / 0.03)
        c0 = 1.5 + 0.4 * z
        eta = sponge_eta(x, z, 0.0, 1.0, 0.8, 0.2, c_max=2.5)
        src = [[0.45, 0.1]]
        rec = np.stack([np.linspace(0.1, 0.9, 6), np.full(6, 0.25)], axis=1)
        f0 = 8.0
    else:
        coords, cells = configs.small_tet(3, seed=10 + k)
        d = Discretization(coords, cells, k)
        x, y, z = d.dof_coords.T
        c_true = 1.5 + 0.3 * z + 0.15 * np.exp(-((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2) / 0.05)
        c0 = 1.5 + 0.3 * z
        eta = 4.0 * np.maximum(0.0, x - 0.7) ** 2
        src = [[0.4, 0.45, 0.2]]
        rec = np.stack([np.linspace(0.15, 0.85, 5), np.full(5, 0.5), np.full(5, 0.3)], axis=1)
        f0 = 6.0
    dt = 0.8 * solver.cfl_dt_gershgorin(d.stiffness(c_true), d.lumped_mass())
    nt = max(60, int(np.ceil(0.5 / dt)))  # 0.5 s: the pulse reaches every receiver
    sh = solver.Shot(d, src, rec, dt, nt, f0=f0, t0=0.1)
    dobs, _ = sh.forward(c_true, eta)
    J, g, tr = sh.misfit_gradient(c0, dobs, eta)
    cache[(kind, k)] = (coords, cells, d, c0, eta, src, rec, nt, f0, dt, dobs, J, g, tr)
    return cache[(kind, k)]


@pytest.mark.parametrize("kind,k", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("small_patches", [False, True])
def test_misfit_gradient_every_element(kind, k, prec, small_patches, oracle_results):
    from paper_2108_10946_amd import Mesh, Problem
    coords, cells, d, c0, eta, src, rec, nt, f0, dt, dobs, J_or, g_or, tr_or = oracle_case(kind, k, oracle_results)
    patch = (9 if kind == "tri" else 5) if small_patches else 0
    say(f"degrees: {kind} k={k} {prec} patch={patch}")
    m = Mesh(coords, cells, k, patch_cells=patch)
    p = dof_map(m.dof_coords(), d.dof_coords)
    prob = Problem(m, dt, nt, precision=prec)
    prob.set_damping(eta[p])
    prob.set_sources(src, f0=f0, t0=0.1)
    prob.set_receivers(rec)
    obs = torch.as_tensor(dobs, dtype=prob.dtype, device="cuda")
    c = torch.as_tensor(c0[p], dtype=torch.float64, device="cuda")
    J, g, tr = prob.misfit_gradient(c, obs, keep_traces=True)
    prob.close()
    et, eg = rel_l2(tr.double().cpu().numpy(), tr_or), rel_l2(g.cpu().numpy(), g_or[p])
    say(f"  J {J:.9e} (oracle {J_or:.9e}) traces {et:.2e} gradient {eg:.2e}")
    if prec == "fp64":
        assert abs(J - J_or) < 1e-10 * J_or
        assert et < 1e-10 and eg < 1e-10
    else:
        assert et < 1e-4 and eg < 1e-3
