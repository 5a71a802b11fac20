"""Degenerate meshes on the GPU against the oracle: a mesh of one cell (one patch,
no DOF shared between patches, so the step kernel's shared-ref work is empty) for
every element, and one-cell patches on small meshes (every DOF on a cell boundary
shared, vertices by up to six patches on triangles, so the three-or-more-patch list
path finishes most shared DOFs).  Misfit, traces and gradient: FP64 1e-10 relative
L2; FP32 1e-4 on the traces and 1e-3 on the gradient, and J within what the traces'
bound allows: |dJ| <= |r| |dr| <= 1e-4 |r| |d| for J = |r|^2 / 2, r the residual and d
the traces (the residual is a small difference of traces on one cell)."""
import numpy as np
import pytest

from gpu_util import say, dof_map, rel_l2
from oracle.fem import Discretization
from oracle import solver
from synth import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

ONE_TRI = (np.array([[0.0, 0.0], [1.0, 0.0], [0.2, 0.9]]), np.array([[0, 1, 2]], dtype=np.int32),
           [[0.35, 0.3]], [[0.2, 0.1], [0.55, 0.2], [0.25, 0.6]])
ONE_TET = (np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.1, 0.9, 0.0], [0.2, 0.1, 0.8]]),
           np.array([[0, 1, 2, 3]], dtype=np.int32),
           [[0.3, 0.25, 0.2]], [[0.15, 0.1, 0.1], [0.4, 0.2, 0.1], [0.2, 0.4, 0.2]])


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_10946_amd as kmv
    kmv.lib()


def oracle_case(coords, cells, k, src, rec):
    d = Discretization(coords, cells, k)
    x = d.dof_coords
    c0 = 1.5 + 0.4 * x[:, 0]
    c_true = c0 + 0.2 * x[:, 1]
    dt = 0.5 * solver.cfl_dt_gershgorin(d.stiffness(c_true), d.lumped_mass())
    nt = max(80, int(np.ceil(0.6 / dt)))  # at least 0.6 s of the wavelet
    sh = solver.Shot(d, src, rec, dt, nt, f0=4.0, t0=0.15)
    dobs, _ = sh.forward(c_true)
    J, g, tr = sh.misfit_gradient(c0, dobs)
    return d, c0, dt, nt, dobs, J, g, tr


def run_gpu(coords, cells, k, src, rec, case, prec, patch=0):
    from paper_2108_10946_amd import Mesh, Problem
    d, c0, dt, nt, dobs, J_or, g_or, tr_or = case
    m = Mesh(coords, cells, k, patch_cells=patch)
    p = dof_map(m.dof_coords(), d.dof_coords)
    prob = Problem(m, dt, nt, precision=prec)
    prob.set_sources(src, f0=4.0, t0=0.15)
    prob.set_receivers(rec)
    c = torch.as_tensor(c0[p], dtype=torch.float64, device="cuda")
    J, g, tr = prob.misfit_gradient(c, torch.as_tensor(dobs, dtype=prob.dtype, device="cuda"), keep_traces=True)
    prob.status()
    prob.close()
    eJ = abs(J - J_or) / J_or
    et, eg = rel_l2(tr.double().cpu().numpy(), tr_or), rel_l2(g.cpu().numpy(), g_or[p])
    say(f"  J {J:.9e} (oracle {J_or:.9e}, {eJ:.1e}) traces {et:.2e} gradient {eg:.2e}")
    if prec == "fp64":
        assert eJ < 1e-10 and et < 1e-10 and eg < 1e-10
    else:
        assert et < 1e-4 and eg < 1e-3
        assert abs(J - J_or) <= 1e-4 * np.sqrt(2 * J_or) * np.linalg.norm(tr_or)
    return m


@pytest.mark.parametrize("kind,k", [("tri", k) for k in (1, 2, 3, 4, 5)] + [("tet", k) for k in (1, 2, 3)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_one_cell_mesh(kind, k, prec):
    coords, cells, src, rec = ONE_TRI if kind == "tri" else ONE_TET
    say(f"one-cell mesh: {kind} k={k} {prec}")
    case = oracle_case(coords, cells, k, src, rec)
    m = run_gpu(coords, cells, k, src, rec, case, prec)
    assert m.n_patches == 1 and m.patch_stats()["max_shared_refs"] == 0


@pytest.mark.parametrize("kind,k", [("tri", 2), ("tri", 4), ("tet", 2)])
def test_one_cell_patches(kind, k):
    if kind == "tri":
        coords, cells = configs.small_tri(3, seed=8)
        src, rec = [[0.45, 0.55]], [[0.2, 0.3], [0.7, 0.4], [0.5, 0.8]]
    else:
        coords, cells = configs.small_tet(2, seed=8)
        src, rec = [[0.45, 0.5, 0.4]], [[0.2, 0.3, 0.3], [0.7, 0.4, 0.6]]
    say(f"one-cell patches: {kind} k={k} ({len(cells)} cells)")
    case = oracle_case(coords, cells, k, src, rec)
    m = run_gpu(coords, cells, k, src, rec, case, "fp64", patch=1)
    assert m.n_patches == len(cells) and m.patch_stats()["max_patch_cells"] == 1
