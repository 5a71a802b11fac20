"""Discrete energy conservation of the library's recursion, with no oracle in between.
Without damping and with Neumann boundaries, the leapfrog M (v^{m-1} - 2 v^m + v^{m+1})
/ dt^2 + K v^m = 0 conserves E = 1/2 |(v^m - v^{m+1}) / dt|_M^2 + 1/2 (v^m)^T K v^{m+1}
exactly (M diagonal, K symmetric).  The adjoint sweep runs that recursion backwards:
driven by data rows only over the last steps of the window, its levels lambda^m
(kmv_adjoint with the levels kept) must hold E constant over every earlier step.  K v
comes from the library's own FP64 apply.  FP64 1e-11 relative over 200 free steps; FP32
levels 1e-5 (rounding of the float32 recursion)."""
import numpy as np
import pytest

from gpu_util import say
from synth import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NT, DRIVE = 260, 40  # data rows in the last DRIVE steps only


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_10946_amd as kmv
    kmv.lib()


@pytest.mark.parametrize("kind,k", [("tri", 2), ("tri", 4), ("tri", 5), ("tet", 2), ("tet", 3)])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 1e-5)])
def test_adjoint_energy_conservation(kind, k, prec, tol):
    from paper_2108_10946_amd import Mesh, Problem
    if kind == "tri":
        coords, cells = configs.small_tri(8, seed=29)
        rec = [[0.3, 0.4], [0.7, 0.55], [0.45, 0.8]]
    else:
        coords, cells = configs.small_tet(3, seed=29)
        rec = [[0.3, 0.4, 0.5], [0.7, 0.55, 0.35]]
    m = Mesh(coords, cells, k, patch_cells=13)
    x = m.dof_coords()
    c = 1.2 + 0.6 * x[:, -1] + 0.2 * np.sin(4 * x[:, 0])
    M = m.lumped_mass()
    dt = 0.6 * m.cfl_dt(c)
    cc = torch.as_tensor(c, device="cuda")
    prob = Problem(m, dt, NT, precision=prec)
    prob.set_sources([rec[0]], f0=8.0, t0=0.1)
    prob.set_receivers(rec)
    y = np.zeros((NT, len(rec)))
    y[NT - DRIVE:] = np.random.default_rng(k).standard_normal((DRIVE, len(rec)))
    lam, _ = prob.adjoint(cc, torch.as_tensor(y, dtype=prob.dtype, device="cuda"), keep_lambda=True)
    lam = lam.double()
    prob.close()
    k64 = Problem(m, dt, 4, precision="fp64")
    # levels lambda^1 .. lambda^(NT - DRIVE): no data row acts between them
    E = []
    for lvl in range(1, NT - DRIVE):
        a, b = lam[lvl - 1], lam[lvl]  # lambda^lvl, lambda^(lvl+1)
        d = ((a - b) / dt).cpu().numpy()
        Kb = k64.stiffness_apply(cc, b).cpu().numpy()
        E.append(0.5 * np.sum(M * d * d) + 0.5 * float(a.cpu().numpy() @ Kb))
    k64.close()
    m.close()
    E = np.array(E)
    drift = np.abs(E - E[-1]).max() / abs(E[-1])
    say(f"energy {kind} k={k} {prec}: E = {E[-1]:.6e}, drift over {len(E)} steps {drift:.1e}")
    assert E[-1] > 0 and drift < tol
