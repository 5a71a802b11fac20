"""Source-receiver reciprocity of the library's forward, with no oracle in between: the
point source is the transpose of the receiver interpolation (section 3.4) and every
operator of the step is symmetric (K(c), the lumped mass, the sponge and the absorbing
boundary's diagonal damping), so the trace recorded at B from a shot at A equals the
trace at A from a shot at B, to rounding.  Jittered meshes with a heterogeneous wave
speed and a sponge, points inside cells, on an edge and on a vertex; every triangle
degree and KMV2/KMV3 tetrahedra; with and without the absorbing boundary.  FP64 1e-12
and FP32 1e-5 relative to the largest sample."""
import numpy as np
import pytest

from gpu_util import say
from synth import configs
from synth.models import sponge_eta, sponge_eta_3d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_10946_amd as kmv
    kmv.lib()


def trace(m, c, eta, dt, nt, src, rec, prec, absorbing):
    from paper_2108_10946_amd import Problem
    prob = Problem(m, dt, nt, precision=prec)
    prob.set_damping(eta)
    if absorbing:
        prob.set_absorbing_boundary(True)
    prob.set_sources([src], f0=8.0, t0=0.1)
    prob.set_receivers([rec])
    out = prob.forward(torch.as_tensor(c, device="cuda")).double().cpu().numpy()[:, 0]
    prob.close()
    return out


CASES = [("tri", k) for k in (1, 2, 3, 4, 5)] + [("tet", k) for k in (2, 3)]


@pytest.mark.parametrize("kind,k", CASES)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
@pytest.mark.parametrize("absorbing", [False, True])
def test_reciprocity(kind, k, prec, tol, absorbing):
    from paper_2108_10946_amd import Mesh
    if kind == "tri":
        coords, cells = configs.small_tri(10, seed=21)
        pts = [(0.31, 0.42), (0.66, 0.27)]
        pts.append(tuple(coords[cells[40, 0]]))                           # a vertex
        pts.append(tuple(0.5 * (coords[cells[70, 0]] + coords[cells[70, 1]])))  # an edge midpoint
    else:
        coords, cells = configs.small_tet(3, seed=21)
        pts = [(0.31, 0.42, 0.37), (0.66, 0.27, 0.58), tuple(coords[cells[30, 0]])]
    m = Mesh(coords, cells, k)
    x = m.dof_coords()
    if kind == "tri":
        c = 1.5 + 0.8 * x[:, 1] + 0.2 * np.sin(5 * x[:, 0])
        eta = sponge_eta(x[:, 0], x[:, 1], 0.15, 0.85, 0.85, 0.15, c_max=2.5)
    else:
        c = 1.5 + 0.8 * x[:, 2] + 0.2 * np.sin(5 * x[:, 0])
        eta = sponge_eta_3d(x[:, 0], x[:, 1], x[:, 2], (0.15, 0.15), (0.85, 0.85, 0.85), 0.15, c_max=2.5)
    dt = 0.5 * m.cfl_dt(c)
    nt = max(150, int(np.ceil(0.5 / dt)))
    say(f"reciprocity {kind} k={k} {prec} absorbing={absorbing}: {m.n_dofs} DOFs, {nt} steps")
    worst = 0.0
    for i in range(len(pts)):
        for j in range(i + 1, len(pts)):
            ab = trace(m, c, eta, dt, nt, pts[i], pts[j], prec, absorbing)
            ba = trace(m, c, eta, dt, nt, pts[j], pts[i], prec, absorbing)
            scale = max(np.abs(ab).max(), np.abs(ba).max())
            assert scale > 0
            worst = max(worst, np.abs(ab - ba).max() / scale)
    say(f"  worst pair {worst:.2e}")
    m.close()
    assert worst < tol
