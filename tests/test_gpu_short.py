"""Degenerate time lengths: N_t = 1, 2, 3, 4 and 7 steps.

The leapfrog recursion, the lagged finishing of shared DOFs (completed one launch
later), the checkpoint segments and the reverse sweep all meet their ends here.  At
N_t = 1 the discrete gradient is exactly zero: the only trace row comes from u^1,
whose adjoint pairs with the zero state u^0.  So it is at N_t = 2 with gradient
subsampling r = 2, where only n = 0 is paired.  The wavelet and the observed data are
seeded random draws, so no step is trivially zero.  Small patches (7 cells) make most
DOFs shared.  FP64 matches the oracle to 1e-10 relative L2; FP32 to 1e-4 (traces) and
1e-3 (gradient)."""
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


CASES = [(k, nt, ck, r, prec)
         for k in (2, 4)
         for nt in (1, 2, 3, 4, 7)
         for ck, r in ((0, 1), (2, 1), (1, 1), (0, 2))
         for prec in ("fp64", "fp32")]


@pytest.mark.parametrize("k,nt,ck,r,prec", CASES)
def test_short_sweeps(k, nt, ck, r, prec):
    from paper_2108_10946_amd import Mesh, Problem
    coords, cells = configs.small_tri(5, seed=3)
    d = Discretization(coords, cells, k)
    c0 = d.nodal_values(lambda x, z: 1.5 + 0.4 * z)
    eta = d.nodal_values(lambda x, z: sponge_eta(x, z, 0.0, 1.0, 0.8, 0.2, c_max=2.5))
    dt = 0.8 * solver.cfl_dt_gershgorin(d.stiffness(c0), d.lumped_mass())
    rng = np.random.default_rng(100 * k + nt)
    w = rng.standard_normal(nt)
    src = np.array([[0.5, 0.5]])
    rec = np.array([[0.3, 0.3], [0.6, 0.45], [0.55, 0.8]])
    dobs = rng.standard_normal((nt, len(rec))) * 1e-3
    sh = solver.Shot(d, src, rec, dt, nt, wavelet=w)
    J, g, tr = sh.misfit_gradient(c0, dobs, eta, r=r)

    m = Mesh(coords, cells, k, patch_cells=7)
    p = dof_map(m.dof_coords(), d.dof_coords)
    say(f"short sweep k={k} nt={nt} checkpoint_every={ck} r={r} {prec}")
    prob = Problem(m, dt, nt, precision=prec, checkpoint_every=ck, gradient_every=r)
    prob.set_damping(eta[p])
    prob.set_sources(src, f0=8.0, t0=0.1)
    prob.set_source_wavelet(w)
    prob.set_receivers(rec)
    cuda = lambda a, t=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=t, device="cuda")
    Jg, gg, trg = prob.misfit_gradient(cuda(c0[p]), cuda(dobs, prob.dtype), keep_traces=True)
    prob.close()
    trg, gg = trg.double().cpu().numpy(), gg.cpu().numpy()
    tol_t, tol_g, tol_j = (1e-10, 1e-10, 1e-10) if prec == "fp64" else (1e-4, 1e-3, 1e-3)
    assert trg.shape == tr.shape
    assert rel_l2(trg, tr) < tol_t
    assert abs(Jg - J) < tol_j * J
    if not np.any(g):  # every pairing is against the zero state u^0
        assert nt == 1 or (nt < 2 * r)
        assert np.all(gg == 0.0)
    else:
        assert rel_l2(gg, g[p]) < tol_g


@pytest.mark.parametrize("kind", ["tri", "tet"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_points_on_vertices_and_shared_edges(prec, kind):
    """A source on the vertex with the most cells, receivers on other such vertices and
    on midpoints of edges shared by two or more cells (in the tetrahedral mesh these
    edges lie on the domain boundary): each point lies in several cells, and every one
    of them gives the same value of the continuous field, so the library and the
    oracle agree whichever cell each picks (FP64 1e-10; FP32 1e-4 traces, 1e-3
    gradient)."""
    from paper_2108_10946_amd import Mesh, Problem
    if kind == "tri":
        coords, cells = configs.small_tri(6, seed=4)
        k, nt = 3, 150
    else:
        coords, cells = configs.small_tet(3, seed=5)
        k, nt = 2, 100
    d = Discretization(coords, cells, k)
    c0 = d.nodal_values(lambda *x: 1.5 + 0.4 * x[-1])
    dt = 0.8 * solver.cfl_dt_gershgorin(d.stiffness(c0), d.lumped_mass())
    # interior vertices: used by the most cells
    use = np.bincount(cells.ravel(), minlength=len(coords))
    inner = np.argsort(-use, kind="stable")[:4]
    src = coords[inner[:1]]
    e = sorted({(min(a, b), max(a, b)) for a, b in cells[:, :2]})
    shared = [(a, b) for (a, b) in e if sum(1 for c in cells if a in c and b in c) >= 2][:3]
    rec = np.vstack([coords[inner[1:]], [(coords[a] + coords[b]) / 2 for a, b in shared]])
    rng = np.random.default_rng(11)
    w = rng.standard_normal(nt)
    dobs = rng.standard_normal((nt, len(rec))) * 1e-3
    sh = solver.Shot(d, src, rec, dt, nt, wavelet=w)
    J, g, tr = sh.misfit_gradient(c0, dobs)
    m = Mesh(coords, cells, k, patch_cells=7)
    p = dof_map(m.dof_coords(), d.dof_coords)
    say(f"points on vertices and shared edges {prec}")
    prob = Problem(m, dt, nt, precision=prec)
    prob.set_sources(src, f0=8.0, t0=0.1)
    prob.set_source_wavelet(w)
    prob.set_receivers(rec)
    cuda = lambda a, t=torch.float64: torch.as_tensor(np.ascontiguousarray(a), dtype=t, device="cuda")
    Jg, gg, trg = prob.misfit_gradient(cuda(c0[p]), cuda(dobs, prob.dtype), keep_traces=True)
    prob.close()
    tol_t, tol_g = (1e-10, 1e-10) if prec == "fp64" else (1e-4, 1e-3)
    assert rel_l2(trg.double().cpu().numpy(), tr) < tol_t
    assert rel_l2(gg.cpu().numpy(), g[p]) < tol_g
    assert abs(Jg - J) < (1e-10 if prec == "fp64" else 1e-3) * J
