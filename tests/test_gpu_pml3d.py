"""The perfectly matched layer on tetrahedra (auxiliary p_x, p_y, p_z and omega) on
the GPU against the oracle (oracle.pml, 3D): misfit, traces and gradient for every
tetrahedron degree, the adjoint's dot-product identity, gradient subsampling, and
the limits of the 3D form.  The layer covers the sides and the bottom of the unit
cube, so its corners carry all three damping functions (the Psi_3 and det Psi_1
terms).  Tolerances: FP64 1e-10 relative L2 on J, traces and gradient; FP32 1e-4 on
the traces and 1e-3 on the gradient; the dot product 1e-12 (FP64) and 1e-5 (FP32)."""
import numpy as np
import pytest

from gpu_util import say, dof_map, rel_l2
from oracle.fem import Discretization
from oracle import solver
from synth import configs
from synth.models import pml_sigma_3d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# (Kuhn-cube subdivisions) per degree: a few hundred to a few thousand DOFs
SIZES = {1: 5, 2: 3, 3: 2}


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_10946_amd as kmv
    kmv.lib()


@pytest.fixture(scope="module")
def cache():
    return {}


def case(k, cache):
    if k in cache:
        return cache[k]
    coords, cells = configs.small_tet(SIZES[k], seed=40 + k)
    d = Discretization(coords, cells, k)
    x, y, z = d.dof_coords.T
    c_true = 1.5 + 0.3 * z + 0.15 * np.exp(-((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.4) ** 2) / 0.03)
    c0 = 1.5 + 0.3 * z
    sig = pml_sigma_3d(x, y, z, (0.25, 0.25), (0.75, 0.75, 0.7), 0.25, c_max=2.0)
    src = [[0.45, 0.5, 0.15]]
    rec = np.stack([np.linspace(0.1, 0.9, 6), np.full(6, 0.45), np.full(6, 0.35)], axis=1)
    # sigma_max dt <= 0.25, as on triangles: the explicit PML terms bound the step too
    dt = min(0.8 * solver.cfl_dt_gershgorin(d.stiffness(c_true), d.lumped_mass()), 0.25 / sig.max())
    nt = max(60, int(np.ceil(0.4 / dt)))
    sh = solver.Shot(d, src, rec, dt, nt, f0=8.0, t0=0.1)
    dobs, _ = sh.forward(c_true, pml=sig)
    J, g, tr = sh.misfit_gradient(c0, dobs, pml=sig)
    cache[k] = dict(coords=coords, cells=cells, d=d, c0=c0, sig=sig, src=src, rec=rec, nt=nt, dt=dt,
                    dobs=dobs, J=J, g=g, tr=tr, sh=sh)
    return cache[k]


def problem(cs, k, prec, gradient_every=1, patch=0):
    from paper_2108_10946_amd import Mesh, Problem
    m = Mesh(cs["coords"], cs["cells"], k, patch_cells=patch)
    p = dof_map(m.dof_coords(), cs["d"].dof_coords)
    prob = Problem(m, cs["dt"], cs["nt"], precision=prec, gradient_every=gradient_every)
    prob.set_pml(cs["sig"][p])
    prob.set_sources(cs["src"], f0=8.0, t0=0.1)
    prob.set_receivers(cs["rec"])
    return m, p, prob


@pytest.mark.parametrize("k", [1, 2, 3])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pml3d_misfit_gradient_every_degree(k, prec, cache):
    cs = case(k, cache)
    say(f"pml 3d: tet k={k} {prec} N={cs['d'].n_dofs} nt={cs['nt']}")
    m, p, prob = problem(cs, k, prec, patch=64 if k == 3 else 0)
    c = torch.as_tensor(cs["c0"][p], dtype=torch.float64, device="cuda")
    obs = torch.as_tensor(cs["dobs"], dtype=prob.dtype, device="cuda")
    trf = prob.forward(c)
    prob.status()
    J, g, tr = prob.misfit_gradient(c, obs, keep_traces=True)
    Jm = prob.misfit(c, obs)
    prob.close()
    ef = rel_l2(trf.double().cpu().numpy(), cs["tr"])
    et, eg = rel_l2(tr.double().cpu().numpy(), cs["tr"]), rel_l2(g.cpu().numpy(), cs["g"][p])
    say(f"  J {J:.9e} (oracle {cs['J']:.9e}) forward {ef:.2e} traces {et:.2e} gradient {eg:.2e}")
    assert Jm == J  # the J-only path runs the same forward
    if prec == "fp64":
        assert abs(J - cs["J"]) < 1e-10 * cs["J"]
        assert ef < 1e-10 and et < 1e-10 and eg < 1e-10
    else:
        assert ef < 1e-4 and et < 1e-4 and eg < 1e-3


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_pml3d_adjoint_dot_product(prec, tol, cache):
    """<y, P u> = dt^2 sum_n w(t_n) s . lambda^{n+1} for the coupled u, p, omega scheme."""
    cs = case(2, cache)
    say(f"pml 3d: dot product {prec}")
    m, p, prob = problem(cs, 2, prec)
    c = torch.as_tensor(cs["c0"][p], dtype=torch.float64, device="cuda")
    u = prob.forward(c)
    y = torch.as_tensor(np.random.default_rng(5).standard_normal(u.shape), dtype=prob.dtype, device="cuda")
    lam, st = prob.adjoint(c, y, src_trace=True, keep_lambda=True)
    w = solver.ricker(np.arange(cs["nt"]) * cs["dt"], 8.0, 0.1)
    lhs = float((y.double() * u.double()).sum())
    rhs = cs["dt"] ** 2 * float(np.sum(w[:, None] * st.double().cpu().numpy()))
    prob.close()
    say(f"  <y, Pu> {lhs:.12e}  dt^2 sum w s.lam {rhs:.12e}")
    assert abs(lhs - rhs) < tol * abs(lhs)
    assert float(lam[-1].abs().max()) == 0.0  # row N_t = lambda^{N_t+1} = 0


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pml3d_gradient_subsampling(prec, cache):
    """gradient_every = 3: the pairing and its PML terms at every third reverse step,
    scaled by 3, as the oracle takes them."""
    cs = case(2, cache)
    say(f"pml 3d: gradient subsampling r=3 {prec}")
    J_or, g_or, _ = cs["sh"].misfit_gradient(cs["c0"], cs["dobs"], pml=cs["sig"], r=3)
    m, p, prob = problem(cs, 2, prec, gradient_every=3)
    c = torch.as_tensor(cs["c0"][p], dtype=torch.float64, device="cuda")
    J, g, _ = prob.misfit_gradient(c, torch.as_tensor(cs["dobs"], dtype=prob.dtype, device="cuda"))
    prob.close()
    eg = rel_l2(g.cpu().numpy(), g_or[p])
    say(f"  J {J:.9e} (oracle {J_or:.9e}) gradient {eg:.2e}")
    assert eg < (1e-10 if prec == "fp64" else 1e-3)


def test_pml3d_limits_and_switching(cache):
    from paper_2108_10946_amd import Mesh, Problem
    from paper_2108_10946_amd import kmvwave as K
    cs = case(1, cache)
    say("pml 3d: limits and switching off")
    m, p, prob = problem(cs, 1, "fp64")
    c = torch.as_tensor(cs["c0"][p], dtype=torch.float64, device="cuda")
    with pytest.raises(K.KMVError) as e:
        prob.set_damping(np.zeros(m.n_dofs))
    assert e.value.code == K.KMV_ESTATE
    with pytest.raises(K.KMVError) as e:
        prob.set_absorbing_boundary(True)
    assert e.value.code == K.KMV_ESTATE
    with pytest.raises(K.KMVError) as e:
        K.kmv_forward_noalloc(prob.handle, c, torch.empty(cs["nt"], len(cs["rec"]), dtype=torch.float64,
                                                          device="cuda"))
    assert e.value.code == K.KMV_ESTATE
    with pytest.raises(ValueError):
        prob.set_pml(np.zeros((m.n_dofs, 2)))  # one column per axis
    # off again: bitwise the problem that never had it
    prob.set_pml(None)
    a = prob.forward(c)
    plain = Problem(m, cs["dt"], cs["nt"], precision="fp64")
    plain.set_sources(cs["src"], f0=8.0, t0=0.1)
    plain.set_receivers(cs["rec"])
    assert torch.equal(a, plain.forward(c))
    plain.close()
    prob.close()
    # several shots per problem: refused
    two = Problem(m, cs["dt"], cs["nt"], precision="fp64", n_shots=2)
    with pytest.raises(K.KMVError) as e:
        two.set_pml(cs["sig"][p])
    assert e.value.code == K.KMV_EINVAL
    two.close()
