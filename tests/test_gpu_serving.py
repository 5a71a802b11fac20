"""Shot server (kmv_server_*): continuous admission, concurrent solves, results
equal alone and in the mix.

Every solve is deterministic and a request shares no buffer with another, so the
results of a request run together with others must be bitwise those it gets when
it runs alone; the FP64 results also match the oracle (1e-10 relative L2)."""
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


def make_requests():
    """Mixed degrees, durations, precisions and forward-only flags on three meshes."""
    from paper_2108_10946_amd import Mesh
    meshes = {}
    for key, (n, k, seed) in {"a": (8, 2, 1), "b": (10, 3, 2), "c": (7, 4, 3)}.items():
        coords, cells = configs.small_tri(n, seed=seed)
        meshes[key] = Mesh(coords, cells, k)
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(9):
        key = "abc"[i % 3]
        m = meshes[key]
        x = m.dof_coords()
        c = 1.5 + 0.5 * x[:, 1] + 0.05 * np.sin(7 * x[:, 0])
        rho_dt = 0.4 * m.cfl_dt(c)
        nt = int(rng.integers(120, 400))
        prec = "fp64" if i % 4 == 0 else "fp32"
        eta = sponge_eta(x[:, 0], x[:, 1], 0.0, 1.0, 0.8, 0.2, c_max=3.0) if i % 2 else None
        xs = [[0.2 + 0.6 * rng.random(), 0.05]]
        xr = np.stack([np.linspace(0.1, 0.9, 12), np.full(12, 0.15)], axis=1)
        fwd_only = i % 5 == 3
        obs = None if fwd_only else rng.standard_normal((nt, 12)) * 1e-3
        reqs.append(dict(mesh=m, c=c, xs=xs, xr=xr, dt=rho_dt, n_steps=nt, precision=prec, eta=eta,
                         observed=obs, forward_only=fwd_only, f0=8.0, t0=0.1))
    return meshes, reqs


def same(r1, r2):
    assert r1["status"] == 0 and r2["status"] == 0
    assert np.array_equal(r1["traces"], r2["traces"])
    if r1["grad"] is not None or r2["grad"] is not None:
        assert np.array_equal(r1["grad"], r2["grad"])
    assert r1["J"] == r2["J"]


def test_alone_equals_mix():
    from paper_2108_10946_amd import Server
    meshes, reqs = make_requests()
    say("serving: each request alone (one slot)")
    alone = []
    srv = Server(max_slots=1)
    for q in reqs:
        alone.append(srv.result(srv.submit(**q)))
    srv.close()
    say("serving: all requests at once (four slots)")
    srv = Server(max_slots=4)
    tickets = [srv.submit(**q) for q in reqs]
    mix = [srv.result(t) for t in tickets]
    srv.close()
    for i, (a, b) in enumerate(zip(alone, mix)):
        same(a, b)
    # requests overlapped in the mix: some request was admitted before another finished
    spans = sorted((r["t_admit"], r["t_done"]) for r in mix)
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))


def test_server_matches_problem_api_and_oracle():
    """A served FP64 shot equals the direct Problem call bitwise and the oracle to 1e-10."""
    from paper_2108_10946_amd import Mesh, Problem, Server
    coords, cells = configs.small_tri(8, seed=1)
    k, nt = 3, 200
    d = Discretization(coords, cells, k)
    c_true = d.nodal_values(lambda x, z: 1.5 + 0.4 * z)
    c0 = np.full(d.n_dofs, 1.5)
    dt = 0.8 * solver.cfl_dt_gershgorin(d.stiffness(c_true), d.lumped_mass())
    src, rec = np.array([[0.5, 0.1]]), np.array([[0.2, 0.2], [0.8, 0.3], [0.5, 0.9]])
    sh = solver.Shot(d, src, rec, dt, nt, f0=8.0, t0=0.1)
    dobs, _ = sh.forward(c_true)
    J, g, tr = sh.misfit_gradient(c0, dobs)
    m = Mesh(coords, cells, k)
    p = dof_map(m.dof_coords(), d.dof_coords)
    say("serving: FP64 request vs oracle")
    srv = Server(max_slots=2)
    r = srv.result(srv.submit(m, c0[p], src, rec, dt, nt, precision="fp64", observed=dobs, f0=8.0, t0=0.1))
    srv.close()
    assert r["status"] == 0
    assert abs(r["J"] - J) < 1e-10 * J
    assert rel_l2(r["traces"], tr) < 1e-10
    assert rel_l2(r["grad"], g[p]) < 1e-10
    prob = Problem(m, dt, nt, precision="fp64")
    prob.set_sources(src, f0=8.0, t0=0.1)
    prob.set_receivers(rec)
    cuda = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    Jd, gd, trd = prob.misfit_gradient(cuda(c0[p]), cuda(dobs), keep_traces=True)
    assert Jd == r["J"]
    assert np.array_equal(gd.cpu().numpy(), r["grad"])
    assert np.array_equal(trd.cpu().numpy(), r["traces"])


def test_admission_by_memory():
    """With a budget that holds one request, requests run one after another and
    still give the same results."""
    from paper_2108_10946_amd import Server
    from paper_2108_10946_amd import kmvwave as K
    meshes, reqs = make_requests()
    reqs = [dict(q) for q in reqs if q["mesh"] is meshes["b"]][:3]
    for q in reqs:  # equal sizes: one request's reservation is every request's
        q["n_steps"] = 150
        q["precision"] = "fp32"
        if q["observed"] is not None:
            q["observed"] = q["observed"][:150]
    say("serving: memory-limited admission")
    srv = Server(max_slots=4)
    free = [srv.result(srv.submit(**q)) for q in reqs]
    srv.close()
    # a budget between one and two requests' reservations
    need = max(r["device_bytes"] for r in free)
    srv = Server(mem_budget=int(need * 1.5), max_slots=4)
    tickets = []
    for q in reqs:
        try:
            tickets.append(srv.submit(**q))
        except K.KMVError as e:
            assert e.code == K.KMV_ENOMEM
            tickets.append(None)
    res = [srv.result(t) if t is not None else None for t in tickets]
    srv.close()
    done = [(r["t_admit"], r["t_done"]) for r in res if r is not None]
    assert len(done) >= 1
    for a, b in zip(done, done[1:]):
        assert b[0] >= a[1] - 1e-6  # admitted only after the previous one finished
    for r0, r in zip(free, res):
        if r is not None:
            same(r0, r)


def test_bad_request_reports_error():
    from paper_2108_10946_amd import Server
    from paper_2108_10946_amd import kmvwave as K
    meshes, reqs = make_requests()
    q = dict(reqs[1])
    q["xr"] = np.array([[5.0, 5.0]])  # outside the mesh
    q["observed"] = None if q["forward_only"] else np.zeros((q["n_steps"], 1))
    say("serving: receiver outside the mesh")
    srv = Server(max_slots=2)
    r = srv.result(srv.submit(**q))
    assert r["status"] == K.KMV_EOUTSIDE
    assert "outside" in r["error"]
    # the server keeps working afterwards
    r2 = srv.result(srv.submit(**reqs[0]))
    assert r2["status"] == 0
    srv.close()
    with pytest.raises(ValueError):
        srv2 = Server(max_slots=1)
        try:
            srv2.submit(**{**reqs[1], "observed": np.zeros(3), "forward_only": False})
        finally:
            srv2.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_multi_shot_request(prec):
    """A request with three shots runs as one multi-shot problem: its traces are
    bitwise those of the three one-shot requests, J and the gradient their sums up
    to float64 rounding of the sum (1e-12 relative), and everything is bitwise what
    the multi-shot Problem call gives.  FP64 also matches the oracle (1e-10)."""
    from paper_2108_10946_amd import Mesh, Problem, Server
    from paper_2108_10946_amd import kmvwave as K
    coords, cells = configs.small_tri(8, seed=1)
    k, nt, nrec = 3, 200, 7
    d = Discretization(coords, cells, k)
    c_true = d.nodal_values(lambda x, z: 1.5 + 0.4 * z + 0.1 * np.sin(6 * x))
    c0 = d.nodal_values(lambda x, z: 1.5 + 0.4 * z)
    eta = d.nodal_values(lambda x, z: sponge_eta(x, z, 0.0, 1.0, 0.8, 0.2, c_max=2.5))
    dt = 0.8 * solver.cfl_dt_gershgorin(d.stiffness(c_true), d.lumped_mass())
    xs = np.array([[[0.25, 0.1]], [[0.5, 0.12]], [[0.75, 0.1]]])
    rec = np.stack([np.linspace(0.1, 0.9, nrec), np.full(nrec, 0.2)], axis=1)
    J_or, g_or, tr_or, obs = 0.0, np.zeros(d.n_dofs), [], []
    for s in range(3):
        sh = solver.Shot(d, xs[s], rec, dt, nt, f0=8.0, t0=0.1)
        dobs, _ = sh.forward(c_true, eta)
        J, g, tr = sh.misfit_gradient(c0, dobs, eta)
        J_or, g_or = J_or + J, g_or + g
        tr_or.append(tr)
        obs.append(dobs)
    obs = np.stack(obs)
    m = Mesh(coords, cells, k, patch_cells=13)
    p = dof_map(m.dof_coords(), d.dof_coords)
    q = dict(dt=dt, n_steps=nt, precision=prec, eta=eta[p], f0=8.0, t0=0.1)
    say(f"serving: three-shot request {prec}")
    srv = Server(max_slots=4)
    t_multi = srv.submit(m, c0[p], xs, rec, observed=obs, **q)
    t_single = [srv.submit(m, c0[p], xs[s], rec, observed=obs[s], **q) for s in range(3)]
    r = srv.result(t_multi)
    singles = [srv.result(t) for t in t_single]
    c_h, xs_h, xr_h = np.ascontiguousarray(c0[p]), np.ascontiguousarray(xs.reshape(-1, 2)), np.ascontiguousarray(rec)
    with pytest.raises(K.KMVError) as e:  # sources not a whole number per shot
        req = K.kmv_request(m.handle, K.KMV_FP64, dt, nt, K._dptr(c_h), None, K._dptr(xs_h), 3, 8.0, 0.1, 1.0,
                            K._dptr(xr_h), nrec, 1, None, 2)
        t = K.C.c_uint64()
        K._check(K.lib().kmv_server_submit(srv.handle, K.C.byref(req), K.C.byref(t)))
    assert e.value.code == K.KMV_EINVAL
    srv.close()
    assert r["status"] == 0 and r["n_shots"] == 3 and r["traces"].shape == (3, nt, nrec)
    for s in range(3):
        assert singles[s]["n_shots"] == 1
        assert np.array_equal(r["traces"][s], singles[s]["traces"])
    assert abs(r["J"] - sum(x["J"] for x in singles)) < 1e-12 * r["J"]
    assert rel_l2(r["grad"], sum(x["grad"] for x in singles)) < 1e-12
    prob = Problem(m, dt, nt, precision=prec, n_shots=3)
    prob.set_damping(eta[p])
    prob.set_sources(xs, f0=8.0, t0=0.1)
    prob.set_receivers(rec)
    Jd, gd, trd = prob.misfit_gradient(torch.as_tensor(c0[p], device="cuda"),
                                       torch.as_tensor(obs, dtype=prob.dtype, device="cuda"), keep_traces=True)
    prob.close()
    assert Jd == r["J"]
    assert np.array_equal(gd.cpu().numpy(), r["grad"])
    assert np.array_equal(trd.cpu().numpy(), r["traces"])
    if prec == "fp64":
        assert abs(r["J"] - J_or) < 1e-10 * J_or
        assert rel_l2(r["traces"], np.stack(tr_or)) < 1e-10
        assert rel_l2(r["grad"], g_or[p]) < 1e-10


def test_absorbing_request_matches_problem_api_and_oracle():
    """A request with the absorbing boundary on equals the Problem call with it on
    (bitwise) and the oracle (FP64, 1e-10); its memory estimate covers the records."""
    from paper_2108_10946_amd import Mesh, Problem, Server
    coords, cells = configs.small_tri(8, seed=1)
    k, nt = 2, 240
    d = Discretization(coords, cells, k)
    c_true = d.nodal_values(lambda x, z: 1.5 + 0.4 * z + 0.1 * np.sin(6 * x))
    c0 = d.nodal_values(lambda x, z: 1.5 + 0.4 * z)
    dt = 0.8 * solver.cfl_dt_gershgorin(d.stiffness(c_true), d.lumped_mass())
    src, rec = np.array([[0.5, 0.2]]), np.stack([np.linspace(0.1, 0.9, 6), np.full(6, 0.1)], axis=1)
    sh = solver.Shot(d, src, rec, dt, nt, f0=8.0, t0=0.1)
    dobs, _ = sh.forward(c_true, absorb=True)
    J, g, tr = sh.misfit_gradient(c0, dobs, absorb=True)
    m = Mesh(coords, cells, k)
    p = dof_map(m.dof_coords(), d.dof_coords)
    say("serving: absorbing-boundary request vs Problem and oracle")
    srv = Server(max_slots=2)
    t_on = srv.submit(m, c0[p], src, rec, dt, nt, precision="fp64", observed=dobs, f0=8.0, t0=0.1, absorbing=True)
    t_off = srv.submit(m, c0[p], src, rec, dt, nt, precision="fp64", observed=dobs, f0=8.0, t0=0.1)
    r, r_off = srv.result(t_on), srv.result(t_off)
    srv.close()
    assert r["status"] == 0 and r_off["status"] == 0
    assert r["device_bytes"] > r_off["device_bytes"]
    assert abs(r["J"] - J) < 1e-10 * J
    assert rel_l2(r["traces"], tr) < 1e-10
    assert rel_l2(r["grad"], g[p]) < 1e-10
    prob = Problem(m, dt, nt, precision="fp64")
    prob.set_absorbing_boundary(True)
    prob.set_sources(src, f0=8.0, t0=0.1)
    prob.set_receivers(rec)
    cuda = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")
    Jd, gd, trd = prob.misfit_gradient(cuda(c0[p]), cuda(dobs), keep_traces=True)
    prob.close()
    assert Jd == r["J"]
    assert np.array_equal(gd.cpu().numpy(), r["grad"])
    assert np.array_equal(trd.cpu().numpy(), r["traces"])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_request_with_per_shot_wavelets(prec):
    """A two-shot request whose shots fire different wavelets (Ricker pulses of other
    centre frequencies and a sign flip) equals the multi-shot Problem call given the
    same wavelets (bitwise), and in FP64 the oracle run shot by shot with each
    wavelet (1e-10 relative L2).  A wavelet array of the wrong size is refused."""
    from paper_2108_10946_amd import Mesh, Problem, Server
    coords, cells = configs.small_tri(8, seed=2)
    k, nt, nrec = 2, 220, 5
    d = Discretization(coords, cells, k)
    c_true = d.nodal_values(lambda x, z: 1.5 + 0.4 * z + 0.1 * np.sin(6 * x))
    c0 = d.nodal_values(lambda x, z: 1.5 + 0.4 * z)
    dt = 0.8 * solver.cfl_dt_gershgorin(d.stiffness(c_true), d.lumped_mass())
    t = np.arange(nt) * dt
    waves = np.stack([solver.ricker(t, 6.0, 0.15, 1.0), solver.ricker(t, 10.0, 0.1, -0.7)])
    xs = np.array([[[0.3, 0.1]], [[0.7, 0.15]]])
    rec = np.stack([np.linspace(0.1, 0.9, nrec), np.full(nrec, 0.2)], axis=1)
    J_or, g_or, tr_or, obs = 0.0, np.zeros(d.n_dofs), [], []
    for s in range(2):
        sh = solver.Shot(d, xs[s], rec, dt, nt, wavelet=waves[s])
        dobs, _ = sh.forward(c_true)
        J, g, tr = sh.misfit_gradient(c0, dobs)
        J_or, g_or = J_or + J, g_or + g
        tr_or.append(tr)
        obs.append(dobs)
    obs = np.stack(obs)
    m = Mesh(coords, cells, k)
    p = dof_map(m.dof_coords(), d.dof_coords)
    say(f"serving: two-shot request with per-shot wavelets {prec}")
    srv = Server(max_slots=2)
    tk = srv.submit(m, c0[p], xs, rec, dt, nt, precision=prec, observed=obs, wavelets=waves)
    r = srv.result(tk)
    with pytest.raises(ValueError):
        srv.submit(m, c0[p], xs, rec, dt, nt, precision=prec, observed=obs, wavelets=waves[0])
    srv.close()
    assert r["status"] == 0 and r["n_shots"] == 2
    prob = Problem(m, dt, nt, precision=prec, n_shots=2)
    prob.set_sources(xs, f0=8.0, t0=0.1)
    prob.set_source_wavelet(waves)
    prob.set_receivers(rec)
    Jd, gd, trd = prob.misfit_gradient(torch.as_tensor(c0[p], device="cuda"),
                                       torch.as_tensor(obs, dtype=prob.dtype, device="cuda"), keep_traces=True)
    prob.close()
    assert Jd == r["J"]
    assert np.array_equal(gd.cpu().numpy(), r["grad"])
    assert np.array_equal(trd.cpu().numpy(), r["traces"])
    if prec == "fp64":
        assert abs(r["J"] - J_or) < 1e-10 * J_or
        assert rel_l2(r["traces"], np.stack(tr_or)) < 1e-10
        assert rel_l2(r["grad"], g_or[p]) < 1e-10
    else:
        assert rel_l2(r["traces"], np.stack(tr_or)) < 1e-4
        assert rel_l2(r["grad"], g_or[p]) < 1e-3
