"""The PML at full size against oracle outputs stored by committed generators.

Triangles: the layered KMV4 workload (150,022 triangles, 1.65 M DOFs) with its 750 m
layer as the PML, tests/golden/gen_pml_fullsize.py (a 200-step window with the shot and
receivers inside the left layer).  FP32 runs in the
launch configuration bench.py times (default 224-cell patches: the PML instance on the
patches that touch the layer, the plain one on the rest); FP64 doubles the PML
instance's LDS, which refuses 224-cell patches (KMV_EINVAL), so it runs on 112-cell
patches.  Checked: the forward traces of the observed model, and J, traces and the
gradient at 400 sampled DOFs of the current model; FP64 1e-10 relative L2; FP32 1e-4 on
traces, 1e-3 on the sampled gradient, and J within the bound the traces' tolerance
implies, |dJ| <= 1e-4 |r| |d|.

Tetrahedra: the box of the 3D PML bench leg (112,896 KMV2 tetrahedra, 502,145 DOFs, the
0.2 km layer on five faces), tests/golden/gen_pml3d_fullsize.py (a 150-step window with
the shot and receivers inside the layer of the x = 0 face), default patches, both
precisions, the same checks and tolerances."""
import importlib.util
import json
import os

import numpy as np
import pytest

from gpu_util import say, rel_l2
from synth import configs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_10946_amd as kmv
    kmv.lib()


@pytest.fixture(scope="module")
def case():
    spec = importlib.util.spec_from_file_location("gen_pml_fullsize", os.path.join(GOLDEN, "gen_pml_fullsize.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    with open(os.path.join(GOLDEN, "pml_fullsize_c2.json")) as f:
        ref = json.load(f)
    w = configs.layered_kmv4()
    return dict(w=w, ref=ref, gen=gen, meshes={})


def mesh(case, patch):
    from scipy.spatial import cKDTree
    from paper_2108_10946_amd import Mesh
    if patch not in case["meshes"]:
        w, ref = case["w"], case["ref"]
        say(f"pml full size: layered KMV4 mesh, patch_cells={patch}")
        m = Mesh(w.coords, w.cells, w.degree, patch_cells=patch)
        assert m.n_dofs == ref["n_dofs"]
        x = m.dof_coords()
        dist, idx = cKDTree(x).query(np.array(ref["grad_coords"]))
        assert dist.max() < 1e-9
        case["meshes"][patch] = (m, x, idx, case["gen"].current_model(w.vp_obs)(*x.T))
    return case["meshes"][patch]


def cuda(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


@pytest.mark.parametrize("prec,patch", [("fp64", 112), ("fp32", 0)])
def test_pml_full_size_vs_oracle(case, prec, patch):
    from paper_2108_10946_amd import Problem
    w, ref = case["w"], case["ref"]
    m, x, idx, c0 = mesh(case, patch)
    say(f"pml full size: {prec}, {m.n_patches} patches, {ref['nt']} steps")
    prob = Problem(m, ref["dt"], ref["nt"], precision=prec)
    prob.set_pml(w.extra["sigma"](*x.T))
    prob.set_sources(ref["src"], f0=ref["f0"], t0=ref["t0"])
    prob.set_receivers(ref["rec"])
    obs_or, tr_or = np.array(ref["observed"]), np.array(ref["traces"])
    d = prob.forward(cuda(w.vp_obs(*x.T))).double().cpu().numpy()
    J, g, tr = prob.misfit_gradient(cuda(c0), cuda(obs_or, prob.dtype), keep_traces=True)
    prob.status()
    prob.close()
    J_or, g_or = ref["J"], np.array(ref["grad_values"])
    ed, et = rel_l2(d, obs_or), rel_l2(tr.double().cpu().numpy(), tr_or)
    eg = rel_l2(g.cpu().numpy()[idx], g_or)
    say(f"  forward {ed:.2e}  J {J:.9e} (oracle {J_or:.9e})  traces {et:.2e}  sampled gradient {eg:.2e}")
    if prec == "fp64":
        assert ed < 1e-10 and et < 1e-10 and eg < 1e-10
        assert abs(J - J_or) < 1e-10 * J_or
    else:
        assert ed < 1e-4 and et < 1e-4 and eg < 1e-3
        assert abs(J - J_or) <= 1e-4 * np.sqrt(2 * J_or) * np.linalg.norm(tr_or)


def test_pml_full_size_fp64_default_patches_refused(case):
    """The FP64 PML instance needs more than the 160 KiB of LDS on 224-cell patches:
    set_pml refuses them before any work."""
    from paper_2108_10946_amd import Problem
    from paper_2108_10946_amd import kmvwave as K
    m, x, _, _ = mesh(case, 0)
    prob = Problem(m, case["ref"]["dt"], 4, precision="fp64")
    with pytest.raises(K.KMVError) as e:
        prob.set_pml(case["w"].extra["sigma"](*x.T))
    assert e.value.code == K.KMV_EINVAL and "LDS" in str(e.value)
    prob.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_pml3d_full_size_vs_oracle(prec):
    from scipy.spatial import cKDTree
    from paper_2108_10946_amd import Mesh, Problem
    spec = importlib.util.spec_from_file_location("gen_pml3d_fullsize", os.path.join(GOLDEN, "gen_pml3d_fullsize.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    with open(os.path.join(GOLDEN, "pml3d_fullsize.json")) as f:
        ref = json.load(f)
    w = configs.gradient_check_3d(le=ref["le"])
    m = Mesh(w.coords, w.cells, w.degree)
    assert m.n_dofs == ref["n_dofs"]
    x = m.dof_coords()
    dist, idx = cKDTree(x).query(np.array(ref["grad_coords"]))
    assert dist.max() < 1e-9
    say(f"pml 3d full size: {prec}, {m.n_dofs} DOFs, {ref['nt']} steps")
    prob = Problem(m, ref["dt"], ref["nt"], precision=prec)
    prob.set_pml(w.extra["sigma"](*x.T))
    prob.set_sources(ref["src"], f0=ref["f0"], t0=ref["t0"])
    prob.set_receivers(ref["rec"])
    obs_or, tr_or = np.array(ref["observed"]), np.array(ref["traces"])
    d = prob.forward(cuda(w.vp_obs(*x.T))).double().cpu().numpy()
    c0 = gen.current_model(w.vp_obs)(*x.T)
    J, g, tr = prob.misfit_gradient(cuda(c0), cuda(obs_or, prob.dtype), keep_traces=True)
    prob.status()
    prob.close()
    m.close()
    J_or, g_or = ref["J"], np.array(ref["grad_values"])
    ed, et = rel_l2(d, obs_or), rel_l2(tr.double().cpu().numpy(), tr_or)
    eg = rel_l2(g.cpu().numpy()[idx], g_or)
    say(f"  forward {ed:.2e}  J {J:.9e} (oracle {J_or:.9e})  traces {et:.2e}  sampled gradient {eg:.2e}")
    if prec == "fp64":
        assert ed < 1e-10 and et < 1e-10 and eg < 1e-10
        assert abs(J - J_or) < 1e-10 * J_or
    else:
        assert ed < 1e-4 and et < 1e-4 and eg < 1e-3
        assert abs(J - J_or) <= 1e-4 * np.sqrt(2 * J_or) * np.linalg.norm(tr_or)
