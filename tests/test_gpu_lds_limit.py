"""The step kernels' dynamic-LDS limit is a property of the kernel function, shared by
every problem on the device.  A problem created later with a smaller footprint (above
the 64 KiB default) must not lower it under an earlier problem's launches: the earlier
problem keeps running, bitwise as before.  FP64 PML instances on KMV4 triangles, whose
footprint exceeds 64 KiB on patches of a hundred cells and more."""
import numpy as np
import pytest

from gpu_util import say
from synth import configs
from synth.models import pml_sigma

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_10946_amd as kmv
    kmv.lib()


def make(coords, cells, patch, nt=150):
    from paper_2108_10946_amd import Mesh, Problem
    from paper_2108_10946_amd import kmvwave as K
    m = Mesh(coords, cells, 4, patch_cells=patch)
    x = m.dof_coords()
    c = 1.5 + 0.5 * x[:, 1]
    dt = 0.4 * m.cfl_dt(c)
    prob = Problem(m, dt, nt, precision="fp64")
    try:
        prob.set_pml(pml_sigma(x[:, 0], x[:, 1], 0.2, 0.8, 0.8, 0.2, c_max=2.0))
    except K.KMVError as e:
        prob.close()
        if e.code == K.KMV_EINVAL and "LDS" in str(e):
            return None
        raise
    prob.set_sources([[0.5, 0.3]], f0=6.0, t0=0.02)
    prob.set_receivers([[0.4, 0.25], [0.6, 0.35], [0.5, 0.45]])
    c_t = torch.as_tensor(c, device="cuda")
    obs = prob.forward(c_t * 1.05)
    return prob, c_t, obs, m


def test_smaller_footprint_does_not_lower_the_limit():
    coords, cells = configs.small_tri(24, seed=31)
    a = None
    for patch in (176, 160, 144, 128):
        a = make(coords, cells, patch)
        if a is not None:
            break
    assert a is not None
    prob_a, c_a, obs_a, _ = a
    J1 = prob_a.misfit(c_a, obs_a)
    b = make(coords, cells, patch - 48)
    assert b is not None
    prob_b, c_b, obs_b, _ = b
    Jb = prob_b.misfit(c_b, obs_b)
    J2 = prob_a.misfit(c_a, obs_a)
    say(f"patches {patch} then {patch - 48}: J {J1:.15e} / {J2:.15e} (other {Jb:.6e})")
    assert J1 > 1e-12 and J2 == J1 and Jb > 1e-12
    prob_a.close()
    prob_b.close()
