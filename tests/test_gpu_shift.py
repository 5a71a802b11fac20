"""Time-shift invariance, with no oracle in between: the recursion starts from rest,
so delaying the source wavelet by s steps delays the traces by s rows, and a problem
whose window is longer by s steps, with the observed data delayed the same way, has the
same gradient (the extra reverse steps pair lambda with the resting states u = 0, which
add exact zeros to the float64 accumulators).  All of it is the same arithmetic on the
same values at other step indices, so the traces and the gradient must match bitwise,
under every storage plan (all states kept, checkpoints of 5 steps, sqrt(2 N_t)
segments), in FP64 and FP32, in 2D and 3D.  J is reduced over the rows in blocks that
the extra rows shift, so it is held to 1e-14."""
import numpy as np
import pytest

from gpu_util import say
from synth import configs
from synth.models import sponge_eta, sponge_eta_3d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NT, SHIFT = 90, 13


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_10946_amd as kmv
    kmv.lib()


def setup(kind):
    from paper_2108_10946_amd import Mesh
    if kind == "tri":
        coords, cells = configs.small_tri(9, seed=5)
        m = Mesh(coords, cells, 3, patch_cells=17)
        x = m.dof_coords()
        c = 1.5 + 0.8 * x[:, 1]
        eta = sponge_eta(x[:, 0], x[:, 1], 0.15, 0.85, 0.85, 0.15, c_max=2.3)
        src, rec = [[0.45, 0.3]], [[0.2, 0.5], [0.7, 0.6], [0.5, 0.8]]
    else:
        coords, cells = configs.small_tet(3, seed=5)
        m = Mesh(coords, cells, 2, patch_cells=9)
        x = m.dof_coords()
        c = 1.5 + 0.8 * x[:, 2]
        eta = sponge_eta_3d(x[:, 0], x[:, 1], x[:, 2], (0.15, 0.15), (0.85, 0.85, 0.85), 0.15, c_max=2.3)
        src, rec = [[0.45, 0.3, 0.4]], [[0.2, 0.5, 0.5], [0.7, 0.6, 0.3]]
    return m, c, eta, src, rec, 0.5 * m.cfl_dt(c)


@pytest.mark.parametrize("kind", ["tri", "tet"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("ckpt", [0, 5, -1])
def test_time_shift(kind, prec, ckpt):
    from paper_2108_10946_amd import Problem
    m, c, eta, src, rec, dt = setup(kind)
    say(f"time shift: {kind} {prec} checkpoint_every={ckpt}")
    rng = np.random.default_rng(17)
    wav = rng.standard_normal(NT)
    cc = torch.as_tensor(c, device="cuda")
    c0 = torch.as_tensor(c * 0.95, device="cuda")

    def run(nt, w, obs=None):
        prob = Problem(m, dt, nt, precision=prec, checkpoint_every=ckpt)
        prob.set_damping(eta)
        prob.set_sources(src, f0=8.0, t0=0.1)
        prob.set_source_wavelet(w)
        prob.set_receivers(rec)
        tr = prob.forward(cc)
        out = (tr,) if obs is None else (tr,) + tuple(prob.misfit_gradient(c0, obs))
        prob.close()
        return out

    (d1,) = run(NT, wav)
    (d2,) = run(NT + SHIFT, np.concatenate([np.zeros(SHIFT), wav]))
    assert torch.equal(d2[SHIFT:], d1) and not d2[:SHIFT].any()
    _, J1, g1, _ = run(NT, wav, d1)
    _, J2, g2, _ = run(NT + SHIFT, np.concatenate([np.zeros(SHIFT), wav]), d2)
    say(f"  J {J1:.15e} / {J2:.15e}")
    assert J1 > 0 and abs(J1 - J2) <= 1e-14 * J1
    assert torch.equal(g1, g2)
