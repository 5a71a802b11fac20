"""kmv_forward_noalloc (the forward sweep with its level buffers in the library's
static per-device workspace) against kmv_forward, through the C ABI: the traces
are bitwise equal, on two calls in a row, the second on a smaller problem (other
mesh, other degree, fewer steps, other shot count), so that it runs over what the
first left in the workspace; FP64 and FP32.  A problem whose two levels exceed the
workspace is refused before any work."""
import numpy as np
import pytest

from gpu_util import say
from synth import configs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2108_10946_amd as kmv
    kmv.lib()


def make(n, k, nt, prec, n_shots, seed):
    from paper_2108_10946_amd import Mesh, Problem
    from synth.models import sponge_eta
    coords, cells = configs.small_tri(n, seed=seed)
    m = Mesh(coords, cells, k)
    x = m.dof_coords()
    c = torch.as_tensor(1.5 + 0.4 * x[:, 1] + 0.1 * np.sin(5 * x[:, 0]), dtype=torch.float64, device="cuda")
    dt = 0.8 * m.cfl_dt(c.cpu().numpy())
    p = Problem(m, dt, nt, precision=prec, n_shots=n_shots)
    p.set_damping(sponge_eta(x[:, 0], x[:, 1], 0.0, 1.0, 0.8, 0.2, c_max=2.0))
    xs = np.array([[[0.2 + 0.6 * s / max(1, n_shots - 1), 0.15]] for s in range(n_shots)])
    p.set_sources(xs if n_shots > 1 else xs[0], f0=8.0, t0=0.1)
    p.set_receivers(np.stack([np.linspace(0.1, 0.9, 7), np.full(7, 0.3)], axis=1))
    return m, p, c


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_forward_equals_forward(prec):
    from paper_2108_10946_amd import kmvwave as K
    cases = [(12, 4, 300, 3, 5), (6, 2, 120, 1, 6)]  # the second call is the smaller problem
    for n, k, nt, shots, seed in cases:
        say(f"no-alloc forward: tri n={n} k={k} nt={nt} shots={shots} {prec}")
        m, p, c = make(n, k, nt, prec, shots, seed)
        ref = p.forward(c)
        out = torch.full_like(ref, float("nan"))
        K.kmv_forward_noalloc(p.handle, c, out)
        p.status()
        torch.cuda.synchronize()
        assert torch.isfinite(ref).all() and float(ref.abs().max()) > 0
        assert torch.equal(out, ref), float((out - ref).abs().max())
        p.close()


def test_noalloc_forward_refuses_oversize():
    from paper_2108_10946_amd import kmvwave as K
    m, p, c = make(24, 5, 10, "fp64", 1, 7)
    x = m.dof_coords()
    shots = int(np.ceil((64 << 20) / (2 * 8 * m.n_dofs))) + 1  # 2 levels x shots x n_dofs doubles > 64 MiB
    from paper_2108_10946_amd import Problem
    big = Problem(m, p.dt, 10, precision="fp64", n_shots=shots)
    big.set_sources(np.tile(np.array([[[0.5, 0.5]]]), (shots, 1, 1)), f0=8.0, t0=0.1)
    big.set_receivers([[0.5, 0.3]])
    tr = torch.empty((shots, 10, 1), dtype=torch.float64, device="cuda")
    say(f"no-alloc forward: oversize ({shots} shots) is refused")
    with pytest.raises(K.KMVError) as e:
        K.kmv_forward_noalloc(big.handle, c, tr)
    assert e.value.code == K.KMV_EINVAL and "workspace" in str(e.value)
    big.close()
    p.close()
