"""The misfit as a torch.autograd.Function (FWIMisfit): J(c) and dJ/dc through the
C ABI, checked against torch.autograd.gradcheck, central finite differences along
a smooth seeded direction, and the multi-shot sum.

The gradient is the exact derivative of the discrete misfit (the discrete adjoint
of the leapfrog recursion), so central differences converge to it as O(h^2):
FP64 relative error <= 1e-6 at h = 3e-4 km/s (the O(h^2) term is ~7e-7 at
h = 1e-3 here); FP32 fields with float64 accumulation <= 1e-2 at h = 1e-3."""
import numpy as np
import pytest

from gpu_util import say, rel_l2
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


def shots(prec, n_shots=3, n=8, k=3, nt=240):
    """A small sponge-damped problem with several surface shots; observed data from a
    model with a smooth bump, current model without it."""
    from paper_2108_10946_amd import Mesh, Problem
    coords, cells = configs.small_tri(n, seed=2)
    m = Mesh(coords, cells, k)
    x = m.dof_coords()
    c_true = 1.5 + 0.6 * x[:, 1] + 0.2 * np.exp(-((x[:, 0] - 0.5) ** 2 + (x[:, 1] - 0.5) ** 2) / 0.02)
    c0 = 1.5 + 0.6 * x[:, 1]
    eta = sponge_eta(x[:, 0], x[:, 1], 0.0, 1.0, 0.8, 0.2, c_max=2.5)
    dt = 0.5 * m.cfl_dt(c_true)
    rec = np.stack([np.linspace(0.1, 0.9, 15), np.full(15, 0.12)], axis=1)
    probs, obs = [], []
    for xs in np.linspace(0.2, 0.8, n_shots):
        p = Problem(m, dt, nt, precision=prec)
        p.set_damping(eta)
        p.set_sources([[xs, 0.05]], f0=8.0, t0=0.1)
        p.set_receivers(rec)
        ct = torch.as_tensor(c_true, dtype=torch.float64, device="cuda")
        obs.append(p.forward(ct))
        probs.append(p)
    return m, x, c0, probs, obs


def direction(x, seed=3):
    """Seeded sum of five Gaussians, max |d| = 1, zero in the sponge."""
    rng = np.random.default_rng(seed)
    d = np.zeros(len(x))
    for _ in range(5):
        cx, cz = rng.uniform(0.15, 0.85, 2)
        d += rng.choice([-1.0, 1.0]) * np.exp(-((x[:, 0] - cx) ** 2 + (x[:, 1] - cz) ** 2) / 0.01)
    d[(x[:, 0] < 0.0) | (x[:, 0] > 1.0) | (x[:, 1] > 0.8)] = 0.0
    return d / np.abs(d).max()


@pytest.mark.parametrize("prec,h,tol", [("fp64", 3e-4, 1e-6), ("fp32", 1e-3, 1e-2)])
def test_central_differences(prec, h, tol):
    from paper_2108_10946_amd import fwi_misfit
    say(f"autograd: central differences {prec}")
    m, x, c0, probs, obs = shots(prec)
    c = torch.as_tensor(c0, dtype=torch.float64, device="cuda").requires_grad_(True)
    J = fwi_misfit(c, probs, obs)
    J.backward()
    g = c.grad.cpu().numpy()
    d = direction(x)
    cp = torch.as_tensor(c0 + h * d, dtype=torch.float64, device="cuda")
    cm = torch.as_tensor(c0 - h * d, dtype=torch.float64, device="cuda")
    fd = (float(fwi_misfit(cp, probs, obs)) - float(fwi_misfit(cm, probs, obs))) / (2 * h)
    an = float(g @ d)
    say(f"  J={float(J.detach()):.6e} fd={fd:.9e} an={an:.9e} rel={abs(fd - an) / abs(an):.2e}")
    assert abs(an) > 0
    assert abs(fd - an) <= tol * abs(an)


def test_multi_shot_sum_and_backward_scaling():
    """J and dJ/dc of several shots are the sums of the single-shot values, and
    backward scales by the incoming gradient."""
    from paper_2108_10946_amd import fwi_misfit
    say("autograd: multi-shot sum")
    m, x, c0, probs, obs = shots("fp64")
    c = torch.as_tensor(c0, dtype=torch.float64, device="cuda")
    Js, gs = [], []
    for p, o in zip(probs, obs):
        J, g, _ = p.misfit_gradient(c, o)
        Js.append(J)
        gs.append(g.cpu().numpy())
    cc = c.clone().requires_grad_(True)
    J = fwi_misfit(cc, probs, obs)
    (3.0 * J).backward()
    assert abs(float(J.detach()) - sum(Js)) <= 1e-12 * abs(sum(Js))
    assert rel_l2(cc.grad.cpu().numpy(), 3.0 * np.sum(gs, axis=0)) < 1e-13


def test_gradcheck():
    """torch.autograd.gradcheck (fast mode) of J(c) on a tiny FP64 problem."""
    from paper_2108_10946_amd import fwi_misfit
    say("autograd: gradcheck")
    m, x, c0, probs, obs = shots("fp64", n_shots=1, n=5, k=2, nt=120)
    c = torch.as_tensor(c0, dtype=torch.float64, device="cuda").requires_grad_(True)
    f = lambda cc: fwi_misfit(cc, probs, obs)
    assert torch.autograd.gradcheck(f, (c,), eps=1e-6, atol=1e-8, rtol=1e-4, fast_mode=True)


def test_zero_misfit_at_true_model():
    from paper_2108_10946_amd import fwi_misfit
    from paper_2108_10946_amd import Problem
    say("autograd: J(c_true) = 0")
    m, x, c0, probs, obs = shots("fp64", n_shots=1)
    c_true = 1.5 + 0.6 * x[:, 1] + 0.2 * np.exp(-((x[:, 0] - 0.5) ** 2 + (x[:, 1] - 0.5) ** 2) / 0.02)
    ct = torch.as_tensor(c_true, dtype=torch.float64, device="cuda").requires_grad_(True)
    J = fwi_misfit(ct, probs, obs)
    J.backward()
    assert float(J) == 0.0
    assert float(ct.grad.abs().max()) == 0.0
