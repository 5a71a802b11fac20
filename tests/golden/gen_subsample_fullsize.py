"""Writes tests/golden/subsample_fullsize_c2.json: the oracle's misfit, traces and
sampled gradient for the layered KMV4 mesh at full size (150,022 triangles, 1.65 M DOFs)
with its sponge, over a 300-step window, with the paper's gradient subsampling at r = 10
(the section on gradient subsampling: the pairing of the adjoint with the forward states
at every 10th step only, the sum scaled by 10), as the subsampling leg of bench.py runs
it.  The oracle at this size takes minutes, too long for a test that holds the GPU, so
its outputs are stored here and tests/test_gpu_fullsize.py compares the library's run
with them.  Run from the repository root:

    python tests/golden/gen_subsample_fullsize.py

Calls only oracle/ (and synth/ for the seeded mesh and model)."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import solver  # noqa: E402
from oracle.fem import Discretization  # noqa: E402
from synth import configs  # noqa: E402

NT = 300
DT = 2.8e-4          # below the power-iteration bound 3.19e-4 of the observed model
T0 = 0.02            # early wavelet delay: the window holds signal
R = 10
SRC = [[4.0, 0.01]]
REC = np.stack([np.linspace(3.85, 4.15, 16), np.full(16, 0.02)], axis=1)
N_TOP, N_RAND = 200, 200  # gradient samples: the largest entries and a seeded random set


def current_model(vp_obs):
    """The current model: the observed one with a -10% bump beside the shot."""
    return lambda x, z: vp_obs(x, z) * (1.0 - 0.1 * np.exp(-((x - 4.05) ** 2 + (z - 0.03) ** 2) / 0.002))


def main():
    t = time.time()
    w = configs.layered_kmv4()
    d = Discretization(w.coords, w.cells, w.degree)
    eta = d.nodal_values(w.eta)
    c_obs = d.nodal_values(w.vp_obs)
    c0 = d.nodal_values(current_model(w.vp_obs))
    sh = solver.Shot(d, SRC, REC, DT, NT, f0=w.f0, t0=T0)
    dobs, _ = sh.forward(c_obs, eta)
    J, g, tr = sh.misfit_gradient(c0, dobs, eta, r=R)
    rng = np.random.default_rng(2108)
    top = np.argsort(-np.abs(g))[:N_TOP]
    live = np.flatnonzero(np.abs(g) > 1e-6 * np.abs(g).max())
    rand = rng.choice(np.setdiff1d(live, top), N_RAND, replace=False)
    idx = np.concatenate([top, rand])
    x = d.dof_coords
    out = {
        "_source": "oracle (oracle/solver.py, oracle/fem.py) via tests/golden/gen_subsample_fullsize.py; "
                   "layered KMV4 workload at full size, sponge, gradient subsampling r = 10",
        "n_dofs": int(d.n_dofs), "r": R, "nt": NT, "dt": DT, "f0": w.f0, "t0": T0,
        "src": SRC, "rec": REC.tolist(),
        "J": float(J),
        "observed": dobs.tolist(),
        "traces": tr.tolist(),
        "grad_coords": x[idx].tolist(),
        "grad_values": g[idx].tolist(),
        "grad_norm": float(np.linalg.norm(g)),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "subsample_fullsize_c2.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}: J = {J:.9e}, |g| = {np.linalg.norm(g):.3e} ({time.time() - t:.0f} s)")


if __name__ == "__main__":
    main()
