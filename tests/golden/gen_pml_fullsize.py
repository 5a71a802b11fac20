"""Writes tests/golden/pml_fullsize_c2.json: the oracle's misfit, traces and sampled
gradient for the layered KMV4 mesh at full size (150,022 triangles, 1.65 M DOFs) with
its 750 m layer as the paper's PML (section 2.1, the 2D PML system with auxiliary p;
the transposed scheme of section 2.2 for the adjoint), over a 200-step window.

The shot and the receivers sit inside the left layer, 300 m from its inner edge, where
sigma_x is about a sixth of its maximum, so the auxiliary field and the damping terms
shape the traces and the gradient from the first steps.  The oracle at this size takes a few
minutes, too long for a test that holds the GPU, so its outputs are stored here and
tests/test_gpu_pml_fullsize.py compares the library's run with them.  Run from the
repository root:

    python tests/golden/gen_pml_fullsize.py

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

NT = 200
DT = 2.8e-4          # below the power-iteration bound 3.19e-4 of the observed model
T0 = 0.02            # early wavelet delay: the window holds signal
SRC = [[-0.3, 0.01]]
REC = np.stack([np.linspace(-0.42, -0.18, 16), np.full(16, 0.03)], axis=1)
N_TOP, N_RAND = 200, 200  # gradient samples: the largest entries and a seeded random set


def current_model(vp_obs):
    """The current model: the observed one with a -10% bump between shot and receivers."""
    return lambda x, z: vp_obs(x, z) * (1.0 - 0.1 * np.exp(-((x + 0.3) ** 2 + (z - 0.04) ** 2) / 0.002))


def main():
    t = time.time()
    w = configs.layered_kmv4()
    d = Discretization(w.coords, w.cells, w.degree)
    x = d.dof_coords
    sig = w.extra["sigma"](*x.T)
    c_obs = d.nodal_values(w.vp_obs)
    c0 = d.nodal_values(current_model(w.vp_obs))
    sh = solver.Shot(d, SRC, REC, DT, NT, f0=w.f0, t0=T0)
    dobs, _ = sh.forward(c_obs, pml=sig)
    J, g, tr = sh.misfit_gradient(c0, dobs, pml=sig)
    rng = np.random.default_rng(2108)
    top = np.argsort(-np.abs(g))[:N_TOP]
    live = np.flatnonzero(np.abs(g) > 1e-6 * np.abs(g).max())
    rand = rng.choice(np.setdiff1d(live, top), N_RAND, replace=False)
    idx = np.concatenate([top, rand])
    out = {
        "_source": "oracle (oracle/solver.py, oracle/pml.py) via tests/golden/gen_pml_fullsize.py; "
                   "layered KMV4 workload at full size with its layer as the PML",
        "n_dofs": int(d.n_dofs), "nt": NT, "dt": DT, "f0": w.f0, "t0": T0,
        "src": SRC, "rec": REC.tolist(),
        "J": float(J),
        "observed": dobs.tolist(),
        "traces": tr.tolist(),
        "grad_coords": x[idx].tolist(),
        "grad_values": g[idx].tolist(),
        "grad_norm": float(np.linalg.norm(g)),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pml_fullsize_c2.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}: J = {J:.9e}, |g| = {np.linalg.norm(g):.3e} ({time.time() - t:.0f} s)")


if __name__ == "__main__":
    main()
