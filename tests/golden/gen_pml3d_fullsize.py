"""Writes tests/golden/pml3d_fullsize.json: the oracle's misfit, traces and sampled
gradient for the tetrahedral box of the 3D PML bench leg (KMV2 tetrahedra of edge
0.05 km: 112,896 cells, 502,145 DOFs; the 0.2 km layer on five faces as the paper's PML
with auxiliary p and omega, section 2.1; the transposed scheme of section 2.2 for the
adjoint) over a 150-step window at the leg's dt.

The shot and the receivers sit inside the layer of the x = 0 face, 0.1 km from its
inner edge, so the auxiliary fields and the damping terms shape the traces and the
gradient from the first steps.  The oracle at this size takes minutes, too long for a
test that holds the GPU, so its outputs are stored here and
tests/test_gpu_pml_fullsize.py compares the library's run with them.  Run from the
repository root:

    python tests/golden/gen_pml3d_fullsize.py

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

LE = 0.05
NT = 150
T0 = 0.03            # early wavelet delay: the window holds signal
SRC = [[-0.1, 0.5, 0.1]]
REC = np.stack([np.linspace(-0.18, 0.1, 12), np.full(12, 0.45), np.full(12, 0.15)], axis=1)
N_TOP, N_RAND = 200, 200  # gradient samples: the largest entries and a seeded random set


def current_model(vp_obs):
    """The current model: the observed one with a -10% bump between shot and receivers."""
    return lambda x, y, z: vp_obs(x, y, z) * (1.0 - 0.1 * np.exp(-((x + 0.05) ** 2 + (y - 0.48) ** 2
                                                                    + (z - 0.12) ** 2) / 0.004))


def main():
    t = time.time()
    w = configs.gradient_check_3d(le=LE)
    d = Discretization(w.coords, w.cells, w.degree)
    x = d.dof_coords
    sig = w.extra["sigma"](*x.T)
    c_obs = d.nodal_values(w.vp_obs)
    c0 = d.nodal_values(current_model(w.vp_obs))
    sh = solver.Shot(d, SRC, REC, w.dt, NT, f0=w.f0, t0=T0)
    dobs, _ = sh.forward(c_obs, pml=sig)
    J, g, tr = sh.misfit_gradient(c0, dobs, pml=sig)
    rng = np.random.default_rng(2108)
    top = np.argsort(-np.abs(g))[:N_TOP]
    live = np.flatnonzero(np.abs(g) > 1e-6 * np.abs(g).max())
    rand = rng.choice(np.setdiff1d(live, top), N_RAND, replace=False)
    idx = np.concatenate([top, rand])
    out = {
        "_source": "oracle (oracle/solver.py, oracle/pml.py) via tests/golden/gen_pml3d_fullsize.py; "
                   "the 3D PML bench leg's box (le = 0.05 km) with its layer as the PML",
        "le": LE, "n_dofs": int(d.n_dofs), "nt": NT, "dt": w.dt, "f0": w.f0, "t0": T0,
        "src": SRC, "rec": REC.tolist(),
        "J": float(J),
        "observed": dobs.tolist(),
        "traces": tr.tolist(),
        "grad_coords": x[idx].tolist(),
        "grad_values": g[idx].tolist(),
        "grad_norm": float(np.linalg.norm(g)),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pml3d_fullsize.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}: J = {J:.9e}, |g| = {np.linalg.norm(g):.3e} ({time.time() - t:.0f} s)")


if __name__ == "__main__":
    main()
