"""Writes tests/golden/shots_fullsize_c2.json: the oracle's per-shot misfits, sampled
traces and summed gradient for eight shots of the 40-shot line of the layered KMV4
workload at full size (150,022 triangles, 1.65 M DOFs, its sponge), over a 200-step
window: the paper's independent per-shot wave equations, whose misfits and gradients are
summed (section 2.2).

The shots are the line's 17th to 24th (x_s = linspace(0.1, 7.9, 40), 10 m deep), one
problem of eight as the 40-shot leg of bench.py runs them, and the 16 receivers sit 20 m
deep along them.  The oracle at this size takes minutes, too long for a test that holds
the GPU, so its outputs are stored here (traces every 5th step) and
tests/test_gpu_fullsize.py compares the library's run with them.  Run from the
repository root:

    python tests/golden/gen_shots_fullsize.py

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
SHOTS = np.linspace(0.1, 7.9, 40)[16:24]
REC = np.stack([np.linspace(SHOTS[0] - 0.05, SHOTS[-1] + 0.05, 16), np.full(16, 0.02)], axis=1)
ROW_STEP = 5         # traces stored every 5th step
N_TOP, N_RAND = 200, 200  # gradient samples: the largest entries and a seeded random set


def current_model(vp_obs):
    """The current model: the observed one with -10% bumps beside every shot."""
    def c(x, z):
        bumps = sum(np.exp(-((x - xs - 0.03) ** 2 + (z - 0.03) ** 2) / 0.002) for xs in SHOTS)
        return vp_obs(x, z) * (1.0 - 0.1 * bumps)
    return c


def main():
    t = time.time()
    w = configs.layered_kmv4()
    d = Discretization(w.coords, w.cells, w.degree)
    eta = d.nodal_values(w.eta)
    c_obs = d.nodal_values(w.vp_obs)
    c0 = d.nodal_values(current_model(w.vp_obs))
    Js, obs_rows, tr_rows, g = [], [], [], np.zeros(d.n_dofs)
    for xs in SHOTS:
        sh = solver.Shot(d, [[xs, 0.01]], REC, DT, NT, f0=w.f0, t0=T0)
        dobs, _ = sh.forward(c_obs, eta)
        J, gs, tr = sh.misfit_gradient(c0, dobs, eta)
        Js.append(float(J))
        g += gs
        obs_rows.append(dobs[ROW_STEP - 1::ROW_STEP].tolist())
        tr_rows.append(tr[ROW_STEP - 1::ROW_STEP].tolist())
        print(f"shot x = {xs:.3f}: J = {J:.6e} ({time.time() - t:.0f} s)", flush=True)
    rng = np.random.default_rng(2108)
    top = np.argsort(-np.abs(g))[:N_TOP]
    live = np.flatnonzero(np.abs(g) > 1e-6 * np.abs(g).max())
    rand = rng.choice(np.setdiff1d(live, top), N_RAND, replace=False)
    idx = np.concatenate([top, rand])
    x = d.dof_coords
    out = {
        "_source": "oracle (oracle/solver.py, oracle/fem.py) via tests/golden/gen_shots_fullsize.py; "
                   "eight shots of the layered KMV4 workload's 40-shot line at full size",
        "n_dofs": int(d.n_dofs), "nt": NT, "dt": DT, "f0": w.f0, "t0": T0, "row_step": ROW_STEP,
        "shots": [[[float(xs), 0.01]] for xs in SHOTS], "rec": REC.tolist(),
        "J_per_shot": Js,
        "observed_rows": obs_rows,
        "traces_rows": tr_rows,
        "grad_coords": x[idx].tolist(),
        "grad_values": g[idx].tolist(),
        "grad_norm": float(np.linalg.norm(g)),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "shots_fullsize_c2.json")
    with open(path, "w") as f:
        json.dump(out, f)
    print(f"wrote {path}: J = {sum(Js):.9e}, |g| = {np.linalg.norm(g):.3e} ({time.time() - t:.0f} s)")


if __name__ == "__main__":
    main()
