"""Writes tests/golden/apply3d_fullsize.json: rows of the stiffness apply y = K(c) u
(the appendix's stiffness matrix with the KMV rule as the quadrature, section 3.3) of
the 3D workload at full size (1.33 M KMV3 tetrahedra, 16.9 M DOFs), at sampled DOFs of
every node class: vertices, edge nodes, face nodes and cell-interior nodes.

The oracle cannot assemble the operator at this size, but row i of K u involves only
the cells that hold DOF i.  So for each sampled entity (a vertex, an edge, a face or a
cell) the cells holding all of its vertices are gathered; the oracle discretises the
union of those cells, and the rows of its DOFs that lie on the sampled entities are
complete rows of the full operator.  The wave speed is the workload's model and u an
oscillating function, both evaluated at the DOF coordinates, so the test can rebuild
them on the library's numbering.  Run from the repository root:

    python tests/golden/gen_apply3d_fullsize.py

Calls only oracle/ (and synth/ for the seeded mesh and model)."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.fem import Discretization  # noqa: E402
from synth import configs  # noqa: E402

N_SAMPLE = {1: 80, 2: 80, 3: 80, 4: 40}  # entities per number of vertices


def u_field(x, y, z):
    """A field that oscillates on the scale of the cells (wavelengths of 60-120 m), so
    that K u has no more cancellation than with random data: sum_j |K_ij u_j| is about
    3x |(K u)_i| in the L2 sense, against about 1000x for a field smooth on the scale
    of the domain, which would amplify FP32 rounding by as much."""
    return (np.sin(97.0 * x + 1.0) * np.cos(89.0 * y - 2.0) * np.sin(83.0 * z + 0.5)
            + np.cos(61.0 * x - 53.0 * z + 0.7))


def main():
    t = time.time()
    w = configs.layered_tet_kmv3()
    cells = np.asarray(w.cells, dtype=np.int64)
    rng = np.random.default_rng(2108)
    # sampled entities: vertex sets of size 1 (vertex), 2 (edge), 3 (face), 4 (cell)
    picked = rng.choice(len(cells), sum(N_SAMPLE.values()), replace=False)
    entities, k = [], 0
    for size, count in N_SAMPLE.items():
        for e in picked[k:k + count]:
            entities.append(tuple(sorted(rng.choice(cells[e], size, replace=False).tolist())))
        k += count
    # the cells holding every vertex of some entity
    member = {}
    for v in {v for ent in entities for v in ent}:
        member[v] = set()
    for e, cell in enumerate(cells):
        for v in cell:
            if v in member:
                member[v].add(e)
    sub = sorted(set().union(*(set.intersection(*(member[v] for v in ent)) for ent in entities)))
    sub_cells = cells[sub]
    verts, local = np.unique(sub_cells, return_inverse=True)
    d = Discretization(w.coords[verts], local.reshape(sub_cells.shape), w.degree)
    x = d.dof_coords
    y = d.stiffness(w.vp(*x.T)) @ u_field(*x.T)
    # the DOFs that lie on a sampled entity: node q of cell e lies on the sub-simplex of
    # the local vertices with a nonzero barycentric coordinate
    xi = d.elem.nodes
    lam = np.concatenate([1.0 - xi.sum(axis=1, keepdims=True), xi], axis=1)
    wanted = set(entities)
    rows = {}
    for e in range(d.n_cells):
        gv = verts[local.reshape(sub_cells.shape)[e]]
        for q in range(d.elem.n_d):
            ent = tuple(sorted(gv[lam[q] > 1e-12].tolist()))
            if ent in wanted:
                rows[int(d.cell_dofs[e, q])] = len(ent)
    idx = np.array(sorted(rows))
    out = {
        "_source": "oracle (oracle/fem.py) via tests/golden/gen_apply3d_fullsize.py; rows of K(c) u of the "
                   "3D KMV3 workload at full size, c = its model, u = u_field of the script",
        "n_cells": int(len(cells)), "n_sub_cells": int(len(sub)),
        "coords": x[idx].tolist(),
        "node_class": [rows[i] for i in idx],
        "y": y[idx].tolist(),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "apply3d_fullsize.json")
    with open(path, "w") as f:
        json.dump(out, f)
    counts = {s: sum(1 for i in idx if rows[i] == s) for s in N_SAMPLE}
    print(f"wrote {path}: {len(idx)} rows {counts} from {len(sub)} cells ({time.time() - t:.0f} s)")


if __name__ == "__main__":
    main()
