"""Helpers shared by the GPU parity tests (test side only)."""
import sys

import numpy as np
from scipy.spatial import cKDTree


def say(msg):
    """Name the case before a GPU step (flushed, so a crash still shows it)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dof_map(x_lib, x_oracle, tol=1e-9):
    """p with x_lib[i] == x_oracle[p[i]]."""
    d, p = cKDTree(x_oracle).query(x_lib)
    assert np.all(d < tol), f"unmatched DOF coordinates (max distance {d.max()})"
    assert len(np.unique(p)) == len(p)
    return p


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
