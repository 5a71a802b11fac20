"""CPU FP64 oracle for the KMV wave-propagation hot path — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and its
Python binding) never imports, links or calls it, and shares no code with it: the
oracle derives its own element tables, numbers its own degrees of freedom (by
physical node coordinates), assembles its own sparse matrices and runs the plain
three-level recursions of the paper in float64.

Modules
  elements  KMV reference elements (nodes, weights, nodal basis, gradients).
  fem       mesh geometry, DOF numbering, lumped mass, assembled stiffness,
            point interpolation, gradient pairing, boundary mass.
  solver    Ricker wavelet, CFL bounds, forward, adjoint, gradient, misfit,
            absorbing boundary damping and its gradient term.
  green     closed-form 2D homogeneous solution used as an accuracy pin.
  pml       the perfectly matched layer (2D: p; 3D: p and omega), its exact
            discrete adjoint and its terms in the gradient.

Parity status: every function is pinned by tests in ``tests/test_oracle_*.py``
except the degree-5 triangle's identity with the published element (the paper does
not print its nodes) — "parity unpinned" for that identity only; the rule itself is
pinned by exactness, positivity and unisolvence.
"""
