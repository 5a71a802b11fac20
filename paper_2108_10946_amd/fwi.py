"""The inversion loop (the paper's Algorithm 1): c^{k+1} = c^k + alpha^k s^k with
L-BFGS search directions and a line search holding the strong Wolfe conditions,
box bounds on the wave speed, and a fixed region (the water layer) whose gradient
is zero.

The paper's gradient is the L2 one (the mass matrix is the inner product, so the
gradient is mesh independent).  L-BFGS in that inner product is ordinary L-BFGS in
x = M^{1/2} c, where dJ/dx = M^{-1/2} dJ/dc and the bounds stay per DOF because M
is diagonal.  The optimiser is SciPy's L-BFGS-B (bounded L-BFGS, Byrd et al. 1995,
whose line search enforces the strong Wolfe conditions); J and dJ/dc come from the
caller, normally `library_objective` below, so every wave solve runs in the
library's kernels.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class InversionResult:
    c: np.ndarray                 # final wave speed (DOF order)
    J: float                      # final misfit
    history: list = field(default_factory=list)   # J after each accepted iteration
    n_eval: int = 0               # misfit + gradient evaluations
    message: str = ""


def invert(objective, c0, mass, bounds=(1.0, 5.0), fixed=None, max_iter=100, grad_tol=1e-10,
           memory=10):
    """Run Algorithm 1.

    objective(c) -> (J, dJ/dc) for c a float64 array in DOF order (Euclidean
    derivative, as kmv_misfit_gradient returns it).  mass: lumped mass M [n_dofs].
    bounds: (lower, upper) in km/s.  fixed: boolean mask of DOFs kept at c0 (their
    gradient is set to zero), e.g. the water layer c0 < 1.51 km/s.  Stops after
    max_iter iterations, or when the projected M^{-1}-norm of the gradient falls
    below grad_tol, or when the line search cannot reduce J."""
    from scipy.optimize import minimize
    c0 = np.asarray(c0, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float64)
    if c0.shape != mass.shape:
        raise ValueError("c0 and mass must have one entry per DOF")
    lo, hi = bounds
    if not lo < hi:
        raise ValueError("bounds must satisfy lower < upper")
    free = np.ones(len(c0), dtype=bool) if fixed is None else ~np.asarray(fixed, dtype=bool)
    if not free.any():
        raise ValueError("every DOF is fixed")
    s = np.sqrt(mass[free])
    base = c0.copy()
    evals = [0]
    history = []

    def c_of(x):
        c = base.copy()
        c[free] = x / s
        return c

    def fun(x):
        evals[0] += 1
        J, g = objective(c_of(x))
        return float(J), np.asarray(g, dtype=np.float64)[free] / s

    def callback(x):
        history.append(float(fun_cache(x)))

    last = {}

    def fun_cache(x):  # J at the accepted iterate (the optimiser evaluated it already)
        key = x.tobytes()
        if key not in last:
            last.clear()
            last[key] = fun(x)[0]
        return last[key]

    def fun_recorded(x):
        J, gx = fun(x)
        last.clear()
        last[x.tobytes()] = J
        return J, gx

    x0 = np.clip(c0[free], lo, hi) * s
    res = minimize(fun_recorded, x0, jac=True, method="L-BFGS-B",
                   bounds=list(zip(lo * s, hi * s)), callback=callback,
                   options={"maxiter": max_iter, "maxcor": memory, "gtol": grad_tol, "ftol": 0.0,
                            "maxls": 20})
    c = c_of(res.x)
    return InversionResult(c=c, J=float(res.fun), history=history, n_eval=evals[0], message=str(res.message))


def library_objective(problems, observed):
    """objective(c) for `invert` from the library: J and dJ/dc summed over the given
    problems (each one or several shots) with their observed traces, on the GPU."""
    import torch

    def objective(c):
        ct = torch.as_tensor(np.ascontiguousarray(c), dtype=torch.float64, device="cuda")
        J, g = 0.0, torch.zeros_like(ct)
        for prob, obs in zip(problems, observed):  # summed in the library, in problem order
            J = prob.misfit_gradient_accumulate(ct, obs, J, g)
        return J, g.cpu().numpy()

    return objective


def directional_derivative_check(problem, c, observed, hs=(1e-3, 1e-4, 1e-5), mask=None, direction=None):
    """The paper's verification of the discrete gradient (section on the numerical
    verification of the discrete gradient): the directional derivative from the
    gradient, d^co = c~^T M G with the mesh-independent gradient G = M^-1 dJ/dc
    (eq. control_deriv), against forward differences of the misfit,
    d^fd_h = (J(c + h c~) - J(c)) / h (eq. discrete_fd).  The direction c~ is G
    itself unless given, zeroed where mask is False (the absorbing layer), as the
    paper takes it.  Every J and G comes from the library (kmv_misfit_gradient,
    then kmv_misfit for the shifted models); the few vector operations of the check
    itself run on the host.

    Returns {"J", "d_co", "d_fd": {h: value}, "rel_err": {h: |d_fd - d_co| / |d_co|},
    "max_step": max_i |h c~_i| for the largest h}."""
    import torch

    M = problem.mesh.lumped_mass()
    J, g, _ = problem.misfit_gradient(c, observed)
    G = g.cpu().numpy() / M
    ct = G.copy() if direction is None else np.asarray(direction, dtype=np.float64).copy()
    if mask is not None:
        ct[~np.asarray(mask, dtype=bool)] = 0.0
    d_co = float(np.sum(ct * M * G))
    c_host = c.detach().cpu().numpy()
    d_fd, rel = {}, {}
    for h in hs:
        ch = torch.as_tensor(c_host + h * ct, dtype=torch.float64, device=c.device)
        Jh = problem.misfit(ch, observed)
        d_fd[h] = (Jh - J) / h
        rel[h] = abs(d_fd[h] - d_co) / abs(d_co)
    return {"J": J, "d_co": d_co, "d_fd": d_fd, "rel_err": rel, "max_step": float(max(hs) * np.abs(ct).max())}
