"""The perfectly matched layer (PML) — oracle, test infrastructure only.

Plain float64 recursions written from the paper's PML formulation (section
"Forward wave simulation in a PML truncated medium", eqs. acoustic_pml,
acoustic_pml_II, acoustic_pml_III and, in 2D, forward2d_I / forward2d_II; the
matrices of the appendix; the transposed scheme of eqs. acoustic_pml_FEM_adj and
the gradient of eq. gradient).

Damping matrices from the per-axis damping functions sigma_k (quadratic in the
distance into the layer, zero in the physical domain):
    Psi_1 = diag(sigma_k),
    Psi_2 = diag(sigma_k - sum_{j != k} sigma_j),
    Psi_3 = diag(prod_{j != k} sigma_j)                       (3D),
so tr Psi_1 = sum sigma, tr Psi_3 = sigma_x sigma_y + sigma_x sigma_z + sigma_y
sigma_z and det Psi_1 = sigma_x sigma_y sigma_z.  In 2D p_y, omega and sigma_y
vanish: Psi_3 is zero and the zeroth-order u term is sigma_x sigma_z u (the 2D
reduction of tr Psi_3 u; reading: the 2D equation's printed "tr Psi_2 u" is
identically zero in 2D).

Space (every variable in the same KMV space, nodal quadrature; reading: the
divergence of p in the u row is integrated by parts with the natural condition
n.p = 0 that the paper states for the forward solution):
    M U'' + M a' U' + M s U + M d1 Y + K U + sum_k D_k^T P_k = F
    M P_k' + M sigma_k P_k + C_k D_k U - E_k D_k Y = 0,   C_k = c^2 Psi_2^kk, E_k = c^2 Psi_3^kk
    M Y' - M U = 0                                         (3D)
with s = tr Psi_3 (2D: sigma_x sigma_z), d1 = det Psi_1 (2D: 0), a' = tr Psi_1, and
(D_k)_ij = integral of phi_i dphi_j/dx_k (fem.Discretization.derivative_matrices).

Time (central differences, eq. Leapfrog; readings: the damping term of each
first-order auxiliary row is centred as (P^{n+1} + P^{n-1})/2, as the u row centres
its first-derivative term; placed at level n, as the printed A_n has it, the
leapfrog of a decaying mode has a root of modulus 1 + sigma dt and grows.  omega is
advanced by the difference centred at t_{n+1/2}, the trapezoid rule; the three-level
difference centred at t_n leaves an undamped parasitic mode that the couplings
amplify, by |z| = 1.0003 per step already at sigma dt = 0.005):
    (1+a) U^{n+1} = 2U^n - (1-a) U^{n-1}
                    + dt^2 M^-1 (F^n - K U^n - M s U^n - M d1 Y^n - sum_k D_k^T P_k^n)
    (1+b_k) P_k^{n+1} = (1-b_k) P_k^{n-1} - 2 dt M^-1 (C_k D_k U^n - E_k D_k Y^n)
    Y^{n+1} = Y^n + dt (U^{n+1} + U^n) / 2                  (3D)
a = dt tr Psi_1 / 2 (+ the absorbing boundary's dt c b / (2M) when on),
b_k = dt sigma_k, all levels zero before n = 1.

Adjoint (the exact transpose; lambda, mu_k, nu zero after N_t, m = N_t..1):
    nu^m = nu^{m+1} - 2 dt d1 lam^{m+1} + 2 dt M^-1 sum_k D_k^T E_k mu_k^{m+1}      (3D)
    (1+a) lam^m = 2 lam^{m+1} - (1-a) lam^{m+2} + M^-1 P^T y^m + dt^2 (nu^m + nu^{m+1}) / 4
                  - dt^2 M^-1 (K lam^{m+1} + M s lam^{m+1} + sum_k D_k^T C_k mu_k^{m+1})
    (1+b_k) mu_k^m = (1-b_k) mu_k^{m+2} - 2 dt M^-1 D_k lam^{m+1}
y^m = dobs^m - d^m.  Gradient (dJ/dc exactly; c enters K, C_k and E_k):
    g_i = 2 c_i dt^2 sum_{n=0}^{N_t-1} [ pairing_i(lam^{n+1}, U^n)
          + sum_k Psi_2^kk_i mu_k,i^{n+1} (D_k U^n)_i - sum_k Psi_3^kk_i mu_k,i^{n+1} (D_k Y^n)_i ]
(+ the absorbing boundary's term).  The PML terms vanish where sigma = 0.
"""
from __future__ import annotations

import numpy as np

from . import solver


def damping_matrices(sigma):
    """Nodal diagonals from sigma [n, d]: tr Psi_1, Psi_2^kk [n, d], Psi_3^kk [n, d],
    s (the zeroth-order u coefficient) and d1 = det Psi_1 (zero in 2D)."""
    sigma = np.asarray(sigma, dtype=np.float64)
    n, d = sigma.shape
    tr1 = sigma.sum(axis=1)
    psi2 = np.stack([sigma[:, k] - (tr1 - sigma[:, k]) for k in range(d)], axis=1)
    if d == 2:
        psi3 = np.zeros((n, 2))
        s = sigma[:, 0] * sigma[:, 1]
        d1 = np.zeros(n)
    else:
        psi3 = np.stack([np.prod(np.delete(sigma, k, axis=1), axis=1) for k in range(d)], axis=1)
        s = psi3.sum(axis=1)
        d1 = np.prod(sigma, axis=1)
    return tr1, psi2, psi3, s, d1


class PML:
    """The operators of one discretisation with damping functions sigma [n, d]."""

    def __init__(self, disc, sigma):
        self.disc = disc
        self.sigma = np.asarray(sigma, dtype=np.float64)
        assert self.sigma.shape == (disc.n_dofs, disc.dim)
        self.tr1, self.psi2, self.psi3, self.s, self.d1 = damping_matrices(self.sigma)
        self.D = disc.derivative_matrices()
        self.dim = disc.dim


def forward(pml, K, M, a, c, dt, nt, load, P=None, keep_states=False):
    """The coupled recursion for n = 0..nt-1 from zero levels.  Returns (traces
    [nt, nrec] with row n-1 = P U^n or None, states U^0..U^nt or None, and the PML
    states (P_k^0..P_k^nt, Y^0..Y^nt) or None)."""
    N, d = K.shape[0], pml.dim
    Minv = 1.0 / M
    c2 = np.asarray(c, dtype=np.float64) ** 2
    C = [c2 * pml.psi2[:, k] for k in range(d)]
    E = [c2 * pml.psi3[:, k] for k in range(d)]
    b = [dt * pml.sigma[:, k] for k in range(d)]
    u_prev, u = np.zeros(N), np.zeros(N)
    p_prev, p = [np.zeros(N) for _ in range(d)], [np.zeros(N) for _ in range(d)]
    y = np.zeros(N)
    traces = None if P is None else np.zeros((nt, P.shape[0]))
    states = [u.copy()] if keep_states else None
    aux = ([[q.copy() for q in p]], [y.copy()]) if keep_states else None
    for n in range(nt):
        rhs = -(K @ u) - M * pml.s * u - M * pml.d1 * y - sum(pml.D[k].T @ p[k] for k in range(d))
        f = load(n)
        if f is not None:
            rhs = rhs + f
        u_next = (2.0 * u - (1.0 - a) * u_prev + dt * dt * Minv * rhs) / (1.0 + a)
        p_next = [((1.0 - b[k]) * p_prev[k]
                   - 2.0 * dt * Minv * (C[k] * (pml.D[k] @ u) - E[k] * (pml.D[k] @ y))) / (1.0 + b[k])
                  for k in range(d)]
        y_next = y + 0.5 * dt * (u_next + u) if d == 3 else y
        u_prev, u = u, u_next
        p_prev, p = p, p_next
        y = y_next
        if traces is not None:
            traces[n] = P @ u
        if keep_states:
            states.append(u.copy())
            aux[0].append([q.copy() for q in p])
            aux[1].append(y.copy())
    return traces, states, aux


def adjoint(pml, K, M, a, c, dt, P, ydata, record=None):
    """Reverse recursion m = nt..1 with adjoint data ydata [nt, nrec] (row m-1 =
    y^m).  record(m, lam^{m+1}, mu^{m+1}) is called before lam^m is formed.
    Returns lam^1..lam^{nt+1} indexed by m-1."""
    nt = ydata.shape[0]
    N, d = K.shape[0], pml.dim
    Minv = 1.0 / M
    c2 = np.asarray(c, dtype=np.float64) ** 2
    C = [c2 * pml.psi2[:, k] for k in range(d)]
    E = [c2 * pml.psi3[:, k] for k in range(d)]
    b = [dt * pml.sigma[:, k] for k in range(d)]
    lam_p2, lam_p1 = np.zeros(N), np.zeros(N)
    mu_p2, mu_p1 = [np.zeros(N) for _ in range(d)], [np.zeros(N) for _ in range(d)]
    nu_p1 = np.zeros(N)
    out = [None] * (nt + 1)
    out[nt] = lam_p1.copy()
    for m in range(nt, 0, -1):
        if record is not None:
            record(m, lam_p1, mu_p1)
        if d == 3:
            nu = (nu_p1 - 2.0 * dt * pml.d1 * lam_p1
                  + 2.0 * dt * Minv * sum(pml.D[k].T @ (E[k] * mu_p1[k]) for k in range(d)))
        else:
            nu = nu_p1
        coup = sum(pml.D[k].T @ (C[k] * mu_p1[k]) for k in range(d))
        lam = (2.0 * lam_p1 - (1.0 - a) * lam_p2 + Minv * (P.T @ ydata[m - 1]) + 0.25 * dt * dt * (nu + nu_p1)
               - dt * dt * Minv * (K @ lam_p1 + M * pml.s * lam_p1 + coup)) / (1.0 + a)
        mu = [((1.0 - b[k]) * mu_p2[k] - 2.0 * dt * Minv * (pml.D[k] @ lam_p1)) / (1.0 + b[k]) for k in range(d)]
        lam_p2, lam_p1 = lam_p1, lam
        mu_p2, mu_p1 = mu_p1, mu
        nu_p1 = nu
        out[m - 1] = lam.copy()
    return out


def gradient(pml, disc, c, K, M, a, dt, P, dobs, states, aux, bmass=None, r=1, offset=0):
    """Misfit J, dJ/dc and the traces d from the stored forward states (U^n and the
    auxiliary Y^n).  r > 1: gradient subsampling as in solver.gradient, the pairing
    and its PML terms taken at the reverse steps m with m % r == offset, scaled by r."""
    nt = dobs.shape[0]
    d = np.stack([P @ states[n] for n in range(1, nt + 1)])
    J = solver.misfit(d, dobs)
    ydata = dobs - d
    acc = np.zeros(disc.n_dofs)
    Ys = aux[1]

    def record(m, lam_mp1, mu_mp1):
        if m % r != offset:
            return
        acc[:] += disc.gradient_pairing(lam_mp1, states[m])
        for k in range(pml.dim):
            acc[:] += pml.psi2[:, k] * mu_mp1[k] * (pml.D[k] @ states[m])
            if pml.dim == 3:
                acc[:] -= pml.psi3[:, k] * mu_mp1[k] * (pml.D[k] @ Ys[m])

    lam = adjoint(pml, K, M, a, c, dt, P, ydata, record=record)
    g = 2.0 * np.asarray(c) * dt * dt * r * acc
    if bmass is not None:
        bt = np.zeros(disc.n_dofs)
        for n in range(1, nt + 1):
            bt += lam[n - 1] * (states[n] - (states[n - 2] if n >= 2 else 0.0))
        g = g + 0.5 * dt * np.asarray(bmass) * bt
    return J, g, d
