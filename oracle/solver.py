"""Time stepping, misfit, adjoint and gradient — oracle, test infrastructure only.

Plain float64 three-level recursions, written from the paper:

* Ricker source w(t) = A (1 - 2 pi^2 f^2 (t-t0)^2) exp(-pi^2 f^2 (t-t0)^2)
  (section on the forward wave simulation; delay t0 and amplitude A are inputs).
* Forward (eqs. Leapfrog and forward3, u block with the damping term only, the
  diagonal A_{n+1} inverted pointwise):
      (1+a) u^{n+1} = 2 u^n - (1-a) u^{n-1} + dt^2 M^{-1} (b^n - K u^n),
  a = eta dt / 2, u^{-1} = u^0 = 0, b^n = w(t_n) s, t_n = n dt; the shot record
  is d^n = P u^n for n = 1..N_t.
* Misfit (eq. l2error with time sums and no dt factor, as the paper states for its
  discrete adjoint): J = 1/2 sum_n sum_j (d^n_j - dobs^n_j)^2.
* Adjoint (the transposed scheme of eq. acoustic_pml_FEM_adj), reverse in time
  from lam^{N_t+1} = lam^{N_t+2} = 0:
      (1+a) lam^m = 2 lam^{m+1} - dt^2 M^{-1} K lam^{m+1} - (1-a) lam^{m+2}
                    + M^{-1} P^T y^m,        y^m = dobs^m - d^m.
* Gradient (eq. gradient3 read as the exact derivative of the discrete J):
      g_i = 2 c_i dt^2 sum_{n=0}^{N_t-1} sum_{(e,q)->i} w_q|det J_e|
            grad lam^{n+1}(x_eq) . grad u^n(x_eq),
  and the mesh-independent (Riesz) gradient G = M^{-1} g.
* Gradient subsampling (section on gradient subsampling): the forward state is
  kept every r steps and the pairing is taken only there, n = m with
  m = offset (mod r); the sum is scaled by r, so r = 1 is the exact gradient and
  r > 1 approximates it (a reading: the paper does not state the scale).
* Absorbing boundary (the first-order condition du/dt + c du/dn = 0 on the outer
  boundary, whose weak form adds the boundary integral of c phi_i phi_j to the
  damping matrix M_{u,1} of the appendix): lumped by rows with c taken at node i it
  is diag(c_i b_i), b_i = the boundary integral of phi_i, and the scheme above holds
  with a = eta dt / 2 + dt c b / (2 M).  Because that damping depends on c, the
  derivative of J gains a boundary term.  Writing the scheme as
  M (u^{n+1} - 2u^n + u^{n-1})/dt^2 + D (u^{n+1} - u^{n-1})/(2dt) + K u^n = b^n with
  D = diag(eta M + c b), the multiplier of its n-th row is -dt^2 lam^{n+1}, so
      dJ/dc_i += (dt b_i / 2) sum_{n=0}^{N_t-1} lam_i^{n+1} (u_i^{n+1} - u_i^{n-1})
               = (dt b_i / 2) sum_{n=1}^{N_t} lam_i^n (u_i^n - u_i^{n-2})
  (u^{-1} = u^0 = 0).  It is taken at every step, also with gradient subsampling.
* CFL bound (eq. spectral): dt <= 2 / sqrt(rho(M^{-1}K)), rho by Gershgorin
  discs, plus a seeded power iteration for the actual spectral radius.
"""
from __future__ import annotations

import numpy as np


def ricker(t, f0, t0, amp=1.0):
    t = np.asarray(t, dtype=np.float64)
    arg = (np.pi * f0 * (t - t0)) ** 2
    return amp * (1.0 - 2.0 * arg) * np.exp(-arg)


def gershgorin_rho(K, M):
    """max_i sum_j |K_ij| / M_i."""
    rowsum = np.asarray(abs(K).sum(axis=1)).ravel()
    return float(np.max(rowsum / M))


def cfl_dt_gershgorin(K, M):
    return 2.0 / np.sqrt(gershgorin_rho(K, M))


def power_rho(K, M, iters=500, seed=0):
    """Spectral radius of M^{-1} K by power iteration on the symmetric form
    M^{-1/2} K M^{-1/2} (same spectrum)."""
    rng = np.random.default_rng(seed)
    s = 1.0 / np.sqrt(M)
    v = rng.standard_normal(len(M))
    v /= np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = s * (K @ (s * v))
        lam = float(v @ w)
        v = w / np.linalg.norm(w)
    return lam


def forward(K, M, a, dt, nt, load, P=None, u0=None, um1=None, keep_states=False):
    """Run the three-level forward recursion for n = 0..nt-1.

    load(n) -> nodal load vector b^n (or None for no load).  Returns
    (traces [nt, nrec] with row n-1 = P u^n, states list u^0..u^nt or None)."""
    N = K.shape[0]
    Minv = 1.0 / M
    a = np.zeros(N) if a is None else np.asarray(a, dtype=np.float64)
    u_prev = np.zeros(N) if um1 is None else np.array(um1, dtype=np.float64)
    u = np.zeros(N) if u0 is None else np.array(u0, dtype=np.float64)
    traces = None if P is None else np.zeros((nt, P.shape[0]))
    states = [u.copy()] if keep_states else None
    for n in range(nt):
        rhs = -(K @ u)
        b = load(n)
        if b is not None:
            rhs = rhs + b
        u_next = (2.0 * u - (1.0 - a) * u_prev + dt * dt * Minv * rhs) / (1.0 + a)
        u_prev, u = u, u_next
        if traces is not None:
            traces[n] = P @ u
        if keep_states:
            states.append(u.copy())
    return traces, states


def point_source_load(s_vec, wavelet):
    """b^n = w(t_n) s for a point source with interpolation vector s."""
    def load(n):
        return wavelet[n] * s_vec
    return load


def misfit(d, dobs):
    r = np.asarray(d) - np.asarray(dobs)
    return 0.5 * float(np.sum(r * r))


def adjoint(K, M, a, dt, P, y, record=None):
    """Reverse recursion for lam^m, m = nt..1, with adjoint data y [nt, nrec]
    (row m-1 is y^m).  ``record(m, lam_mp1)`` is called with lam^{m+1} before
    lam^m is formed.  Returns lam^1..lam^{nt+1} as a list indexed by m-1."""
    nt = y.shape[0]
    N = K.shape[0]
    Minv = 1.0 / M
    a = np.zeros(N) if a is None else np.asarray(a, dtype=np.float64)
    lam_p2 = np.zeros(N)
    lam_p1 = np.zeros(N)
    out = [None] * (nt + 1)
    out[nt] = lam_p1.copy()
    for m in range(nt, 0, -1):
        if record is not None:
            record(m, lam_p1)
        lam = (2.0 * lam_p1 - dt * dt * Minv * (K @ lam_p1) - (1.0 - a) * lam_p2
               + Minv * (P.T @ y[m - 1])) / (1.0 + a)
        lam_p2, lam_p1 = lam_p1, lam
        out[m - 1] = lam.copy()
    return out


def gradient(disc, c, K, M, a, dt, P, dobs, states, r=1, offset=0, bmass=None):
    """Misfit J, dJ/dc (Euclidean) and the traces d, from stored forward states
    u^0..u^nt.  The pairing at reverse step m is (lam^{m+1}, u^m), m = nt..1; the
    n = 0 term vanishes because u^0 = 0.  With r > 1 only the steps with
    m % r == offset are paired and the sum is multiplied by r.  bmass: the
    boundary mass b when the absorbing boundary is on (its term is added)."""
    nt = dobs.shape[0]
    d = np.stack([P @ states[n] for n in range(1, nt + 1)])
    J = misfit(d, dobs)
    y = dobs - d
    acc = np.zeros(disc.n_dofs)

    def record(m, lam_mp1):
        if m % r == offset:
            acc[:] += disc.gradient_pairing(lam_mp1, states[m])

    lam = adjoint(K, M, a, dt, P, y, record=record)  # lam[m-1] = lam^m
    g = 2.0 * np.asarray(c) * dt * dt * r * acc
    if bmass is not None:
        bt = np.zeros(disc.n_dofs)
        for n in range(1, nt + 1):
            bt += lam[n - 1] * (states[n] - (states[n - 2] if n >= 2 else 0.0))
        g = g + 0.5 * dt * np.asarray(bmass) * bt
    return J, g, d


class Shot:
    """One shot on one discretisation: source/receiver operators and wavelet."""

    def __init__(self, disc, src_pts, rec_pts, dt, nt, f0=5.0, t0=None, amp=1.0,
                 wavelet=None):
        self.disc = disc
        self.dt = dt
        self.nt = nt
        S = disc.interpolation_matrix(src_pts)
        self.s_vec = np.asarray(S.sum(axis=0)).ravel()
        self.P = disc.interpolation_matrix(rec_pts)
        if wavelet is None:
            t0 = 1.0 / f0 if t0 is None else t0
            wavelet = ricker(np.arange(nt) * dt, f0, t0, amp)
        self.wavelet = np.asarray(wavelet, dtype=np.float64)

    def damping(self, c, M, eta, absorb):
        """a = eta dt / 2, plus dt c b / (2 M) with the absorbing boundary."""
        a = None if eta is None else np.asarray(eta) * self.dt / 2.0
        if absorb:
            ab = self.dt * np.asarray(c) * self.disc.boundary_mass() / (2.0 * M)
            a = ab if a is None else a + ab
        return a

    def forward(self, c, eta=None, keep_states=False, absorb=False, pml=None):
        """pml: per-axis damping functions sigma [n_dofs, dim] of the PML (oracle.pml),
        which then replaces the sponge (eta must be None)."""
        disc = self.disc
        K = disc.stiffness(c)
        M = disc.lumped_mass()
        if pml is not None:
            from . import pml as PML
            assert eta is None, "the PML replaces the sponge"
            pm = PML.PML(disc, pml)
            a = self.damping(c, M, pm.tr1, absorb)
            tr, st, _ = PML.forward(pm, K, M, a, c, self.dt, self.nt,
                                    point_source_load(self.s_vec, self.wavelet), P=self.P,
                                    keep_states=keep_states)
            return tr, st
        a = self.damping(c, M, eta, absorb)
        return forward(K, M, a, self.dt, self.nt, point_source_load(self.s_vec, self.wavelet),
                       P=self.P, keep_states=keep_states)

    def misfit_gradient(self, c, dobs, eta=None, r=1, offset=0, absorb=False, pml=None):
        disc = self.disc
        K = disc.stiffness(c)
        M = disc.lumped_mass()
        if pml is not None:
            from . import pml as PML
            assert eta is None, "the PML replaces the sponge"
            pm = PML.PML(disc, pml)
            a = self.damping(c, M, pm.tr1, absorb)
            _, states, aux = PML.forward(pm, K, M, a, c, self.dt, self.nt,
                                         point_source_load(self.s_vec, self.wavelet), P=None,
                                         keep_states=True)
            return PML.gradient(pm, disc, c, K, M, a, self.dt, self.P, dobs, states, aux,
                                bmass=disc.boundary_mass() if absorb else None, r=r, offset=offset)
        a = self.damping(c, M, eta, absorb)
        _, states = forward(K, M, a, self.dt, self.nt,
                            point_source_load(self.s_vec, self.wavelet), P=None,
                            keep_states=True)
        return gradient(disc, c, K, M, a, self.dt, self.P, dobs, states, r=r, offset=offset,
                        bmass=disc.boundary_mass() if absorb else None)
