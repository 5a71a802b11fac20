"""Mesh geometry, degrees of freedom and assembled operators — oracle, test
infrastructure only.  Plain float64 NumPy/SciPy, written from the definitions:

* affine map x = x_0 + J_e xi, physical gradients J_e^{-T} grad_xi (section
  "Spatial discretization");
* one degree of freedom per distinct physical node (the local-to-global map g(j,k)
  of the section on receivers and sources), found here by grouping coincident
  node coordinates — no mesh topology is used;
* lumped mass M_i = sum over (e,q) with g(e,q)=i of w_q |det J_e| (the KMV rule
  makes the mass matrix of the appendix diagonal);
* stiffness K_ij = sum_e sum_q w_q |det J_e| c^2(x_eq) grad phi_i(x_eq).grad phi_j(x_eq)
  (appendix, matrix K), with c nodal so c^2(x_eq) = c^2_{g(e,q)};
* point interpolation / Dirac injection with weights phi_a(xi) in the containing
  cell (section "Receivers and sources");
* gradient pairing sum_{(e,q)->i} w_q |det J_e| grad lam(x_eq).grad u(x_eq), the
  integrand of eq. gradient3 at the quadrature nodes;
* derivative matrices D_k, (D_k)_ij = integral of phi_i dphi_j/dx_k by the nodal
  rule (appendix, matrix D; the PML couplings of eqs. acoustic_pml_FEM and
  acoustic_pml_II_FEM);
* boundary mass b_i = integral over the mesh boundary of phi_i, the row sums of the
  boundary integral of c phi_i phi_j in the damping matrix M_{u,1} (appendix, with c
  taken at node i), by Gauss quadrature of the trace of the cell basis on every
  facet that belongs to one cell only.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps
from scipy.sparse.csgraph import connected_components
from scipy.spatial import cKDTree

from .elements import kmv_element


class Discretization:
    def __init__(self, coords, cells, degree):
        coords = np.asarray(coords, dtype=np.float64)
        cells = np.asarray(cells, dtype=np.int64)
        self.dim = coords.shape[1]
        self.degree = degree
        self.elem = kmv_element(self.dim, degree)
        self.coords = coords
        self.cells = cells
        self.n_cells = len(cells)
        d = self.dim
        x0 = coords[cells[:, 0]]
        J = np.stack([coords[cells[:, r + 1]] - x0 for r in range(d)], axis=2)  # [e, i, r]
        self.J = J
        self.detJ = np.linalg.det(J)
        if np.any(self.detJ == 0.0):
            raise ValueError("degenerate cell")
        self.absdet = np.abs(self.detJ)
        self.Jinv = np.linalg.inv(J)
        # physical coordinates of every (cell, node) pair
        X = x0[:, None, :] + np.einsum("eir,qr->eqi", J, self.elem.nodes)
        self.cell_node_coords = X
        self.cell_dofs, self.dof_coords = self._number_dofs(X)
        self.n_dofs = len(self.dof_coords)
        # quadrature weight per (e, q)
        self.W = self.absdet[:, None] * self.elem.weights[None, :]
        # physical gradient of basis a at node q of cell e: B[e, q, a, :]
        self.B = np.einsum("esi,qas->eqai", self.Jinv, self.elem.D)

    @staticmethod
    def _number_dofs(X):
        ne, nd, d = X.shape
        flat = X.reshape(-1, d)
        span = np.ptp(flat, axis=0).max()
        tol = 1e-9 * span
        pairs = cKDTree(flat).query_pairs(r=tol, output_type="ndarray")
        n = len(flat)
        G = sps.coo_matrix((np.ones(len(pairs)), (pairs[:, 0], pairs[:, 1])), shape=(n, n))
        ncomp, labels = connected_components(G, directed=False)
        # number components in order of first appearance
        first = np.full(ncomp, n, dtype=np.int64)
        np.minimum.at(first, labels, np.arange(n))
        order = np.argsort(first)
        rank = np.empty(ncomp, dtype=np.int64)
        rank[order] = np.arange(ncomp)
        dofs = rank[labels].reshape(ne, nd)
        coords = flat[first[order]]
        return dofs, coords

    # ------------------------------------------------------------------ operators
    def lumped_mass(self):
        return np.bincount(self.cell_dofs.ravel(), weights=self.W.ravel(),
                           minlength=self.n_dofs)

    def element_stiffness(self, c):
        """K_e[a, b] = sum_q W[e,q] c^2_{g(e,q)} B[e,q,a,:].B[e,q,b,:]."""
        c2q = np.asarray(c, dtype=np.float64)[self.cell_dofs] ** 2
        coef = self.W * c2q
        return np.einsum("eq,eqai,eqbi->eab", coef, self.B, self.B, optimize=True)

    def stiffness(self, c):
        Ke = self.element_stiffness(c)
        nd = self.elem.n_d
        rows = np.repeat(self.cell_dofs, nd, axis=1).ravel()
        cols = np.tile(self.cell_dofs, (1, nd)).ravel()
        K = sps.coo_matrix((Ke.ravel(), (rows, cols)), shape=(self.n_dofs, self.n_dofs))
        return K.tocsr()

    def nodal_gradients(self, u):
        """grad u at every (cell, node): [e, q, dim]."""
        ue = np.asarray(u)[self.cell_dofs]
        nd, d = self.elem.n_d, self.dim
        # reference gradients: ghat[e, q, s] = sum_a D[q, a, s] u_e[a]
        ghat = (ue @ self.elem.D.transpose(1, 0, 2).reshape(nd, nd * d)).reshape(-1, nd, d)
        # physical gradients: J_e^{-T} ghat
        g = np.zeros_like(ghat)
        for s in range(d):
            g += self.Jinv[:, None, s, :] * ghat[:, :, s, None]
        return g

    def derivative_matrices(self):
        """D_k [n_dofs, n_dofs], k < dim: (D_k)_ij = integral of phi_i dphi_j/dx_k by the
        nodal rule, sum over (e,q) with g(e,q) = i of W[e,q] dphi_a/dx_k(x_eq) with
        j = g(e,a) (appendix, matrix D).  (D_k u)_i is the mass-weighted sum over the
        cells at DOF i of du/dx_k there; D_k^T is the weak divergence of the
        appendix's u-row coupling, integrated by parts."""
        nd = self.elem.n_d
        rows = np.repeat(self.cell_dofs, nd, axis=1).ravel()       # i = g(e, q)
        cols = np.tile(self.cell_dofs, (1, nd)).ravel()            # j = g(e, a)
        out = []
        for k in range(self.dim):
            vals = (self.W[:, :, None] * self.B[:, :, :, k]).ravel()  # [e, q, a]
            out.append(sps.coo_matrix((vals, (rows, cols)), shape=(self.n_dofs, self.n_dofs)).tocsr())
        return out

    def gradient_pairing(self, lam, u):
        """r_i = sum_{(e,q) -> i} W[e,q] grad lam(x_eq) . grad u(x_eq)."""
        gl = self.nodal_gradients(lam)
        gu = self.nodal_gradients(u)
        s = self.W * sum(gl[:, :, i] * gu[:, :, i] for i in range(self.dim))
        return np.bincount(self.cell_dofs.ravel(), weights=s.ravel(), minlength=self.n_dofs)

    # ------------------------------------------------------------------ points
    def locate(self, pts, tol=1e-12):
        """Containing cell (lowest id among ties) and reference coordinates."""
        pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
        x0 = self.coords[self.cells[:, 0]]
        out_cell = np.full(len(pts), -1, dtype=np.int64)
        out_xi = np.zeros((len(pts), self.dim))
        for p, x in enumerate(pts):
            xi = np.einsum("eri,ei->er", self.Jinv, x[None, :] - x0)
            bary = np.concatenate([1.0 - xi.sum(axis=1, keepdims=True), xi], axis=1)
            inside = np.nonzero(np.all(bary >= -tol, axis=1))[0]
            if len(inside) == 0:
                raise ValueError(f"point {x} lies outside the mesh")
            e = inside[0]
            out_cell[p] = e
            out_xi[p] = xi[e]
        return out_cell, out_xi

    def interpolation_matrix(self, pts):
        """Sparse P [npts, n_dofs] with P[p, g(e_p, a)] = phi_a(xi_p)."""
        cell, xi = self.locate(pts)
        vals, _ = self.elem.tabulate(xi)
        nd = self.elem.n_d
        rows = np.repeat(np.arange(len(cell)), nd)
        cols = self.cell_dofs[cell].ravel()
        P = sps.coo_matrix((vals.ravel(), (rows, cols)), shape=(len(cell), self.n_dofs))
        return P.tocsr()

    def boundary_mass(self, n_gauss=8):
        """b_i = integral over the boundary of phi_i (zero off the boundary).

        A facet (d vertices) on the boundary belongs to one cell; on it the cell's
        basis is integrated with an n_gauss-point Gauss-Legendre rule on an edge, or
        the collapsed (Duffy) n_gauss^2 product rule on a triangle."""
        d = self.dim
        x, w = np.polynomial.legendre.leggauss(n_gauss)
        x, w = (x + 1.0) / 2.0, w / 2.0
        if d == 2:   # facet barycentrics (1-t, t), weights summing to 1
            fb = np.stack([1.0 - x, x], axis=1)
            fw = w
        else:        # (s, r) = (x_i, (1-x_i) x_j) covers the triangle; weights sum to 1
            s = np.repeat(x, n_gauss)
            r = (1.0 - s) * np.tile(x, n_gauss)
            fb = np.stack([1.0 - s - r, s, r], axis=1)
            fw = 2.0 * np.repeat(w, n_gauss) * np.tile(w, n_gauss) * (1.0 - s)
        owners = {}
        for e, cell in enumerate(self.cells):
            for v in range(d + 1):
                owners.setdefault(tuple(sorted(np.delete(cell, v))), []).append((e, v))
        b = np.zeros(self.n_dofs)
        for key, own in owners.items():
            if len(own) != 1:
                continue
            e, v = own[0]
            V = self.coords[np.delete(self.cells[e], v)]          # facet vertices [d, d]
            if d == 2:
                measure = np.linalg.norm(V[1] - V[0])
            else:
                measure = 0.5 * np.linalg.norm(np.cross(V[1] - V[0], V[2] - V[0]))
            X = fb @ V                                             # physical points
            xi = (X - self.coords[self.cells[e, 0]]) @ self.Jinv[e].T
            vals, _ = self.elem.tabulate(xi)
            np.add.at(b, self.cell_dofs[e], measure * (fw @ vals))
        return b

    def nodal_values(self, fn):
        """Evaluate a function of point coordinates at the DOF coordinates."""
        return fn(*[self.dof_coords[:, r] for r in range(self.dim)])
