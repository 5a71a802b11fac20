"""KMV (Kong–Mulder–Veldhuizen) mass-lumped reference elements — oracle, test
infrastructure only.

What the paper fixes (section "Higher-order mass lumping" and the implementation
section on higher-order mass-lumped elements):
  * the function space is P_k enriched with bubble functions;
  * the interpolation nodes double as the points of a quadrature rule, so the
    mass matrix is diagonal;
  * node coordinates are printed for KMV2tri, KMV3tri (figure fig:2dels) and
    KMV2tet, KMV3tet (figure fig:3dels).

Readings taken here where the paper is silent:
  * spaces: tri P1; P2+b; P3+b*P1; P4+b*P2; P5+b*P4 (b = l0*l1*l2);
    tet P1; P2+{b_F}+b_T; P3+{b_F*P1(F)}+b_T*P1;
  * weights are the nodal rule exact for polynomials of degree 2k-1: 1, 3, 5, 7 on
    triangles of degree 1..4 and 1, 3, 5 on tetrahedra; the degree-5 triangle's rule
    is exact to degree 10.  KMV2tet, whose degree-3 system leaves a one-parameter
    family, also integrates b_T exactly;
  * KMV4tri and KMV5tri nodes are not printed: they are the solution of the moment
    system with orbit structures {v, m, e, 3, 3} and {v, e, e, 3, 3, 3, 6}, found by
    Newton from the starting values below (degree-5 triangle: identity with the
    published element is parity-unpinned);
  * the KMV3tet interior orbit is the printed (1/6,1/6,1/6,1/2) (the 32-node set in
    the figure; the text's node count of 50 is not used).

Everything is derived in extended precision (mpmath, 50 digits) and rounded to
float64 at the end.
"""
from __future__ import annotations

import functools
import itertools
import math

import mpmath as mp
import numpy as np
import sympy as sp

DPS = 50
_SYM = sp.symbols("x y z")

# Orbits of the reference simplex in barycentric coordinates: label pattern and a
# map from free parameters to label values.
_ORBITS = {
    2: {
        "v": (("a", "o", "o"), lambda: {"a": 1, "o": 0}),
        "m": (("a", "a", "o"), lambda: {"a": mp.mpf(1) / 2, "o": 0}),
        "e": (("a", "b", "o"), lambda t: {"a": t, "b": 1 - t, "o": 0}),
        "c": (("a", "a", "a"), lambda: {"a": mp.mpf(1) / 3}),
        "s3": (("a", "a", "b"), lambda t: {"a": t, "b": 1 - 2 * t}),
        "s6": (("a", "b", "c"), lambda p, q: {"a": p, "b": q, "c": 1 - p - q}),
    },
    3: {
        "v": (("a", "o", "o", "o"), lambda: {"a": 1, "o": 0}),
        "m": (("a", "a", "o", "o"), lambda: {"a": mp.mpf(1) / 2, "o": 0}),
        "e": (("a", "b", "o", "o"), lambda t: {"a": t, "b": 1 - t, "o": 0}),
        "fc": (("a", "a", "a", "o"), lambda: {"a": mp.mpf(1) / 3, "o": 0}),
        "f3": (("a", "a", "b", "o"), lambda t: {"a": t, "b": 1 - 2 * t, "o": 0}),
        "c": (("a", "a", "a", "a"), lambda: {"a": mp.mpf(1) / 4}),
        "i4": (("a", "a", "a", "b"), lambda t: {"a": t, "b": 1 - 3 * t}),
    },
}

# (dim, k) -> list of (orbit kind, starting parameters, parameters free?)
_S = mp.mpf
_DEFS = {
    (2, 1): [("v", (), False)],
    (2, 2): [("v", (), False), ("m", (), False), ("c", (), False)],
    # printed KMV3tri nodes (fig:2dels): edge pair 0.29346955590904..,
    # interior (b, b, 1-2b) with b = 0.20734517566359..
    (2, 3): [("v", (), False), ("e", (_S("0.2934695559090401"),), True),
             ("s3", (_S("0.2073451756635909"),), True)],
    # not printed: solved for from coarse starting values
    (2, 4): [("v", (), False), ("m", (), False), ("e", (_S("0.21"),), True),
             ("s3", (_S("0.42"),), True), ("s3", (_S("0.13"),), True)],
    # not printed: degree-10 solution of the square symmetric moment system
    (2, 5): [("v", (), False),
             ("e", (_S("0.3632980741532427"),), True),
             ("e", (_S("0.1322645816324106"),), True),
             ("s3", (_S("0.2568591072618919"),), True),
             ("s3", (_S("0.4578368380792569"),), True),
             ("s3", (_S("0.0575276844114003"),), True),
             ("s6", (_S("0.2210012187597522"), _S("0.7008061976147790")), True)],
    (3, 1): [("v", (), False)],
    (3, 2): [("v", (), False), ("m", (), False), ("fc", (), False), ("c", (), False)],
    # printed KMV3tet nodes (fig:3dels)
    (3, 3): [("v", (), False), ("e", (_S("0.314210342418033"),), True),
             ("f3", (_S("0.21548220313557542"),), True),
             ("i4", (_S(1) / 6,), False)],
}

_DEGREE = {(2, 1): 1, (2, 2): 3, (2, 3): 5, (2, 4): 7, (2, 5): 10,
           (3, 1): 1, (3, 2): 3, (3, 3): 5}

# Weight starting values where a Newton solve for nodes is needed (orbit order).
_W0 = {
    (2, 4): ["0.003", "0.0127", "0.0107", "0.079", "0.05"],
    (2, 5): ["0.0007094239706781", "0.0061905650036728", "0.0034805786404815",
             "0.0459012376308416", "0.0345304303773024", "0.0116261354595990",
             "0.0272785759699685"],
}


def orbit_points(dim, kind, params):
    """Distinct barycentric points of one orbit, in lexicographic label order."""
    pattern, fn = _ORBITS[dim][kind]
    vals = fn(*params)
    perms = sorted(set(itertools.permutations(pattern)))
    return [tuple(mp.mpf(vals[l]) for l in p) for p in perms]


def _monomial_exponents(dim, deg):
    out = []
    for total in range(deg + 1):
        for e in itertools.product(range(total + 1), repeat=dim):
            if sum(e) == total:
                out.append(e)
    return out


def reference_monomial_integral(exps):
    """Exact integral of prod x_r^e_r over the reference simplex
    {x_r >= 0, sum x_r <= 1}:  prod(e_r!) / (sum(e_r) + dim)!."""
    num = 1
    for e in exps:
        num *= math.factorial(e)
    return mp.mpf(num) / math.factorial(sum(exps) + len(exps))


def _cart(bary):
    return bary[1:]


def _rule_residual(dim, k, structure, params, weights):
    """Moment residuals sum_i w_i m(x_i) - int m for all monomials of degree <= q
    (plus b_T for KMV2tet)."""
    pts_by_orbit = []
    pi = 0
    for kind, p0, free in structure:
        n = len(p0)
        p = params[pi:pi + n] if free else p0
        if free:
            pi += n
        pts_by_orbit.append([_cart(b) for b in orbit_points(dim, kind, p)])
    res = []
    for e in _monomial_exponents(dim, _DEGREE[(dim, k)]):
        s = mp.mpf(0)
        for w, pts in zip(weights, pts_by_orbit):
            for x in pts:
                t = mp.mpf(1)
                for r in range(dim):
                    t *= x[r] ** e[r]
                s += w * t
        res.append(s - reference_monomial_integral(e))
    if (dim, k) == (3, 2):
        s = mp.mpf(0)
        for w, pts in zip(weights, pts_by_orbit):
            for x in pts:
                s += w * (1 - sum(x)) * x[0] * x[1] * x[2]
        res.append(s - mp.mpf(1) / 5040)
    return res


def _solve_rule(dim, k):
    structure = _DEFS[(dim, k)]
    params = [p for kind, p0, free in structure if free for p in p0]
    nw = len(structure)
    w0 = _W0.get((dim, k))
    weights = [mp.mpf(w) for w in w0] if w0 else [mp.mpf(1) / (10 * nw)] * nw
    x = list(params) + list(weights)
    npar = len(params)
    h = mp.mpf(10) ** (-(DPS // 2))
    for _ in range(60):
        r = mp.matrix(_rule_residual(dim, k, structure, x[:npar], x[npar:]))
        if mp.norm(r) < mp.mpf(10) ** (-(DPS - 10)):
            break
        J = mp.matrix(len(r), len(x))
        for j in range(len(x)):
            xp = list(x)
            xm = list(x)
            xp[j] += h
            xm[j] -= h
            rp = _rule_residual(dim, k, structure, xp[:npar], xp[npar:])
            rm = _rule_residual(dim, k, structure, xm[:npar], xm[npar:])
            for i in range(len(r)):
                J[i, j] = (rp[i] - rm[i]) / (2 * h)
        JT = J.T
        dx = mp.lu_solve(JT * J, -(JT * r))
        x = [x[i] + dx[i] for i in range(len(x))]
    else:
        raise RuntimeError(f"KMV rule ({dim},{k}) did not converge")
    res = _rule_residual(dim, k, structure, x[:npar], x[npar:])
    return structure, x[:npar], x[npar:], max(abs(v) for v in res)


def _space(dim, k):
    """Spanning polynomials of the KMV space (sympy expressions)."""
    X = _SYM[:dim]
    lam = [1 - sum(X)] + list(X)
    polys = []
    for e in _monomial_exponents(dim, k):
        m = sp.Integer(1)
        for r in range(dim):
            m *= X[r] ** e[r]
        polys.append(m)
    if dim == 2:
        b = lam[0] * lam[1] * lam[2]
        if k == 2:
            polys.append(b)
        elif k == 3:
            polys += [b * X[0], b * X[1]]
        elif k == 4:
            polys += [b * X[0] ** 2, b * X[0] * X[1], b * X[1] ** 2]
        elif k == 5:
            for e in _monomial_exponents(2, 4):
                if sum(e) >= 3:
                    polys.append(b * X[0] ** e[0] * X[1] ** e[1])
    else:
        bT = lam[0] * lam[1] * lam[2] * lam[3]
        faces = [[i for i in range(4) if i != j] for j in range(4)]
        if k == 2:
            for F in faces:
                polys.append(lam[F[0]] * lam[F[1]] * lam[F[2]])
            polys.append(bT)
        elif k == 3:
            for F in faces:
                bF = lam[F[0]] * lam[F[1]] * lam[F[2]]
                polys += [bF * lam[F[0]], bF * lam[F[1]]]
            polys += [bT * lam[j] for j in range(4)]
    return [sp.expand(p) for p in polys]


class KMVElement:
    """Float64 tables of one KMV element.

    nodes   [n_d, dim]  reference coordinates (the quadrature points)
    weights [n_d]       quadrature weights (reference simplex measure 1/2 or 1/6)
    D       [n_d, n_d, dim]  D[q, a, r] = d phi_a / d x_r at node q
    """

    def __init__(self, dim, k):
        if (dim, k) not in _DEFS:
            raise ValueError(f"no KMV element for dim={dim}, k={k}")
        self.dim, self.k = dim, k
        with mp.workdps(DPS):
            structure, params, weights, resid = _solve_rule(dim, k)
            self.rule_residual = float(resid)
            pts, wts = [], []
            pi = 0
            for (kind, p0, free), w in zip(structure, weights):
                n = len(p0)
                p = params[pi:pi + n] if free else p0
                if free:
                    pi += n
                for b in orbit_points(dim, kind, p):
                    pts.append(_cart(b))
                    wts.append(w)
            self.orbit_params = [float(v) for v in params]
            self.orbit_weights = [float(w) for w in weights]
            funcs = _space(dim, k)
            n = len(funcs)
            if n != len(pts):
                raise RuntimeError(f"space dim {n} != node count {len(pts)}")
            X = _SYM[:dim]
            f_mp = [sp.lambdify(X, f, modules="mpmath") for f in funcs]
            df_mp = [[sp.lambdify(X, sp.diff(f, X[r]), modules="mpmath") for r in range(dim)]
                     for f in funcs]
            V = mp.matrix(n, n)
            for i, x in enumerate(pts):
                for j in range(n):
                    V[i, j] = f_mp[j](*x)
            C = mp.inverse(V)
            self.vandermonde_cond = float(mp.norm(V, 1) * mp.norm(C, 1))
            D = np.zeros((n, n, dim))
            for q, x in enumerate(pts):
                dvals = [[df_mp[j][r](*x) for r in range(dim)] for j in range(n)]
                for a in range(n):
                    for r in range(dim):
                        s = mp.mpf(0)
                        for j in range(n):
                            s += dvals[j][r] * C[j, a]
                        D[q, a, r] = float(s)
            self.nodes = np.array([[float(v) for v in x] for x in pts])
            self.weights = np.array([float(w) for w in wts])
            self.D = D
            self._C = np.array([[float(C[i, j]) for j in range(n)] for i in range(n)])
        self.n_d = len(self.nodes)
        self._f_np = [sp.lambdify(X, f, modules="numpy") for f in funcs]
        self._df_np = [[sp.lambdify(X, sp.diff(f, X[r]), modules="numpy") for r in range(dim)]
                       for f in funcs]

    def tabulate(self, pts):
        """Basis values [npts, n_d] and reference gradients [npts, n_d, dim] at the
        reference points ``pts`` [npts, dim] (float64)."""
        pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
        cols = [pts[:, r] for r in range(self.dim)]
        F = np.stack([np.broadcast_to(np.asarray(f(*cols), dtype=np.float64), (len(pts),))
                      for f in self._f_np], axis=1)
        dF = np.stack([np.stack([np.broadcast_to(np.asarray(df[r](*cols), dtype=np.float64),
                                                 (len(pts),))
                                 for df in self._df_np], axis=1) for r in range(self.dim)],
                      axis=2)
        vals = F @ self._C
        grads = np.einsum("pjr,ja->par", dF, self._C)
        return vals, grads


@functools.lru_cache(maxsize=None)
def kmv_element(dim, k):
    return KMVElement(dim, k)
