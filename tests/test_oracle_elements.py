"""Pins for the oracle's KMV reference elements (section "Higher-order mass
lumping", figures fig:2dels and fig:3dels)."""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle.elements import kmv_element

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "kmv_printed_nodes.json")))
ALL = [(2, 1), (2, 2), (2, 3), (2, 4), (2, 5), (3, 1), (3, 2), (3, 3)]
DEGREE = {(2, 1): 1, (2, 2): 3, (2, 3): 5, (2, 4): 7, (2, 5): 10, (3, 1): 1, (3, 2): 3, (3, 3): 5}


def collapsed_gauss(dim, n):
    """Independent reference rule: Gauss-Legendre on the cube mapped to the
    simplex by the Duffy collapse (numpy's leggauss)."""
    x, w = np.polynomial.legendre.leggauss(n)
    x = 0.5 * (x + 1.0)
    w = 0.5 * w
    if dim == 2:
        U, V = np.meshgrid(x, x, indexing="ij")
        WU, WV = np.meshgrid(w, w, indexing="ij")
        pts = np.stack([U.ravel(), (V * (1 - U)).ravel()], 1)
        wts = (WU * WV * (1 - U)).ravel()
    else:
        U, V, Wc = np.meshgrid(x, x, x, indexing="ij")
        WU, WV, WW = np.meshgrid(w, w, w, indexing="ij")
        p0 = U
        p1 = V * (1 - U)
        p2 = Wc * (1 - U) * (1 - V)
        pts = np.stack([p0.ravel(), p1.ravel(), p2.ravel()], 1)
        wts = (WU * WV * WW * (1 - U) ** 2 * (1 - V)).ravel()
    return pts, wts


def random_poly(dim, deg, rng):
    exps = [e for e in itertools.product(range(deg + 1), repeat=dim) if sum(e) <= deg]
    coef = rng.standard_normal(len(exps))

    def f(p):
        return sum(c * np.prod([p[:, r] ** e[r] for r in range(dim)], axis=0) for c, e in zip(coef, exps))
    return f


def same_set(a, b, tol):
    a = np.asarray(a)
    b = np.asarray(b)
    if a.shape != b.shape:
        return False
    used = np.zeros(len(b), dtype=bool)
    for p in a:
        d = np.linalg.norm(b - p, axis=1)
        d[used] = np.inf
        j = int(np.argmin(d))
        if d[j] > tol:
            return False
        used[j] = True
    return True


@pytest.mark.parametrize("key,dk,tol", [("tri2", (2, 2), 1e-15), ("tri3", (2, 3), 2e-15),
                                        ("tet2", (3, 2), 1e-15), ("tet3", (3, 3), 2e-15)])
def test_nodes_match_printed(key, dk, tol):
    e = kmv_element(*dk)
    assert same_set(e.nodes, GOLD[key], tol)


@pytest.mark.parametrize("dk", ALL)
def test_rule_exactness_against_gauss(dk):
    """The nodal rule integrates every polynomial of its degree exactly and fails
    one degree higher (so the stated degree is the true one)."""
    dim, _ = dk
    e = kmv_element(*dk)
    q = DEGREE[dk]
    gp, gw = collapsed_gauss(dim, 12)
    rng = np.random.default_rng(1)
    for _ in range(3):
        f = random_poly(dim, q, rng)
        exact = gw @ f(gp)
        assert abs(e.weights @ f(e.nodes) - exact) <= 1e-13 * max(1.0, abs(exact))
    worst = 0.0
    for _ in range(5):
        f = random_poly(dim, q + 1, rng)
        worst = max(worst, abs(e.weights @ f(e.nodes) - gw @ f(gp)))
    assert worst > 1e-8


@pytest.mark.parametrize("dk", ALL)
def test_weights_positive_and_sum(dk):
    dim, _ = dk
    e = kmv_element(*dk)
    assert np.all(e.weights > 0)
    assert abs(e.weights.sum() - (0.5 if dim == 2 else 1.0 / 6.0)) < 1e-15


def test_closed_form_weights():
    e2 = kmv_element(2, 2)
    assert np.allclose(sorted(set(np.round(e2.weights, 15))), [1 / 40, 1 / 15, 9 / 40], atol=1e-16)
    # KMV2tet: the interior bubble b_T is only nonzero at the centroid, where it is
    # 1/256, and integrates to 1/5040, so the centroid weight is 256/5040 = 16/315.
    t2 = kmv_element(3, 2)
    cen = np.argmin(np.linalg.norm(t2.nodes - 0.25, axis=1))
    assert abs(t2.weights[cen] - 16 / 315) < 1e-16
    # KMV4tri: edge points at the 2-point Gauss-Legendre abscissae of the edge
    e4 = kmv_element(2, 4)
    assert abs(e4.orbit_params[0] - (1 - 1 / math.sqrt(3)) / 2) < 1e-15
    assert np.allclose(e4.orbit_weights[:3], [1 / 315, 4 / 315, 3 / 280], atol=1e-16)


@pytest.mark.parametrize("dk", ALL)
def test_nodal_basis(dk):
    dim, k = dk
    e = kmv_element(*dk)
    vals, grads = e.tabulate(e.nodes)
    assert np.allclose(vals, np.eye(e.n_d), atol=1e-11)
    assert np.allclose(grads, e.D, atol=1e-9)
    rng = np.random.default_rng(2)
    pts = rng.random((50, dim))
    pts = pts[pts.sum(1) <= 1]
    v, g = e.tabulate(pts)
    assert np.allclose(v.sum(1), 1.0, atol=1e-11)
    assert np.allclose(g.sum(1), 0.0, atol=1e-9)
    # the space contains P_k: the interpolant of a random P_k polynomial is exact
    f = random_poly(dim, k, rng)
    assert np.allclose(v @ f(e.nodes), f(pts), atol=1e-10)
    # D differentiates nodal values of x_r exactly
    for r in range(dim):
        gr = np.einsum("qas,a->qs", e.D, e.nodes[:, r])
        expect = np.zeros_like(gr)
        expect[:, r] = 1.0
        assert np.allclose(gr, expect, atol=1e-10)


@pytest.mark.parametrize("dk", ALL)
def test_gradient_table_vs_finite_differences(dk):
    dim, _ = dk
    e = kmv_element(*dk)
    rng = np.random.default_rng(3)
    p = rng.random((6, dim)) * 0.5 / dim + 0.1
    h = 1e-6
    _, g = e.tabulate(p)
    for r in range(dim):
        dp = np.zeros(dim)
        dp[r] = h
        vp, _ = e.tabulate(p + dp)
        vm, _ = e.tabulate(p - dp)
        assert np.allclose((vp - vm) / (2 * h), g[:, :, r], atol=1e-6)


@pytest.mark.parametrize("dk", ALL)
def test_unisolvent(dk):
    e = kmv_element(*dk)
    assert np.isfinite(e.vandermonde_cond) and e.vandermonde_cond < 1e10
