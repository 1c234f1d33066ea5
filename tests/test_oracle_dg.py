"""Pins of the DG shallow-water volume-term oracle (paper section 4.3).

Independent checks, chosen so that a slip in the nodes, the basis, the
matrices, the affine map, the fluxes or the source fails one of them:
  * nodes: N = 1 vertices, N = 2 vertices and edge midpoints, edge nodes at
    the Gauss-Lobatto points, invariance under the triangle's symmetries;
  * basis: orthonormal under collapsed-coordinate Gauss quadrature;
  * mass matrix and weak derivatives: exact rational integrals of monomials
    over the reference triangle;
  * Dr, Ds: exact derivatives of polynomials of degree <= N;
  * affine factors: J = area / 2 and the inverse-Jacobian identities;
  * the whole volume term: for polynomial states (constant depth, polynomial
    momenta and bathymetry) every weak volume integral against a monomial
    test function equals its value by Gauss quadrature on the physical
    triangle."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import dg


def _exact_tri(a, b):
    """Exact integral of r^a s^b over the reference triangle (vertices
    (-1,-1), (1,-1), (-1,1)): r = 2x - 1, s = 2y - 1 on the unit triangle,
    where x^p y^q integrates to p! q! / (p + q + 2)!."""
    tot = Fraction(0)
    for p in range(a + 1):
        for q in range(b + 1):
            c = (math.comb(a, p) * math.comb(b, q) * 2 ** (p + q)
                 * (-1) ** (a - p + b - q))
            tot += c * Fraction(math.factorial(p) * math.factorial(q),
                                math.factorial(p + q + 2))
    return tot * 4  # dr ds = 4 dx dy


def _duffy_rule(q):
    """Collapsed-coordinate Gauss rule on the reference triangle: exact for
    polynomials of total degree <= 2q - 2."""
    x, w = np.polynomial.legendre.leggauss(q)
    A, Bq = np.meshgrid(x, x, indexing="ij")
    WA, WB = np.meshgrid(w, w, indexing="ij")
    r = (1 + A) * (1 - Bq) / 2 - 1
    s = Bq
    wt = WA * WB * (1 - Bq) / 2
    return r.ravel(), s.ravel(), wt.ravel()


def test_nodes_low_order_closed_forms():
    r, s = dg.nodes(1)
    np.testing.assert_allclose(np.c_[r, s], [[-1, -1], [1, -1], [-1, 1]],
                               atol=1e-15)
    r, s = dg.nodes(2)
    ref = {(-1, -1), (0, -1), (1, -1), (-1, 0), (0, 0), (-1, 1)}
    got = {(round(a, 12) + 0.0, round(b, 12) + 0.0) for a, b in zip(r, s)}
    assert got == {(float(a), float(b)) for a, b in ref}


@pytest.mark.parametrize("N", range(1, 9))
def test_edge_nodes_are_gauss_lobatto_and_set_is_symmetric(N):
    r, s = dg.nodes(N)
    assert len(r) == dg.num_nodes(N)
    gl = dg.gauss_lobatto(N)
    edge = np.sort(r[np.abs(s + 1) < 1e-12])
    np.testing.assert_allclose(edge, gl, atol=1e-13)
    # barycentric coordinates; every permutation maps the set onto itself
    lam = np.c_[(s + 1) / 2, -(r + s) / 2, (r + 1) / 2]
    key = lambda L: np.array(sorted(map(tuple, np.round(L, 11))))
    base = key(lam)
    for perm in itertools.permutations(range(3)):
        np.testing.assert_allclose(key(lam[:, perm]), base, atol=1e-10)
    # inside the triangle
    assert np.all(lam > -1e-13)


@pytest.mark.parametrize("N", [1, 3, 6, 8])
def test_basis_orthonormal(N):
    r, s, w = _duffy_rule(N + 3)
    V = dg.vandermonde(N, r, s)
    G = V.T @ (w[:, None] * V)
    np.testing.assert_allclose(G, np.eye(dg.num_nodes(N)), atol=1e-12)


def _monomials(N):
    return [(a, b) for a in range(N + 1) for b in range(N + 1 - a)]


@pytest.mark.parametrize("N", [1, 2, 4, 7, 8])
def test_mass_matrix_exact_on_monomials(N):
    ops = dg.reference_operators(N)
    r, s, M = ops["r"], ops["s"], ops["M"]
    mons = _monomials(N)
    for (a, b), (c, d) in itertools.product(mons[::2], mons[::3]):
        got = (r ** a * s ** b) @ M @ (r ** c * s ** d)
        ref = float(_exact_tri(a + c, b + d))
        assert abs(got - ref) < 1e-12 * max(1.0, abs(ref)), (a, b, c, d)
    assert abs(np.ones_like(r) @ M @ np.ones_like(r) - 2.0) < 1e-13


@pytest.mark.parametrize("N", [1, 3, 5, 8])
def test_derivative_matrices_exact(N):
    ops = dg.reference_operators(N)
    r, s = ops["r"], ops["s"]
    for a, b in _monomials(N):
        f = r ** a * s ** b
        fr = a * r ** max(a - 1, 0) * s ** b if a else 0 * r
        fs = b * r ** a * s ** max(b - 1, 0) if b else 0 * r
        np.testing.assert_allclose(ops["Dr"] @ f, fr, atol=1e-11 * (N + 1) ** 2)
        np.testing.assert_allclose(ops["Ds"] @ f, fs, atol=1e-11 * (N + 1) ** 2)


@pytest.mark.parametrize("N", [2, 4, 8])
def test_weak_derivatives_integrate_by_parts(N):
    """g^T M (Drw f) = integral of (dg/dr) f, and likewise in s, for
    monomials f, g of degree <= N (exact rationals on the right)."""
    ops = dg.reference_operators(N)
    r, s, M = ops["r"], ops["s"], ops["M"]
    mons = _monomials(N)
    for (a, b), (c, d) in itertools.product(mons[::3], mons[::2]):
        f, g = r ** a * s ** b, r ** c * s ** d
        lhs_r = g @ M @ (ops["Drw"] @ f)
        lhs_s = g @ M @ (ops["Dsw"] @ f)
        ref_r = c * _exact_tri(a + c - 1, b + d) if c else Fraction(0)
        ref_s = d * _exact_tri(a + c, b + d - 1) if d else Fraction(0)
        assert abs(lhs_r - float(ref_r)) < 1e-11, (a, b, c, d)
        assert abs(lhs_s - float(ref_s)) < 1e-11, (a, b, c, d)


def test_affine_factors():
    rng = np.random.default_rng(3)
    vx, vy = rng.uniform(-1, 1, 30), rng.uniform(-1, 1, 30)
    etov = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8], [9, 10, 11]])
    # make every triangle counterclockwise
    for e in etov:
        a, b, c = e
        if (vx[b] - vx[a]) * (vy[c] - vy[a]) - (vx[c] - vx[a]) * (vy[b] - vy[a]) < 0:
            e[1], e[2] = e[2], e[1]
    rx, sx, ry, sy, J = dg.geometric_factors(vx, vy, etov)
    for k, (a, b, c) in enumerate(etov):
        area = 0.5 * ((vx[b] - vx[a]) * (vy[c] - vy[a])
                      - (vx[c] - vx[a]) * (vy[b] - vy[a]))
        assert abs(J[k] - area / 2) < 1e-14
        xr, xs = (vx[b] - vx[a]) / 2, (vx[c] - vx[a]) / 2
        yr, ys = (vy[b] - vy[a]) / 2, (vy[c] - vy[a]) / 2
        np.testing.assert_allclose([[rx[k], sx[k]], [ry[k], sy[k]]] @
                                   np.array([[xr, yr], [xs, ys]]),
                                   np.eye(2), atol=1e-12)


@pytest.mark.parametrize("N", [2, 4, 6, 8])
def test_volume_term_against_quadrature(N):
    """Constant depth h0, momenta of degree <= N // 2 and bathymetry of
    degree <= N: the fluxes and the source are polynomials of degree <= N, so
    the nodal volume term is exact.  For monomial test functions v(x, y) of
    degree <= N: v^T (J M) rhs = integral over the element of
    F v_x + G v_y + S v (Gauss quadrature on the physical triangle)."""
    g, h0 = 9.81, 2.0
    ops = dg.reference_operators(N)
    vx = np.array([0.1, 1.3, 0.4, 1.6])
    vy = np.array([-0.2, 0.1, 1.1, 1.4])
    etov = np.array([[0, 1, 2], [1, 3, 2]])
    geo = dg.geometric_factors(vx, vy, etov)
    X, Y = dg.physical_nodes(ops, vx, vy, etov)
    p = N // 2
    hu_f = lambda x, y: 0.3 + 0.2 * x ** p - 0.1 * y ** max(p - 1, 0) * x
    hv_f = lambda x, y: -0.1 + 0.15 * y ** p + 0.05 * x * y ** max(p - 1, 0)
    B_f = lambda x, y: 0.2 * x ** N - 0.1 * (x * y) ** (N // 2) + 0.05 * y
    Bx_f = lambda x, y: 0.2 * N * x ** (N - 1) - 0.1 * (N // 2) * x ** max(N // 2 - 1, 0) * y ** (N // 2)
    By_f = lambda x, y: -0.1 * (N // 2) * y ** max(N // 2 - 1, 0) * x ** (N // 2) + 0.05
    Q = np.stack([np.full_like(X, h0), hu_f(X, Y), hv_f(X, Y)], axis=1)
    Bx, By = dg.bathymetry_gradient(ops, geo, B_f(X, Y))
    np.testing.assert_allclose(Bx, Bx_f(X, Y), atol=1e-10)
    np.testing.assert_allclose(By, By_f(X, Y), atol=1e-10)
    rhs = dg.volume_rhs(ops, geo, Q, Bx, By, g)
    rq, sq, wq = _duffy_rule(N + 3)
    rx, sx, ry, sy, J = geo
    for e in range(2):
        a, b, c = etov[e]
        xq = -(rq + sq) / 2 * vx[a] + (1 + rq) / 2 * vx[b] + (1 + sq) / 2 * vx[c]
        yq = -(rq + sq) / 2 * vy[a] + (1 + rq) / 2 * vy[b] + (1 + sq) / 2 * vy[c]
        hu, hv = hu_f(xq, yq), hv_f(xq, yq)
        F = [hu, hu * hu / h0 + 0.5 * g * h0 * h0, hu * hv / h0]
        G = [hv, hu * hv / h0, hv * hv / h0 + 0.5 * g * h0 * h0]
        S = [0 * xq, -g * h0 * Bx_f(xq, yq), -g * h0 * By_f(xq, yq)]
        for (ka, kb) in [(0, 0), (1, 0), (0, 1), (N, 0), (1, N - 1), (0, N)]:
            v = xq ** ka * yq ** kb
            vxq = ka * xq ** max(ka - 1, 0) * yq ** kb
            vyq = kb * xq ** ka * yq ** max(kb - 1, 0)
            vn = X[e] ** ka * Y[e] ** kb
            for q in range(3):
                ref = np.sum(wq * J[e] * (F[q] * vxq + G[q] * vyq + S[q] * v))
                got = vn @ (J[e] * ops["M"]) @ rhs[e, q]
                # magnitude of the integrand's terms, floored by the fluxes'
                # own size (the exact value can vanish, e.g. q = 0, v = 1)
                scale = np.sum(wq * J[e] * (
                    (np.abs(F[q]) + np.abs(G[q]) + np.abs(S[q]))
                    * (1 + np.abs(v) + np.abs(vxq) + np.abs(vyq))))
                assert abs(got - ref) < 1e-11 * scale, (N, e, ka, kb, q, got, ref)
