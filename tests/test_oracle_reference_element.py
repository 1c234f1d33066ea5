"""Pins of the oracle's reference element: GLL nodes/weights and the nodal
derivative matrix (paper section 4.2.1: tensor-product Lagrange basis on the
1D Gauss-Lobatto-Legendre nodes), checked against closed forms, quadrature
exactness and independently differentiated Lagrange polynomials."""
import math
import os

import numpy as np
import pytest

from oracle import oracle as orc

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _eval(expr):
    return float(eval(expr, {"sqrt": math.sqrt, "__builtins__": {}}))


def _read(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append([c.strip() for c in line.split(";")])
    return rows


@pytest.mark.parametrize("row", _read("gll_closed_forms.txt"))
def test_gll_closed_forms(row):
    N = int(row[0])
    xs = [_eval(t) for t in row[1].split(",")]
    ws = [_eval(t) for t in row[2].split(",")]
    xi, w = orc.gll(N)
    np.testing.assert_allclose(xi, xs, rtol=0, atol=2e-16)
    np.testing.assert_allclose(w, ws, rtol=2e-15, atol=0)


@pytest.mark.parametrize("row", _read("dhat_closed_forms.txt"))
def test_dhat_closed_forms(row):
    N = int(row[0])
    ref = np.array([[_eval(t) for t in r.split(",")] for r in row[1].split("|")])
    D = orc.dmat(N)
    np.testing.assert_allclose(D, ref, rtol=0, atol=1e-15)


@pytest.mark.parametrize("N", range(1, 17))
def test_gll_quadrature_exactness(N):
    xi, w = orc.gll(N)
    assert abs(w.sum() - 2.0) < 1e-14
    # exact for x^p, p <= 2N-1; integral over [-1,1] is 2/(p+1) for even p
    for p in range(0, 2 * N):
        exact = 0.0 if p % 2 else 2.0 / (p + 1)
        assert abs(np.dot(w, xi ** p) - exact) < 1e-13, (N, p)
    # and not exact at p = 2N (the rule has degree 2N-1)
    if N <= 8:
        p = 2 * N
        assert abs(np.dot(w, xi ** p) - 2.0 / (p + 1)) > 1e-9


@pytest.mark.parametrize("N", range(2, 17))
def test_gll_interior_nodes_are_roots_of_dPN(N):
    xi, _ = orc.gll(N)
    dP = np.polynomial.legendre.Legendre.basis(N).deriv()
    assert np.all(np.abs(dP(xi[1:-1])) < 1e-10 * np.abs(dP(0.3)) + 1e-12)
    assert np.all(np.diff(xi) > 0)
    np.testing.assert_array_equal(xi, -xi[::-1])


@pytest.mark.parametrize("N", range(1, 13))
def test_dhat_differentiates_polynomials_exactly(N):
    """D applied to nodal values of x^p gives p x^(p-1) for p <= N."""
    xi, _ = orc.gll(N)
    D = orc.dmat(N, xi)
    for p in range(0, N + 1):
        d = D @ xi ** p
        ref = p * xi ** (p - 1) if p > 0 else np.zeros_like(xi)
        assert np.max(np.abs(d - ref)) < 1e-12 * max(1.0, N * N), (N, p)


@pytest.mark.parametrize("N", range(1, 13))
def test_dhat_matches_differentiated_lagrange_polynomials(N):
    xi, _ = orc.gll(N)
    D = orc.dmat(N, xi)
    L = orc.lagrange_derivs_at_nodes(xi)  # L[a][m] = l_a'(xi_m)
    np.testing.assert_allclose(D, L.T, rtol=0, atol=1e-10 * N * N)
