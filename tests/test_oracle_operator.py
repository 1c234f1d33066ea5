"""Pins of the oracle's local stiffness action w = D^T G D u (paper section
4.2.1, factored stiffness operator; the hot kernel of section 4.2.2).

Checks, each of which a plausible slip (dropped cross term, wrong sign,
transposed D, swapped index) fails:
  1. exact differentiation: on affine meshes and u in Q_{N-1} the interior
     rows of the assembled operator equal B (-Laplace u) at the node;
  2. symmetry and positive semi-definiteness;
  3. the constant null space of the Neumann operator (curved mesh, kappa);
  4. brute force: the assembled operator equals the sparse matrix built
     from explicit Lagrange-derivative element matrices on 2x2x2 meshes;
plus the N=1 reduction to h times the 7-point Laplacian stencil and the
Jacobi-diagonal formula."""
import numpy as np
import pytest

from oracle import oracle as orc
from seminputs import grf_features, uniform


def _dense_global(m):
    """Q^T A_L Q (masked when m is Dirichlet) by applying the fast oracle
    operator to every unit vector."""
    A = np.zeros((m.nG, m.nG))
    e = np.zeros(m.nG)
    for g in range(m.nG):
        e[g] = 1.0
        A[:, g] = orc.apply_global(m, e)
        e[g] = 0.0
    return A


def _kappa_params(seed=7, M=64):
    omega, b, sigma = grf_features(seed=seed, M=M, ell=0.3, sigma=0.5)
    return omega, b, sigma


def test_n1_is_h_times_seven_point_stencil():
    n = 4
    m = orc.mesh(1, n, n, n, orc.MAP_AFFINE, dirichlet=0)
    A = _dense_global(m)
    h = 1.0 / n
    Gd = n + 1
    for gz in range(1, Gd - 1):
        for gy in range(1, Gd - 1):
            for gx in range(1, Gd - 1):
                g = gx + Gd * (gy + Gd * gz)
                row = A[g].copy()
                assert abs(row[g] - 6 * h) < 1e-14
                for d in (1, Gd, Gd * Gd):
                    assert abs(row[g + d] + h) < 1e-14
                    assert abs(row[g - d] + h) < 1e-14
                    row[g + d] = row[g - d] = 0
                row[g] = 0
                assert np.max(np.abs(row)) < 1e-14


POLYS = [
    # (u, -Laplace u), all of degree <= 3 per variable
    (lambda x, y, z: x ** 2, lambda x, y, z: -2.0 + 0 * x),
    (lambda x, y, z: x * y * z, lambda x, y, z: 0 * x),
    (lambda x, y, z: x ** 2 - y ** 2, lambda x, y, z: 0 * x),
    (lambda x, y, z: x ** 3 * y + z ** 2 * y, lambda x, y, z: -6 * x * y - 2 * y),
    (lambda x, y, z: (x * y * z) ** 3, lambda x, y, z:
     -6 * x * (y * z) ** 3 - 6 * y * (x * z) ** 3 - 6 * z * (x * y) ** 3),
]


@pytest.mark.parametrize("k", range(len(POLYS)))
def test_exact_on_polynomials_affine(k):
    """GLL quadrature with N+1 points is exact to degree 2N-1, so for
    u in Q_{N-1} every interior row of the assembled Neumann operator equals
    the assembled lumped mass times -Laplace u at that node."""
    N = 4
    u_f, lap_f = POLYS[k]
    m = orc.mesh(N, 3, 2, 4, orc.MAP_AFFINE, dirichlet=0)
    Xg = np.zeros((3, m.nG))
    Xg[:, m.l2g] = m.X
    u = u_f(*Xg)
    Au = orc.apply_global(m, u)
    Bg = orc.to_global(m, orc.gs(m, m.B))
    ref = Bg * lap_f(*Xg)
    interior = np.all((Xg > 1e-12) & (Xg < 1 - 1e-12), axis=0)
    scale = np.max(np.abs(orc.to_global(m, orc.ax_abs(m, orc.to_local(m, u)))))
    err = np.max(np.abs(Au[interior] - ref[interior]))
    assert err < 1e-13 * scale, (err, scale)


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7])
def test_neumann_constant_null_space_curved_kappa(N):
    m = orc.mesh(N, 3, 2, 2, orc.MAP_SINE_CYCLIC, dirichlet=0,
                 kappa_params=_kappa_params())
    one = np.ones(m.nL)
    w = orc.ax(m, one)
    bound = orc.ax_abs(m, one)
    assert np.max(np.abs(w) / bound) < 1e-14 * (N + 1) ** 2


@pytest.mark.parametrize("N", [2, 4, 7])
@pytest.mark.parametrize("dirichlet", [0, 1])
def test_symmetry_random_vectors(N, dirichlet):
    m = orc.mesh(N, 2, 3, 2, orc.MAP_SINE_CYCLIC, dirichlet=dirichlet,
                 kappa_params=_kappa_params())
    u = uniform(m.nG, seed=1)
    v = uniform(m.nG, seed=2)
    Au, Av = orc.apply_global(m, u), orc.apply_global(m, v)
    scale = np.linalg.norm(u) * np.linalg.norm(v) * np.max(
        np.abs(orc.ax_abs(m, np.ones(m.nL))))
    assert abs(v @ Au - u @ Av) < 1e-13 * scale


def test_local_operator_symmetric_per_element():
    """w = D^T G D u is symmetric element by element (discontinuous
    inputs), which fails if one contraction stage is transposed."""
    m = orc.mesh(3, 2, 1, 1, orc.MAP_SINE_CYCLIC, dirichlet=0,
                 kappa_params=_kappa_params())
    u = uniform(m.nL, seed=1)
    v = uniform(m.nL, seed=2)
    a = v @ orc.ax(m, u)
    b = u @ orc.ax(m, v)
    assert abs(a - b) < 1e-13 * abs(a)
    assert u @ orc.ax(m, u) > 0


@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7])
def test_brute_force_2x2x2(N):
    """Fast operator == SciPy assembly of dense element matrices built from
    explicit basis derivatives (no sum factorisation), on a curved mesh with
    variable kappa; plus PSD and the one-dimensional Neumann null space."""
    m = orc.mesh(N, 2, 2, 2, orc.MAP_SINE_CYCLIC, dirichlet=0,
                 kappa_params=_kappa_params())
    A_fast = _dense_global(m)
    A_brute = orc.assemble_sparse(m).toarray()
    amax = np.max(np.abs(A_brute))
    assert np.max(np.abs(A_fast - A_brute)) < 1e-13 * amax
    if N <= 5:
        lam = np.linalg.eigvalsh(0.5 * (A_brute + A_brute.T))
        assert lam[0] > -1e-12 * lam[-1]
        assert np.sum(lam < 1e-10 * lam[-1]) == 1          # constants only
        md = orc.mesh(N, 2, 2, 2, orc.MAP_SINE_CYCLIC, dirichlet=1,
                      kappa_params=_kappa_params())
        Ad = orc.assemble_sparse(md).toarray()
        free = np.ones(md.nG, bool)
        free[md.l2g[md.bmask.astype(bool)]] = False
        lam_d = np.linalg.eigvalsh(Ad[np.ix_(free, free)])
        assert lam_d[0] > 1e-8 * lam_d[-1]                  # interior SPD


@pytest.mark.parametrize("N", [1, 3, 7])
def test_diagonal_formula_matches_brute_force(N):
    m = orc.mesh(N, 2, 2, 2, orc.MAP_SINE_CYCLIC, dirichlet=0,
                 kappa_params=_kappa_params())
    d = orc.local_diag(m)
    n3 = m.n1 ** 3
    for e in range(m.E):
        Ae = orc.brute_element_matrix(N, m.xi, m.G[e])
        np.testing.assert_allclose(d[e * n3:(e + 1) * n3], np.diag(Ae),
                                   rtol=1e-12, atol=1e-14 * np.abs(Ae).max())


def test_abs_bound_dominates():
    m = orc.mesh(5, 2, 2, 1, orc.MAP_SINE_CYCLIC, dirichlet=0,
                 kappa_params=_kappa_params())
    u = uniform(m.nL, seed=9)
    assert np.all(np.abs(orc.ax(m, u)) <= orc.ax_abs(m, u) * (1 + 1e-12))
