"""Pins of the oracle's learned coarse correction: the element-interior
node list, the bubble basis against its closed form and the reference
scaling, the Galerkin coarse matrix from the dense element matrix against
the sum-factorised operator (an independent code path), the factor loss and
its backpropagation against central differences, the normalised coarse
target and the correction against what they must reproduce (coarse-space
solutions exactly, Galerkin orthogonality, zero face values, invariance of
the normalised inverse under scaling of kappa and of the element), and the
reading behind the layout: the exact element coarse correction needs
clearly fewer flexible-CG iterations than Jacobi."""
import numpy as np
import pytest

from oracle import mlp
from oracle import oracle as orc
from seminputs import fourier_modes, grf_features, uniform


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7])
def test_interior_nodes(N):
    n1 = N + 1
    I = mlp.interior_nodes(N)
    assert I.shape[0] == max(N - 1, 0) ** 3
    assert np.all(np.diff(I) > 0)
    i, j, k = I % n1, (I // n1) % n1, I // (n1 * n1)
    for c in (i, j, k):
        assert np.all((c >= 1) & (c <= N - 1))
    if N == 2:
        assert list(I) == [1 + 3 * (1 + 3 * 1)]


def _curved_mesh(N, n=2):
    kap = grf_features(seed=3, M=256, ell=0.5, sigma=0.7)
    return orc.mesh(N, n, n, n, orc.MAP_SINE_CYCLIC, 1, kap)


# ---------------------------------------------------------------------------
# coarse layout: bubble basis, Galerkin coarse matrices, factor loss
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("N", [2, 3, 5, 7])
def test_bubble_basis(N):
    xi, _ = orc.gll(N)
    B = mlp.bubble_basis(N, xi, scaled=False)
    p = mlp.coarse_degree(N)
    assert B.shape == ((N - 1) ** 3, (p + 1) ** 3)
    # first column: the product (1-x^2)(1-y^2)(1-z^2) at the interior nodes
    m = N - 1
    q = np.arange(m ** 3)
    x, y, z = xi[1 + q % m], xi[1 + (q // m) % m], xi[1 + q // (m * m)]
    assert np.allclose(B[:, 0], (1 - x ** 2) * (1 - y ** 2) * (1 - z ** 2), atol=1e-15)
    if p >= 1:   # column (a, b, c) = (1, 0, 0): P_1(x) = x
        assert np.allclose(B[:, 1], x * (1 - x ** 2) * (1 - y ** 2) * (1 - z ** 2),
                           atol=1e-15)
    assert np.linalg.matrix_rank(B) == B.shape[1]
    # scaled basis: the unit reference element's coarse inverse has unit
    # diagonal (and the scaling is positive and per column)
    Bs = mlp.bubble_basis(N, xi)
    s = Bs[0] / B[0]
    assert np.all(s > 0) and np.allclose(Bs, B * s[None, :], rtol=1e-14, atol=0)
    ref = orc.mesh(N, 1, 1, 1, orc.MAP_AFFINE, 0, None)
    I = mlp.interior_nodes(N)
    A_II = orc.brute_element_matrix(N, ref.xi, ref.G[0])[np.ix_(I, I)]
    assert np.allclose(np.diag(np.linalg.inv(Bs.T @ A_II @ Bs)), 1.0, atol=1e-12)


@pytest.mark.parametrize("N", [3, 5])
def test_coarse_galerkin_against_operator(N):
    """G_e = B^T A_II B from the dense element matrix equals the same
    quantity from the sum-factorised operator applied to the bubbles."""
    m = _curved_mesh(N)
    n3 = m.n1 ** 3
    I = mlp.interior_nodes(N)
    B = mlp.bubble_basis(N, m.xi)
    e = 1
    G = mlp.coarse_galerkin(orc.brute_element_matrix(N, m.xi, m.G[e]), N, m.xi)
    cols = []
    for k in range(B.shape[1]):
        u = np.zeros(n3)
        u[I] = B[:, k]
        cols.append(B.T @ orc.ax_raw(N, m.D, m.G[e:e + 1], u)[I])
    G2 = np.stack(cols, 1)
    assert np.max(np.abs(G - G2)) <= 1e-12 * np.max(np.abs(G))
    assert np.allclose(G, G.T, rtol=0, atol=1e-12 * np.max(np.abs(G)))
    assert np.min(np.linalg.eigvalsh(G)) > 0


def test_factor_loss_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    K, S = 4, 3
    O = rng.standard_normal((S, K * (K + 1) // 2))
    Y = rng.standard_normal((S, K))
    A = rng.standard_normal((S, K))
    loss, dO = mlp.factor_loss_and_grad(O, Y, A)
    hh = 1e-6
    fd = np.zeros_like(O)
    for s_ in range(S):
        for q in range(O.shape[1]):
            Op = O.copy(); Op[s_, q] += hh
            Om = O.copy(); Om[s_, q] -= hh
            fd[s_, q] = (mlp.factor_loss_and_grad(Op, Y, A)[0]
                         - mlp.factor_loss_and_grad(Om, Y, A)[0]) / (2 * hh)
    assert np.max(np.abs(fd - dO)) <= 1e-7 * max(1.0, np.max(np.abs(dO)))
    # an exact factor gives zero loss
    M = np.eye(K) * 2.0 + 0.1
    L = np.linalg.cholesky(M)
    Ot = np.tile(L[np.tril_indices(K)], (S, 1))
    loss0, _ = mlp.factor_loss_and_grad(Ot, Y, Y @ M.T)
    assert loss0 < 1e-28


def test_exact_coarse_correction_beats_jacobi():
    """The reading behind the coarse layout: the exact element coarse
    correction (bubble Galerkin) needs fewer iterations than Jacobi."""
    N, n = 5, 3
    kap = grf_features(seed=7, M=512, ell=0.6, sigma=1.0)
    m = orc.mesh(N, n, n, n, orc.MAP_AFFINE, 1, kap)
    n3 = m.n1 ** 3
    I = mlp.interior_nodes(N)
    B = mlp.bubble_basis(N, m.xi)
    k, a, phi = fourier_modes(seed=900)
    b = orc.to_global(m, orc.rhs_local(m, orc.src_fourier(m.X, k, a, phi)))
    dinv = orc.jacobi_dinv_global(m)
    Ms = [np.linalg.inv(mlp.coarse_galerkin(orc.brute_element_matrix(N, m.xi, m.G[e]),
                                            N, m.xi)) for e in range(m.E)]
    gI = [m.l2g[e * n3 + I] for e in range(m.E)]

    def prec(r):
        z = dinv * r
        for e in range(m.E):
            z[gI[e]] += B @ (Ms[e] @ (B.T @ r[gI[e]]))
        return z

    _, st_j, it_j, _ = orc.pcg(m, b, 1e-8, 5000)
    _, st_c, it_c, _ = orc.fcg(m, b, prec, 1e-8, 5000)
    assert st_j == 0 and st_c == 0
    assert it_c < 0.9 * it_j, (it_c, it_j)


def test_factor_network_gradient_matches_central_differences():
    rng = np.random.default_rng(4)
    K, nin, nh, S = 3, 5, 6, 4
    no = K * (K + 1) // 2
    theta = rng.standard_normal(mlp.n_params(nin, nh, no)) * 0.5
    X = rng.standard_normal((S, nin))
    Y = rng.standard_normal((S, K))
    A = rng.standard_normal((S, K))
    loss, g = mlp.factor_net_loss_and_grad(theta, X, Y, A, nin, nh, K)
    hh = 1e-6
    fd = np.zeros_like(theta)
    for q in range(theta.size):
        tp = theta.copy(); tp[q] += hh
        tm = theta.copy(); tm[q] -= hh
        fd[q] = (mlp.factor_net_loss_and_grad(tp, X, Y, A, nin, nh, K)[0]
                 - mlp.factor_net_loss_and_grad(tm, X, Y, A, nin, nh, K)[0]) / (2 * hh)
    assert np.max(np.abs(fd - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))


def _vertex_kappa(m, e):
    n1, N, n3 = m.n1, m.N, m.n1 ** 3
    return np.array([m.kappa[e * n3 + (v & 1) * N + n1 * ((v >> 1) & 1) * N
                             + n1 * n1 * (v >> 2) * N] for v in range(8)])


@pytest.mark.parametrize("N", [3, 5, 7])
def test_coarse_correction_reproduces_coarse_space_solutions(N):
    """If the element-interior solution of A_II d = r_I lies in the coarse
    space (d = B y), the exact coarse correction returns it: c_I = B y, zero
    on the faces.  The kappa_mean h of the target and the 1 / (kappa_mean h)
    of the correction cancel for any vertex values and element size; a
    swapped B / B^T, a dropped factor or a wrong index fails this."""
    m = _curved_mesh(N)
    n3 = m.n1 ** 3
    I = mlp.interior_nodes(N)
    B = mlp.bubble_basis(N, m.xi)
    rng = np.random.default_rng(N)
    for e in (0, m.E - 1):
        A_e = orc.brute_element_matrix(N, m.xi, m.G[e])
        A_II = A_e[np.ix_(I, I)]
        y = rng.standard_normal(B.shape[1])
        r_e = uniform(n3, seed=40 + e)     # face values must not enter
        r_e[I] = A_II @ (B @ y)
        kv = np.exp(rng.standard_normal(8))
        h = 0.37
        M = mlp.coarse_target(A_e, N, m.xi, kv, h)
        c = mlp.coarse_correction(r_e, M, N, m.xi, kv, h)
        faces = np.setdiff1d(np.arange(n3), I)
        assert np.all(c[faces] == 0.0)
        err = np.max(np.abs(c[I] - B @ y)) / np.max(np.abs(B @ y))
        assert err <= 1e-10, err
        # damping scales the correction
        c2 = mlp.coarse_correction(r_e, M, N, m.xi, kv, h, damping=0.25)
        np.testing.assert_allclose(c2, 0.25 * c, rtol=1e-14, atol=0)


@pytest.mark.parametrize("N", [3, 5])
def test_coarse_correction_galerkin_orthogonality(N):
    """For any residual, c_I is in the coarse space and the interior
    residual left by it is orthogonal to the coarse space:
    B^T (r_I - A_II c_I) = 0 (the defining property of the Galerkin
    projection of A_II^{-1} r_I onto span B)."""
    m = _curved_mesh(N)
    n3 = m.n1 ** 3
    I = mlp.interior_nodes(N)
    B0 = mlp.bubble_basis(N, m.xi, scaled=False)
    e = 2
    A_e = orc.brute_element_matrix(N, m.xi, m.G[e])
    A_II = A_e[np.ix_(I, I)]
    r_e = uniform(n3, seed=7)
    kv = _vertex_kappa(m, e)
    c = mlp.coarse_correction(r_e, mlp.coarse_target(A_e, N, m.xi, kv, 0.5),
                              N, m.xi, kv, 0.5)
    res = B0.T @ (r_e[I] - A_II @ c[I])
    assert np.max(np.abs(res)) <= 1e-11 * np.max(np.abs(B0.T @ r_e[I]))
    coef, *_ = np.linalg.lstsq(B0, c[I], rcond=None)
    assert np.max(np.abs(B0 @ coef - c[I])) <= 1e-11 * np.max(np.abs(c[I]))


@pytest.mark.parametrize("N", [2, 4, 7])
def test_normalised_target_is_scale_invariant(N):
    """On affine cube elements with constant kappa the stiffness is
    kappa h times that of the unit reference cube, so the normalised
    inverse kappa h G_e^{-1} equals the reference one for every kappa and
    every element size -- and the reference has unit diagonal in the
    scaled basis."""
    ref = None
    for n, kap in ((1, 1.0), (3, 1.0), (2, 7.5), (4, 0.2)):
        m = orc.mesh(N, n, n, n, orc.MAP_AFFINE, 1, None)
        e = m.E // 2
        A_e = kap * orc.brute_element_matrix(N, m.xi, m.G[e])
        M = mlp.coarse_target(A_e, N, m.xi, np.full(8, kap), 1.0 / n)
        if ref is None:
            ref = M
            np.testing.assert_allclose(np.diag(M), 1.0, rtol=1e-11)
        np.testing.assert_allclose(M, ref, rtol=1e-10, atol=1e-12)
