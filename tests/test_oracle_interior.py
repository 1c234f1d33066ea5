"""Pins of the oracle's interior layout of the learned correction: the
element-interior node list, the dense element-interior solve against the
sum-factorised operator (an independent code path), the target's closed
form on a known solution, and the reading that the exact element-interior
block solve converges in fewer flexible-CG iterations than Jacobi."""
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


@pytest.mark.parametrize("N", [2, 4, 7])
def test_interior_solve_against_operator(N):
    m = _curved_mesh(N)
    n3 = m.n1 ** 3
    I = mlp.interior_nodes(N)
    for e in (0, m.E - 1):
        A_e = orc.brute_element_matrix(N, m.xi, m.G[e])
        r_e = uniform(n3, seed=10 + e)
        d = mlp.interior_solve(A_e, r_e, N)
        u = np.zeros(n3)
        u[I] = d
        w = orc.ax_raw(N, m.D, m.G[e:e + 1], u)
        err = np.max(np.abs(w[I] - r_e[I])) / np.max(np.abs(r_e[I]))
        assert err < 1e-10


def test_interior_target_known_solution():
    N = 5
    m = _curved_mesh(N)
    n3 = m.n1 ** 3
    I = mlp.interior_nodes(N)
    e = 3
    A_e = orc.brute_element_matrix(N, m.xi, m.G[e])
    v = uniform(I.shape[0], seed=4)
    r_e = uniform(n3, seed=5)          # face values do not enter
    r_e[I] = A_e[np.ix_(I, I)] @ v
    dinv_e = 1.0 / np.abs(uniform(n3, seed=6) + 2.0)
    kv = np.array([1.0, 2.0, 0.5, 1.5, 1.0, 1.0, 3.0, 0.25])
    h = 0.5
    s = np.linalg.norm(r_e[I])
    t = mlp.interior_target(A_e, r_e, dinv_e, kv, h, N)
    want = (v - dinv_e[I] * r_e[I]) * kv.mean() * h / s
    assert np.max(np.abs(t - want)) < 1e-9 * np.max(np.abs(want))
    # the correction undoes the scaling: dinv r + c = d on the interior
    c = mlp.interior_correction(t, s, kv, h, N)
    assert np.max(np.abs(dinv_e[I] * r_e[I] + c[I] - v)) < 1e-9 * np.max(np.abs(v))
    assert np.all(c[np.setdiff1d(np.arange(n3), I)] == 0.0)
    x, s2 = mlp.interior_features(r_e, kv, N)
    assert s2 == s and np.allclose(x[:I.shape[0]] * s, r_e[I], rtol=0, atol=1e-14 * s)
    assert np.allclose(x[I.shape[0]:], np.log(kv) - np.log(kv).mean())


def test_exact_interior_block_beats_jacobi():
    """The reading behind the interior layout: a perfect network reproduces
    the element-interior block solve, which needs clearly fewer flexible-CG
    iterations than Jacobi-PCG on a variable-coefficient problem."""
    N, n = 5, 3
    kap = grf_features(seed=7, M=512, ell=0.6, sigma=1.0)
    m = orc.mesh(N, n, n, n, orc.MAP_AFFINE, 1, kap)
    n3 = m.n1 ** 3
    I = mlp.interior_nodes(N)
    k, a, phi = fourier_modes(seed=900)
    b = orc.to_global(m, orc.rhs_local(m, orc.src_fourier(m.X, k, a, phi)))
    dinv = orc.jacobi_dinv_global(m)
    AII = [np.linalg.inv(orc.brute_element_matrix(N, m.xi, m.G[e])[np.ix_(I, I)])
           for e in range(m.E)]
    gI = [m.l2g[e * n3 + I] for e in range(m.E)]

    def block(r):
        z = dinv * r
        for e in range(m.E):
            z[gI[e]] = AII[e] @ r[gI[e]]
        return z

    _, st_j, it_j, _ = orc.pcg(m, b, 1e-8, 5000)
    _, st_b, it_b, _ = orc.fcg(m, b, block, 1e-8, 5000)
    assert st_j == 0 and st_b == 0
    assert it_b < 0.8 * it_j, (it_b, it_j)


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
