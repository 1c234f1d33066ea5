"""FP64 oracle of the learned per-element coarse correction (TEST
INFRASTRUCTURE ONLY; only tests, the smoke check and the benchmark's CPU
baseline may import it).

The paper solves the system by PCG and leaves the preconditioner open
(section 4.2.2).  The learned correction adds to Jacobi an element coarse
correction whose operator a three-layer perceptron predicts:

    z1 = x W1^T + b1,  h1 = relu(z1)
    z2 = h1 W2^T + b2, h2 = relu(z2)
    o  = h2 W3^T + b3

trained with Adam (Kingma & Ba 2015).  Every function here is plain NumPy in
FP64; parameters are one flat vector in the order W1, b1, W2, b2, W3, b3
(row-major weights of shape [out][in]).

Coarse space: the interior "bubble" basis b_a(xi) = (1 - xi^2) P_a(xi),
a = 0..p (P_a Legendre, p = min(2, N - 2)), B[(i,j,k)][(a,b,c)] =
b_a(xi_i) b_b(xi_j) b_c(xi_k) on the element-interior nodes (K = (p+1)^3
columns, each scaled by the square root of the matching diagonal entry of
the unit reference element's coarse inverse so that every mode is O(1)).
The element's Galerkin coarse matrix is G_e = B^T A_II B (A_II the element
stiffness on its interior nodes) and its exact coarse correction
c_I = B G_e^{-1} B^T r_I.  The network sees the 8 log-kappa vertex
deviations of the element and outputs a lower-triangular factor L
(row-major packed, K(K+1)/2 values); M = L L^T approximates the normalised
inverse kappa_mean h G_e^{-1}, so the correction B (M / (kappa_mean h)) B^T
r_I is symmetric positive semi-definite for any network.  Training pairs:
y = B^T r_I / ||B^T r_I||, target alpha* = kappa_mean h G_e^{-1} y, loss
mean (L L^T y - alpha*)^2.

Parity status: forward/backward pinned by central finite differences and by
the linear-network closed form; Adam by its first-step closed form; the
coarse target and correction by reproduction of coarse-space solutions,
Galerkin orthogonality, zero face values and the invariance of the
normalised inverse under scaling of kappa and of the element.  Trained
weights are "parity unpinned" (non-convex, seed dependent).
"""
from __future__ import annotations

import numpy as np


def shapes(n_in, n_hidden, n_out):
    return [(n_hidden, n_in), (n_hidden,), (n_hidden, n_hidden), (n_hidden,),
            (n_out, n_hidden), (n_out,)]


def n_params(n_in, n_hidden, n_out):
    return sum(int(np.prod(s)) for s in shapes(n_in, n_hidden, n_out))


def unpack(theta, n_in, n_hidden, n_out):
    out, k = [], 0
    for s in shapes(n_in, n_hidden, n_out):
        size = int(np.prod(s))
        out.append(np.asarray(theta[k:k + size], dtype=np.float64).reshape(s))
        k += size
    return out


def pack(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1)
                           for p in parts])


def relu(a):
    return np.maximum(a, 0.0)


def forward(theta, X, n_in, n_hidden, n_out, keep=False):
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, n_hidden, n_out)
    z1 = X @ W1.T + b1
    h1 = relu(z1)
    z2 = h1 @ W2.T + b2
    h2 = relu(z2)
    o = h2 @ W3.T + b3
    if keep:
        return o, (X, z1, h1, z2, h2)
    return o


def backward(theta, acts, do, n_in, n_hidden, n_out):
    """Parameter gradient from the output gradient do (B x n_out) and the
    activations kept by forward(..., keep=True)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, n_hidden, n_out)
    X, z1, h1, z2, h2 = acts
    dW3 = do.T @ h2
    db3 = do.sum(axis=0)
    dh2 = do @ W3
    dz2 = dh2 * (z2 > 0)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2
    dz1 = dh1 * (z1 > 0)
    dW1 = dz1.T @ X
    db1 = dz1.sum(axis=0)
    return pack([dW1, db1, dW2, db2, dW3, db3])


def adam_step(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t is the 1-based step number); returns new
    (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v


def he_init(n_in, n_hidden, n_out, seed):
    rng = np.random.default_rng(seed)
    parts = []
    for s in shapes(n_in, n_hidden, n_out):
        if len(s) == 2:
            parts.append(rng.standard_normal(s) * np.sqrt(2.0 / s[1]))
        else:
            parts.append(np.zeros(s))
    return pack(parts)


def interior_nodes(N):
    """Local indices i + n1 j + n1^2 k of the element-interior nodes
    1 <= i, j, k <= N-1 in lexicographic order (i fastest)."""
    n1, m = N + 1, N - 1
    q = np.arange(max(m, 0) ** 3)
    if m <= 0:
        return q
    i = q % m + 1
    j = (q // m) % m + 1
    k = q // (m * m) + 1
    return i + n1 * (j + n1 * k)


def coarse_degree(N):
    """Polynomial degree p of the bubble basis (K = (p+1)^3 columns)."""
    return min(2, N - 2)


def bubble_basis(N, xi, scaled=True):
    """B [(N-1)^3][(p+1)^3]: tensor products of b_a(x) = (1 - x^2) P_a(x) at
    the interior GLL nodes; rows in interior lexicographic order (i fastest),
    columns (a, b, c) with a fastest.  scaled: every column is multiplied by
    sqrt of the matching diagonal entry of the reference coarse inverse
    (G_ref^{-1} of the unit-cube element with kappa = 1, whose kappa h is 1),
    which makes the normalised coarse inverses O(1) in every mode."""
    from numpy.polynomial import legendre as leg
    p = coarse_degree(N)
    xin = np.asarray(xi, dtype=np.float64)[1:N]
    B1 = np.stack([(1 - xin ** 2) * leg.legval(xin, np.eye(p + 1)[a])
                   for a in range(p + 1)], 1)
    # row (i, j, k) = i + m j + m^2 k and column (a, b, c) = a + q b + q^2 c
    B = np.kron(B1, np.kron(B1, B1))
    if not scaled:
        return B
    from . import oracle as orc
    ref = orc.mesh(N, 1, 1, 1, orc.MAP_AFFINE, 0, None)
    I = interior_nodes(N)
    A_II = orc.brute_element_matrix(N, ref.xi, ref.G[0])[np.ix_(I, I)]
    Mref = np.linalg.inv(B.T @ A_II @ B)
    return B * np.sqrt(np.diag(Mref))[None, :]


def coarse_galerkin(A_e, N, xi):
    """G_e = B^T A_II B from the element stiffness A_e (n1^3 x n1^3)."""
    I = interior_nodes(N)
    B = bubble_basis(N, xi)
    A_II = np.asarray(A_e, dtype=np.float64)[np.ix_(I, I)]
    return B.T @ A_II @ B


def coarse_target(A_e, N, xi, kappa_vertices, h):
    """kappa_mean h G_e^{-1}: the normalised exact coarse inverse."""
    G = coarse_galerkin(A_e, N, xi)
    kbar = float(np.mean(np.asarray(kappa_vertices, dtype=np.float64)))
    return np.linalg.inv(G) * kbar * h


def factor_unpack(o, K):
    """Lower-triangular L from K(K+1)/2 row-major packed values."""
    L = np.zeros((K, K))
    L[np.tril_indices(K)] = np.asarray(o, dtype=np.float64)
    return L


def factor_loss_and_grad(O, Y, Astar):
    """Mean over samples and components of (L L^T y - alpha*)^2 and its
    gradient with respect to the packed outputs O [S][K(K+1)/2]."""
    O = np.asarray(O, dtype=np.float64)
    S = O.shape[0]
    K = Y.shape[1]
    tri = np.tril_indices(K)
    loss = 0.0
    dO = np.zeros_like(O)
    for s_ in range(S):
        L = factor_unpack(O[s_], K)
        y = Y[s_]
        v = L.T @ y
        a = L @ v
        d = a - Astar[s_]
        loss += float(d @ d)
        g = 2.0 * d / (S * K)
        dL = np.outer(g, v) + np.outer(y, L.T @ g)
        dO[s_] = dL[tri]
    return loss / (S * K), dO


def coarse_correction(r_e, M_e, N, xi, kappa_vertices, h, damping=1.0):
    """Correction on the element's n1^3 nodes: damping B (M / (kappa_mean
    h)) B^T r_I on the interior nodes, zero on the faces."""
    I = interior_nodes(N)
    B = bubble_basis(N, xi)
    kbar = float(np.mean(np.asarray(kappa_vertices, dtype=np.float64)))
    c = np.zeros((N + 1) ** 3)
    r_I = np.asarray(r_e, dtype=np.float64)[I]
    c[I] = damping * (B @ (np.asarray(M_e) @ (B.T @ r_I))) / (kbar * h)
    return c


def factor_net_loss_and_grad(theta, X, Y, Astar, n_in, n_hidden, K):
    """Factor loss of the coarse layout through the network: outputs
    O = forward(X) are the packed factors; returns (loss, gradient)."""
    n_out = K * (K + 1) // 2
    O, acts = forward(theta, X, n_in, n_hidden, n_out, keep=True)
    loss, dO = factor_loss_and_grad(O, Y, Astar)
    return loss, backward(theta, acts, dO, n_in, n_hidden, n_out)
