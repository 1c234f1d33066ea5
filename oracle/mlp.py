"""FP64 oracle of the learned per-element coarse correction (TEST
INFRASTRUCTURE ONLY; only tests, the smoke check and the benchmark's CPU
baseline may import it).

The paper leaves the PCG preconditioner open (section 4.2.2).  The learned
correction is a per-element three-layer perceptron:

    z1 = x W1^T + b1,  h1 = relu(z1)
    z2 = h1 W2^T + b2, h2 = relu(z2)
    o  = h2 W3^T + b3                        (8 coarse vertex values)

whose output is prolonged to the element's GLL nodes by the trilinear (Q1)
basis, P[node(i,j,k)][v(a,b,c)] = phi_a(xi_i) phi_b(xi_j) phi_c(xi_k) with
phi_0 = (1 - xi)/2, phi_1 = (1 + xi)/2 and v = a + 2b + 4c.  Training
minimises the mean squared error between P o and the normalised element
error with Adam (Kingma & Ba 2015).  Every function here is plain NumPy in
FP64; parameters are one flat vector in the order W1, b1, W2, b2, W3, b3
(row-major weights of shape [out][in]).

Features of an element e (unique-node residual r, map l2g, coefficient
kappa): r_e = r[l2g of e's nodes], s_e = ||r_e||_2;
x = [r_e / s_e, log kappa at the 8 element vertices minus their mean, 0 pad];
the correction is c_e = s_e / (kappa_mean_e h_e) * P o, summed over the
copies of each node and divided by its multiplicity.

Interior layout (the element-interior solve as target): the network sees
only the residual at the element-interior nodes (1 <= i, j, k <= N-1),
x = [r_I / s, log kappa vertex deviations], s = ||r_I||_2, and predicts the
(N-1)^3 values t = (d - dinv_I r_I) kappa_mean h / s, where d solves
A_II d = r_I with A_II the element stiffness restricted to its interior
nodes (zero values on the element's faces) and dinv the assembled Jacobi
inverse.  The preconditioner z = dinv r + c then reproduces the
element-interior block solve where the network is exact.  Interior nodes
belong to one element only, so no averaging is involved.

Coarse layout (a learned element coarse operator): with the interior
"bubble" basis b_a(xi) = (1 - xi^2) P_a(xi), a = 0..p (P_a Legendre,
p = min(2, N - 2)), B[(i,j,k)][(a,b,c)] = b_a(xi_i) b_b(xi_j) b_c(xi_k) on
the interior nodes (K = (p+1)^3 columns, each scaled by the square root of
the matching diagonal entry of the unit reference element's coarse inverse
so that every mode is O(1)), the element's Galerkin coarse
matrix is G_e = B^T A_II B and its exact coarse correction
c_I = B G_e^{-1} B^T r_I.  The network sees only the 8 log-kappa vertex
deviations and outputs a lower-triangular factor L (row-major packed,
K(K+1)/2 values); M = L L^T approximates kappa_mean h G_e^{-1}, so the
correction B (M / (kappa_mean h)) B^T r_I is symmetric positive
semi-definite for any network.  Training pairs come from solver residuals:
y = B^T r_I / ||B^T r_I||, target alpha* = kappa_mean h G_e^{-1} y, loss
mean (L L^T y - alpha*)^2.

Parity status: forward/backward pinned by central finite differences and by
the linear-network closed form; Adam pinned by its first-step closed form;
prolongation pinned by exact reproduction of trilinear functions.  Trained
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


def prolongation(xi):
    """P[node][v] for the GLL nodes xi of one direction (n1^3 x 8)."""
    xi = np.asarray(xi, dtype=np.float64)
    phi = np.stack([(1.0 - xi) / 2.0, (1.0 + xi) / 2.0])  # [a][i]
    n1 = xi.shape[0]
    P = np.zeros((n1 ** 3, 8))
    for k in range(n1):
        for j in range(n1):
            for i in range(n1):
                node = i + n1 * j + n1 * n1 * k
                for c in range(2):
                    for b in range(2):
                        for a in range(2):
                            P[node, a + 2 * b + 4 * c] = (
                                phi[a, i] * phi[b, j] * phi[c, k])
    return P


def loss_and_grad(theta, X, T, P, n_in, n_hidden, n_out):
    """MSE between P o and the targets T (B x n_nodes) and its gradient."""
    W1, b1, W2, b2, W3, b3 = unpack(theta, n_in, n_hidden, n_out)
    o, (X, z1, h1, z2, h2) = forward(theta, X, n_in, n_hidden, n_out, keep=True)
    B, nn = T.shape
    diff = o @ P.T - T
    loss = float(np.sum(diff * diff) / (B * nn))
    dY = 2.0 * diff / (B * nn)          # d loss / d (P o)
    do = dY @ P                          # B x n_out
    return loss, backward(theta, (X, z1, h1, z2, h2), do, n_in, n_hidden, n_out)


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


def element_features(r_global, l2g, n1, e, kappa_vertices, n_in):
    """Features x (n_in) and the scale s_e of element e."""
    n3 = n1 ** 3
    r_e = np.asarray(r_global, dtype=np.float64)[l2g[e * n3:(e + 1) * n3]]
    s = float(np.linalg.norm(r_e))
    x = np.zeros(n_in)
    if s > 0:
        x[:n3] = r_e / s
    lk = np.log(np.asarray(kappa_vertices, dtype=np.float64))
    x[n3:n3 + 8] = lk - lk.mean()
    return x, s


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


def interior_features(r_e, kappa_vertices, N, n_in=None):
    """Features of the interior layout from the element's n1^3 nodal
    residual values r_e: x = [r_I / s, log kappa vertex deviations], s."""
    I = interior_nodes(N)
    ni = I.shape[0]
    r_I = np.asarray(r_e, dtype=np.float64)[I]
    s = float(np.linalg.norm(r_I))
    x = np.zeros(ni + 8 if n_in is None else n_in)
    if s > 0:
        x[:ni] = r_I / s
    lk = np.log(np.asarray(kappa_vertices, dtype=np.float64))
    x[ni:ni + 8] = lk - lk.mean()
    return x, s


def interior_solve(A_e, r_e, N):
    """d = A_II^{-1} r_I: the element stiffness A_e (n1^3 x n1^3) restricted
    to the interior nodes, solved densely."""
    I = interior_nodes(N)
    A_II = np.asarray(A_e, dtype=np.float64)[np.ix_(I, I)]
    return np.linalg.solve(A_II, np.asarray(r_e, dtype=np.float64)[I])


def interior_target(A_e, r_e, dinv_e, kappa_vertices, h, N):
    """Target of the interior layout: (d - dinv_I r_I) kappa_mean h / s with
    d = interior_solve(A_e, r_e, N); dinv_e holds the assembled Jacobi
    inverse at the element's n1^3 nodes."""
    I = interior_nodes(N)
    r_I = np.asarray(r_e, dtype=np.float64)[I]
    s = float(np.linalg.norm(r_I))
    if s == 0:
        return np.zeros(I.shape[0])
    d = interior_solve(A_e, r_e, N)
    kbar = float(np.mean(np.asarray(kappa_vertices, dtype=np.float64)))
    return (d - np.asarray(dinv_e, dtype=np.float64)[I] * r_I) * kbar * h / s


def interior_correction(o, s, kappa_vertices, h, N, damping=1.0):
    """Correction on the element's n1^3 nodes from the network output o
    ((N-1)^3 values): damping s / (kappa_mean h) o on the interior nodes,
    zero on the faces."""
    n1 = N + 1
    c = np.zeros(n1 ** 3)
    kbar = float(np.mean(np.asarray(kappa_vertices, dtype=np.float64)))
    c[interior_nodes(N)] = damping * s / (kbar * h) * np.asarray(o, dtype=np.float64)
    return c


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
