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
    return loss, pack([dW1, db1, dW2, db2, dW3, db3])


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
