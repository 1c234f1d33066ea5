"""Pins of the FP64 oracle of the learned per-element correction: gradients
against central finite differences, the purely linear regime against its
closed form, Adam's first step against its closed form, and the trilinear
prolongation against exact reproduction of trilinear functions."""
import numpy as np
import pytest

from oracle import mlp
from oracle import oracle as orc

NI, NH, NO = 20, 7, 8


def _problem(seed=0, B=5, nn=12):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(mlp.n_params(NI, NH, NO)) * 0.5
    X = rng.standard_normal((B, NI))
    T = rng.standard_normal((B, nn))
    P = rng.standard_normal((nn, NO))
    return theta, X, T, P


def test_gradient_matches_central_differences():
    theta, X, T, P = _problem()
    loss, g = mlp.loss_and_grad(theta, X, T, P, NI, NH, NO)
    h = 1e-6
    fd = np.zeros_like(theta)
    for q in range(theta.size):
        tp = theta.copy()
        tm = theta.copy()
        tp[q] += h
        tm[q] -= h
        fd[q] = (mlp.loss_and_grad(tp, X, T, P, NI, NH, NO)[0]
                 - mlp.loss_and_grad(tm, X, T, P, NI, NH, NO)[0]) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))
    # the loss is the plain mean of squared differences
    o = mlp.forward(theta, X, NI, NH, NO)
    assert abs(loss - np.mean((o @ P.T - T) ** 2)) < 1e-14 * max(1.0, loss)


def test_linear_regime_closed_form():
    """With positive weights, biases and inputs every ReLU passes its input,
    so the network is the affine map W3 (W2 (W1 x + b1) + b2) + b3."""
    rng = np.random.default_rng(1)
    parts = [np.abs(rng.standard_normal(s)) for s in mlp.shapes(NI, NH, NO)]
    theta = mlp.pack(parts)
    X = np.abs(rng.standard_normal((4, NI)))
    W1, b1, W2, b2, W3, b3 = parts
    ref = ((X @ W1.T + b1) @ W2.T + b2) @ W3.T + b3
    np.testing.assert_allclose(mlp.forward(theta, X, NI, NH, NO), ref,
                               rtol=1e-14)
    # and relu really cuts: negating W1 zeroes the first hidden layer
    parts2 = [-parts[0]] + parts[1:]
    parts2[1] = -parts[1]
    out = mlp.forward(mlp.pack(parts2), X, NI, NH, NO)
    np.testing.assert_allclose(out, np.broadcast_to(
        np.maximum(b2, 0) @ W3.T + b3, out.shape), rtol=1e-14)


def test_adam_first_step_closed_form():
    """Step 1: m_hat = g and v_hat = g^2, so theta moves by
    -lr g / (|g| + eps) -- essentially lr against the sign of g."""
    rng = np.random.default_rng(2)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    lr, eps = 1e-3, 1e-8
    t1, m, v = mlp.adam_step(theta, g, np.zeros(50), np.zeros(50), 1, lr,
                             eps=eps)
    np.testing.assert_allclose(t1, theta - lr * g / (np.abs(g) + eps),
                               rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(m, 0.1 * g, rtol=1e-14)
    np.testing.assert_allclose(v, 0.001 * g * g, rtol=1e-14)


@pytest.mark.parametrize("N", [1, 3, 7])
def test_prolongation_reproduces_trilinear_functions(N):
    xi, _ = orc.gll(N)
    P = mlp.prolongation(xi)
    n1 = N + 1
    np.testing.assert_allclose(P.sum(axis=1), 1.0, rtol=1e-15)
    rng = np.random.default_rng(N)
    c = rng.standard_normal(8)   # f = sum_v c_v phi_v, any trilinear function
    f = lambda x, y, z: (c[0] * (1 - x) * (1 - y) * (1 - z) +
                         c[1] * (1 + x) * (1 - y) * (1 - z) +
                         c[2] * (1 - x) * (1 + y) * (1 - z) +
                         c[3] * (1 + x) * (1 + y) * (1 - z) +
                         c[4] * (1 - x) * (1 - y) * (1 + z) +
                         c[5] * (1 + x) * (1 - y) * (1 + z) +
                         c[6] * (1 - x) * (1 + y) * (1 + z) +
                         c[7] * (1 + x) * (1 + y) * (1 + z)) / 8
    verts = np.array([f(2 * (v & 1) - 1, 2 * ((v >> 1) & 1) - 1,
                        2 * ((v >> 2) & 1) - 1) for v in range(8)])
    vals = P @ verts
    for k in range(n1):
        for j in range(n1):
            for i in range(n1):
                assert abs(vals[i + n1 * j + n1 * n1 * k]
                           - f(xi[i], xi[j], xi[k])) < 1e-14


def test_element_features():
    m = orc.mesh(3, 2, 2, 2, orc.MAP_AFFINE)
    r = np.random.default_rng(0).standard_normal(m.nG)
    kap = np.exp(np.random.default_rng(1).standard_normal(8))
    x, s = mlp.element_features(r, m.l2g, m.n1, 3, kap, 72)
    assert abs(np.linalg.norm(x[:64]) - 1.0) < 1e-14
    assert abs(x[64:72].sum()) < 1e-14 and np.all(x[72:] == 0)
    np.testing.assert_allclose(x[:64] * s, r[m.l2g[3 * 64:4 * 64]], rtol=1e-14)


def test_training_reduces_loss_on_a_learnable_target():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((64, NI))
    Wt = rng.standard_normal((NO, NI)) * 0.3
    P = rng.standard_normal((12, NO))
    T = (X @ Wt.T) @ P.T
    theta = mlp.he_init(NI, NH, NO, seed=4)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss_and_grad(theta, X, T, P, NI, NH, NO)[0]
    for t in range(1, 301):
        _, g = mlp.loss_and_grad(theta, X, T, P, NI, NH, NO)
        theta, m, v = mlp.adam_step(theta, g, m, v, t, 1e-2)
    l1 = mlp.loss_and_grad(theta, X, T, P, NI, NH, NO)[0]
    assert l1 < 0.2 * l0
