"""Pins of the FP64 oracle of the correction network: gradients of the
factor loss through the network against central finite differences, the
purely linear regime against its closed form, Adam's first step against its
closed form, and Adam on a target the network can represent."""
import numpy as np

from oracle import mlp

NI, NH, K = 8, 7, 3
NO = K * (K + 1) // 2


def _problem(seed=0, S=5):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(mlp.n_params(NI, NH, NO)) * 0.5
    X = rng.standard_normal((S, NI))
    Y = rng.standard_normal((S, K))
    A = rng.standard_normal((S, K))
    return theta, X, Y, A


def test_gradient_matches_central_differences():
    theta, X, Y, A = _problem()
    loss, g = mlp.factor_net_loss_and_grad(theta, X, Y, A, NI, NH, K)
    h = 1e-6
    fd = np.zeros_like(theta)
    for q in range(theta.size):
        tp = theta.copy()
        tm = theta.copy()
        tp[q] += h
        tm[q] -= h
        fd[q] = (mlp.factor_net_loss_and_grad(tp, X, Y, A, NI, NH, K)[0]
                 - mlp.factor_net_loss_and_grad(tm, X, Y, A, NI, NH, K)[0]) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-7 * max(1.0, np.max(np.abs(g)))
    # the loss is the plain mean over samples and components
    O = mlp.forward(theta, X, NI, NH, NO)
    ref = np.mean([(L @ L.T @ y - a) ** 2 for L, y, a in
                   zip([mlp.factor_unpack(o, K) for o in O], Y, A)])
    assert abs(loss - ref) < 1e-14 * max(1.0, loss)


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


def test_training_reaches_a_representable_target():
    """Targets from a fixed SPD operator M (alpha* = M y) are reachable by
    the output bias alone (L = chol(M)); Adam drives the loss down."""
    rng = np.random.default_rng(3)
    S = 64
    X = rng.standard_normal((S, NI))
    Y = rng.standard_normal((S, K))
    C = rng.standard_normal((K, K))
    M = C @ C.T + K * np.eye(K)
    A = Y @ M.T
    theta = mlp.he_init(NI, NH, NO, seed=4)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.factor_net_loss_and_grad(theta, X, Y, A, NI, NH, K)[0]
    for t in range(1, 401):
        _, g = mlp.factor_net_loss_and_grad(theta, X, Y, A, NI, NH, K)
        theta, m, v = mlp.adam_step(theta, g, m, v, t, 1e-2)
    l1 = mlp.factor_net_loss_and_grad(theta, X, Y, A, NI, NH, K)[0]
    assert l1 < 0.05 * l0, (l0, l1)
