"""Pins of the oracle's geometric factors and lumped mass (paper section
4.2.1: chain rule, G^T G metric precomputed per elemental node, lumped mass
J w_abc).  Checked against the closed form of affine boxes, the exact
volume of the mapped cubes, the analytic metric of the sine mappings, and the
placement of kappa on the flux."""
import numpy as np
import pytest

from oracle import oracle as orc

PAIRS = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


@pytest.mark.parametrize("N,ex,ey,ez", [(1, 2, 3, 4), (4, 3, 2, 1), (7, 2, 2, 3)])
def test_affine_closed_form(N, ex, ey, ez):
    m = orc.mesh(N, ex, ey, ez, orc.MAP_AFFINE)
    hx, hy, hz = 1.0 / ex, 1.0 / ey, 1.0 / ez
    w3 = np.einsum("k,j,i->kji", m.w, m.w, m.w).reshape(-1)
    ref = np.zeros((6, (N + 1) ** 3))
    ref[0] = w3 * hy * hz / (2 * hx)
    ref[3] = w3 * hx * hz / (2 * hy)
    ref[5] = w3 * hx * hy / (2 * hz)
    for e in range(m.E):
        np.testing.assert_allclose(m.G[e], ref, rtol=1e-12, atol=1e-14 * ref.max())
    B = m.B.reshape(m.E, -1)
    np.testing.assert_allclose(B, np.broadcast_to(w3 * hx * hy * hz / 8, B.shape),
                               rtol=1e-12)
    assert abs(m.B.sum() - 1.0) < 1e-13
    assert abs(m.minJ - hx * hy * hz / 8) < 1e-12 * hx * hy * hz


@pytest.mark.parametrize("N", [2, 4, 7])
def test_sine_x_unit_jacobian(N):
    """x + 0.05 sin(2 pi y) sin(2 pi z) is volume preserving: det = 1 for the
    interpolated geometry as well (the shear term does not depend on x)."""
    m = orc.mesh(N, 3, 3, 3, orc.MAP_SINE_X)
    w3 = np.einsum("k,j,i->kji", m.w, m.w, m.w).reshape(-1)
    J = m.B.reshape(m.E, -1) / w3
    np.testing.assert_allclose(J, 1.0 / 27 / 8, rtol=1e-12)
    assert abs(m.B.sum() - 1.0) < 1e-13


def _analytic_metric(N, ex, ey, ez, X_affine):
    """G from the exact derivative of the cyclic sine mapping at the nodes."""
    x, y, z = X_affine
    s = lambda t: np.sin(2 * np.pi * t)
    ds = lambda t: 2 * np.pi * np.cos(2 * np.pi * t)
    n = x.shape[0]
    F = np.zeros((n, 3, 3))
    F[:, 0, 0] = F[:, 1, 1] = F[:, 2, 2] = 1.0
    F[:, 0, 1] = 0.05 * ds(y) * s(z)
    F[:, 0, 2] = 0.05 * s(y) * ds(z)
    F[:, 1, 0] = 0.05 * s(z) * ds(x)
    F[:, 1, 2] = 0.05 * ds(z) * s(x)
    F[:, 2, 0] = 0.05 * ds(x) * s(y)
    F[:, 2, 1] = 0.05 * s(x) * ds(y)
    h = np.array([1.0 / ex, 1.0 / ey, 1.0 / ez])
    Jm = F * (h / 2)[None, None, :]          # dX/dr = F diag(h/2)
    det = np.linalg.det(Jm)
    inv = np.linalg.inv(Jm)                  # rows: grad r, grad s, grad t
    return det, inv


@pytest.mark.parametrize("N", [4, 6, 8, 10])
def test_cyclic_metric_converges_to_analytic(N):
    ex = ey = ez = 3
    m = orc.mesh(N, ex, ey, ez, orc.MAP_SINE_CYCLIC)
    Xa = orc.coords(N, ex, ey, ez, orc.MAP_AFFINE)
    det, inv = _analytic_metric(N, ex, ey, ez, Xa)
    w3 = np.tile(np.einsum("k,j,i->kji", m.w, m.w, m.w).reshape(-1), m.E)
    n3 = (N + 1) ** 3
    err = 0.0
    for q, (a, b) in enumerate(PAIRS):
        ref = w3 * det * np.einsum("nd,nd->n", inv[:, a, :], inv[:, b, :])
        got = m.G[:, q, :].reshape(-1)
        err = max(err, np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    tol = {4: 2e-2, 6: 2e-3, 8: 1e-4, 10: 5e-6}[N]
    assert err < tol, err
    assert m.minJ > 0.6 * (1 / 27) / 8


@pytest.mark.parametrize("E", [2, 3, 5])
@pytest.mark.parametrize("N", [2, 4, 7])
def test_cyclic_volume_is_one(N, E):
    """Every cross term of det(dX/dx) for the cyclic sine map is a product
    containing the derivative of a periodic factor in one variable.  GLL
    quadrature integrates the derivative of the degree-N interpolant exactly
    (degree N-1 <= 2N-1), so each such factor telescopes to s(1) - s(0) = 0
    and the discrete volume sum(B) equals 1 to roundoff for every N."""
    m = orc.mesh(N, E, E, E, orc.MAP_SINE_CYCLIC)
    assert abs(m.B.sum() - 1.0) < 1e-13


def test_kappa_scales_flux_metric_not_mass():
    """kappa sits on the flux (kappa grad u . grad v): G scales with kappa,
    B does not."""
    N = 3
    base = orc.mesh(N, 2, 2, 1, orc.MAP_SINE_CYCLIC)
    X = base.X
    kap = 2.0 + np.sin(3 * X[0]) * np.cos(2 * X[1]) + X[2]
    G, B, _ = orc.geom(N, base.E, base.w, base.D, X, kap)
    np.testing.assert_array_equal(B, base.B)
    np.testing.assert_allclose(
        G, base.G * kap.reshape(base.E, 1, -1), rtol=1e-15, atol=0)


def test_kappa_field_has_the_squared_exponential_covariance():
    """g = log kappa from orc_kappa_rff, over independent feature draws:
    mean 0 and covariance sigma^2 exp(-|x - y|^2 / (2 l^2)) (random Fourier
    features of that kernel, Rahimi & Recht 2007), within the sampling error
    of the draws.  A wrong amplitude factor (sqrt(2 / M), sigma vs
    sigma^2) or length scale moves some of these by far more."""
    from seminputs import grf_features
    ell, sigma, M, S = 0.3, 0.8, 64, 3000
    x0 = np.array([0.4, 0.5, 0.6])
    d = np.array([0.0, 0.5, 1.0, 2.0]) * ell
    pts = np.stack([x0 + np.array([dd, 0.0, 0.0]) for dd in d])
    X = np.ascontiguousarray(pts.T)            # [3][n] blocks
    g = np.empty((S, len(d)))
    for s in range(S):
        om, b, sg = grf_features(seed=10_000 + s, M=M, ell=ell, sigma=sigma)
        g[s] = np.log(orc.kappa_rff(X, om, b, sg))
    mean = g.mean(0)
    cov = (g * g[:, :1]).mean(0)               # E[g(x0) g(x0 + d e1)]
    want = sigma ** 2 * np.exp(-d ** 2 / (2 * ell ** 2))
    se = sigma ** 2 * np.sqrt(2.0 / S)         # standard error of a product mean
    assert np.all(np.abs(mean) <= 5 * sigma / np.sqrt(S)), mean
    assert np.all(np.abs(cov - want) <= 5 * se), (cov, want)
