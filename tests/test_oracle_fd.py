"""Pins of the finite-difference oracle (paper section 4.1: the 2D acoustic
wave equation on a periodic grid, leapfrog in time, 2r-order central stencil
in space).

Each check fails on a plausible slip: a wrong weight or order (textbook
tables, an independent closed form, polynomial exactness, the symbol's
truncation order), a swapped roll direction or boundary wrap (translation
invariance, Fourier-mode symbol), an x/y asymmetry (transpose), a wrong sign
or time level in the leapfrog update (time reversibility, the standing-wave
convergence)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import fd

GOLDEN = os.path.join(os.path.dirname(__file__), "golden",
                      "fd_weights_closed_forms.txt")


def _golden():
    out = {}
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        r, vals = line.split(":")
        out[int(r)] = [Fraction(v) for v in vals.split()]
    return out


def test_weights_match_textbook_tables():
    g = _golden()
    assert sorted(g) == [1, 2, 3, 4]
    for r, ref in g.items():
        assert fd.weights_exact(r) == ref, r


@pytest.mark.parametrize("r", range(1, 8))
def test_weights_closed_form(r):
    """w_k = 2 (-1)^(k+1) (r!)^2 / (k^2 (r-k)! (r+k)!) for k != 0 and
    w_0 = -2 sum_{k>0} w_k (the maximal-order centred formula)."""
    w = fd.weights_exact(r)
    f = math.factorial
    wk = {k: Fraction(2 * (-1) ** (k + 1) * f(r) ** 2,
                      k * k * f(r - k) * f(r + k)) for k in range(1, r + 1)}
    for k in range(1, r + 1):
        assert w[r + k] == wk[k] and w[r - k] == wk[k]
    assert w[r] == -2 * sum(wk.values())


@pytest.mark.parametrize("r", range(1, 8))
def test_weights_exact_on_polynomials_to_order_2r(r):
    """sum_k w_k (x0 + k)^p = p (p-1) x0^(p-2) exactly for p <= 2r + 1 (odd
    p by symmetry), and not for p = 2r + 2: the order is exactly 2r."""
    w = fd.weights_exact(r)
    x0 = Fraction(3, 7)
    for p in range(0, 2 * r + 3):
        lhs = sum(w[r + k] * (x0 + k) ** p for k in range(-r, r + 1))
        rhs = Fraction(p * (p - 1)) * x0 ** (p - 2) if p >= 2 else Fraction(0)
        if p <= 2 * r + 1:
            assert lhs == rhs, (r, p)
        else:
            assert lhs != rhs, (r, p)


@pytest.mark.parametrize("r", range(1, 8))
def test_symbol_truncation_order(r):
    """lambda(theta) = sum_k w_k cos(k theta) = -theta^2 + O(theta^(2r+2))."""
    w = fd.weights(r)

    def err(t):
        lam = sum(w[r + k] * math.cos(k * t) for k in range(-r, r + 1))
        return abs(lam + t * t)

    t = 0.8
    rate = math.log2(err(t) / err(t / 2))
    assert abs(rate - (2 * r + 2)) < 0.35, (r, rate)


def _mode(nx, ny, a, b):
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    return np.cos(2 * np.pi * a * i / nx + 0.3) * np.cos(2 * np.pi * b * j / ny - 0.7)


@pytest.mark.parametrize("r", [1, 3, 7])
def test_step_on_fourier_mode(r):
    """On a discrete Fourier mode the stencil acts by its symbol:
    u_{n+1} = (2 + c (lambda(tx) + lambda(ty))) u_n - u_{n-1}."""
    nx, ny, a, b = 48, 40, 5, 3
    u = _mode(nx, ny, a, b)
    w = fd.weights(r)
    lam = lambda t: sum(w[r + k] * math.cos(k * t) for k in range(-r, r + 1))
    lx, ly = lam(2 * np.pi * a / nx), lam(2 * np.pi * b / ny)
    up = 0.5 * u
    dx = 2.0 / nx
    dt = 0.25 * dx
    c = dt * dt / (dx * dx)
    got = fd.step(u, up, r, dt, dx)
    ref = (2 + c * (lx + ly)) * u - up
    assert np.max(np.abs(got - ref)) < 1e-14 * (2 + c * 4 * r * r) * np.max(np.abs(u))


@pytest.mark.parametrize("r", [1, 4, 7])
def test_time_reversibility(r):
    """Leapfrog is reversible: K steps forward, then K steps from the swapped
    final pair, return the initial pair to rounding."""
    rng = np.random.default_rng(5)
    nx, ny = 37, 29
    u0p, u0c = rng.uniform(-1, 1, (ny, nx)), rng.uniform(-1, 1, (ny, nx))
    dx = 2.0 / nx
    dt = 0.25 * dx
    a, b = fd.run(u0p, u0c, r, dt, dx, 25)
    ra, rb = fd.run(b, a, r, dt, dx, 25)
    assert np.max(np.abs(ra - u0c)) < 1e-11
    assert np.max(np.abs(rb - u0p)) < 1e-11


@pytest.mark.parametrize("r", [2, 5])
def test_translation_and_transpose(r):
    rng = np.random.default_rng(6)
    n = 23
    u, up = rng.uniform(-1, 1, (n, n)), rng.uniform(-1, 1, (n, n))
    dx = 2.0 / n
    dt = 0.3 * dx
    out = fd.step(u, up, r, dt, dx)
    sh = (4, -7)
    out_s = fd.step(np.roll(u, sh, axis=(0, 1)), np.roll(up, sh, axis=(0, 1)), r,
                    dt, dx)
    np.testing.assert_array_equal(out_s, np.roll(out, sh, axis=(0, 1)))
    out_t = fd.step(u.T.copy(), up.T.copy(), r, dt, dx)
    np.testing.assert_array_equal(out_t, out.T)


def _standing_wave_error(n, r, T=0.5, cfl=0.25):
    """u = cos(pi x) cos(pi y) cos(sqrt(2) pi t) on [-1, 1)^2 (period 2)."""
    dx = 2.0 / n
    x = -1.0 + dx * np.arange(n)
    X, Y = np.meshgrid(x, x)
    om = math.sqrt(2) * math.pi
    exact = lambda t: np.cos(math.pi * X) * np.cos(math.pi * Y) * math.cos(om * t)
    dt0 = cfl * dx
    K = int(round(T / dt0))
    dt = T / K
    a, b = fd.run(exact(0.0), exact(dt), r, dt, dx, K)
    return np.max(np.abs(b - exact((K + 1) * dt)))


def test_standing_wave_second_order():
    """r = 1 with dt proportional to dx: the leapfrog solution converges at
    second order to the exact standing wave."""
    e1, e2, e3 = (_standing_wave_error(n, 1) for n in (16, 32, 64))
    r1, r2 = math.log2(e1 / e2), math.log2(e2 / e3)
    assert 1.8 < r2 < 2.3, (r1, r2)


@pytest.mark.parametrize("r", [2, 3])
def test_spatial_operator_order_2r(r):
    """The scaled stencil applied to cos(pi x) cos(pi y) approaches
    -2 pi^2 u at order 2r."""
    errs = []
    for n in (16, 32):
        dx = 2.0 / n
        x = -1.0 + dx * np.arange(n)
        X, Y = np.meshgrid(x, x)
        u = np.cos(math.pi * X) * np.cos(math.pi * Y)
        lap = fd.laplacian_unscaled(u, r) / (dx * dx)
        errs.append(np.max(np.abs(lap + 2 * math.pi ** 2 * u)))
    rate = math.log2(errs[0] / errs[1])
    assert abs(rate - 2 * r) < 0.3, (r, rate)
