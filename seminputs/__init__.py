"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module draws random numbers only; it holds none of the method's
arithmetic (no nodes, no geometry, no operator).  Every generator takes an
explicit seed and uses ``numpy.random.default_rng``.

Workload recipes (synthetic stand-ins; the paper publishes no mesh or data
for its spectral-element benchmark):

* ``fourier_modes(seed)``: the smooth right-hand side is a sum of 8 random
  Fourier modes f(X) = sum_m a_m cos(2 pi k_m . X + phi_m) with integer wave
  vectors k_m in {0..3}^3 minus the zero vector, a_m ~ N(0,1),
  phi_m ~ U[0, 2 pi).
* ``grf_features(seed)``: a Gaussian random field with squared-exponential
  covariance (correlation length 0.1, sigma 1) represented by M random
  Fourier features (Rahimi & Recht 2007): omega_m ~ N(0, ell^-2 I),
  b_m ~ U[0, 2 pi).  kappa = exp(field).
* ``uniform(n, seed)``: U[-1, 1) samples (operator inputs on unique nodes or
  on local nodes).
* ``batch_configs(count, seed)``: uneven batched solves, cubic grids n^3 with
  n ~ U{6..24} and order N ~ U{3, 5, 7}.
* ``tri_mesh(nx, ny, seed)``: the stand-in for the shallow-water example's
  triangle mesh (its mesh and bathymetry are not published with the paper):
  a rectangle of nx x ny cells, interior grid points moved by a uniform
  random offset of up to 15 % of the cell size in each direction, every cell
  split into two counterclockwise triangles with the diagonal alternating
  from cell to cell (266 x 400 cells give the example's 212,800 triangles).
"""
from __future__ import annotations

import numpy as np


def fourier_modes(seed: int = 0, nmodes: int = 8, kmax: int = 3):
    rng = np.random.default_rng(seed)
    ks = []
    while len(ks) < nmodes:
        k = rng.integers(0, kmax + 1, size=3)
        if np.any(k != 0):
            ks.append(k)
    k = np.array(ks, dtype=np.float64)
    a = rng.standard_normal(nmodes)
    phi = rng.uniform(0.0, 2.0 * np.pi, nmodes)
    return k, a, phi


def grf_features(seed: int = 7, M: int = 4096, ell: float = 0.1,
                 sigma: float = 1.0):
    rng = np.random.default_rng(seed)
    omega = rng.standard_normal((M, 3)) / ell
    b = rng.uniform(0.0, 2.0 * np.pi, M)
    return omega, b, sigma


def uniform(n: int, seed: int = 0):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, n)


def normal(shape, seed: int = 0, scale: float = 1.0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) * scale


def batch_configs(count: int = 256, seed: int = 0, nmin: int = 6,
                  nmax: int = 24, orders=(3, 5, 7)):
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        N = int(rng.choice(orders))
        out.append((n, N))
    return out


def tri_mesh(nx: int, ny: int, seed: int = 0, lx: float = 1.0,
             ly: float = 1.0, jitter: float = 0.15):
    """Vertex coordinates vx, vy and int32 connectivity [2 nx ny][3]."""
    rng = np.random.default_rng(seed)
    hx, hy = lx / nx, ly / ny
    I, J = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
    vx = (I * hx).astype(np.float64)
    vy = (J * hy).astype(np.float64)
    inner = (I > 0) & (I < nx) & (J > 0) & (J < ny)
    vx[inner] += rng.uniform(-jitter, jitter, inner.sum()) * hx
    vy[inner] += rng.uniform(-jitter, jitter, inner.sum()) * hy
    vid = lambda i, j: j * (nx + 1) + i
    tris = []
    for j in range(ny):
        for i in range(nx):
            a, b, c, d = vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)
            if (i + j) % 2 == 0:
                tris += [(a, b, c), (a, c, d)]
            else:
                tris += [(a, b, d), (b, c, d)]
    return vx.ravel(), vy.ravel(), np.array(tris, dtype=np.int32)
