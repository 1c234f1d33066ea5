"""FP64 CPU oracle for the finite-difference wave-equation example of the
paper's section 4.1 (its pseudocode and kernel `fd2d`).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the benchmark's CPU-baseline leg may import this module.  It shares no code
with the HIP product library and never imports it.

Problem (section 4.1.1): u_tt = u_xx + u_yy, sound speed 1, on the square
[-1, 1]^2 discretised by a periodic grid of nx x ny nodes (section 4.1.2),
node (i, j) stored at j * nx + i, spacing dx = 2 / nx.

Discretisation (section 4.1.2): the time derivative by the three-point
stencil {1, -2, 1} / dt^2, the space derivatives by a central stencil of
2r + 1 nodes per direction and order 2r.  The update is the leapfrog step

    u_{n+1}(i, j) = 2 u_n(i, j) - u_{n-1}(i, j)
                    + (dt^2 / dx^2) sum_{k=-r..r} w_k (u_n(i+k, j) + u_n(i, j+k))

with w the unit-spacing weights of the second derivative.  (The printed
update carries the opposite sign on every term; taken literally it grows
without bound, so the standard leapfrog that the stated time stencil defines
is the reading used here.)  Indices wrap around (periodic boundary).

Parity status: weights pinned by textbook values, a closed form and
polynomial exactness; the step by the Fourier symbol, time reversibility,
translation and transpose invariance and the convergence order
(tests/test_oracle_fd.py).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def weights_exact(r: int) -> list[Fraction]:
    """Central weights of the second derivative on unit spacing, order 2r,
    as exact rationals w[r + k], k = -r..r, from the Taylor moment
    conditions sum_k w_k k^p = 2 [p == 2], p = 0..2r, solved by Gaussian
    elimination over the rationals (symmetric weights: even p only)."""
    if r < 1:
        raise ValueError("stencil radius r must be >= 1")
    n = r + 1  # unknowns v_0 = w_0, v_k = w_k = w_{-k} (k = 1..r)
    A = []
    for q in range(n):  # moment p = 2q
        row = [Fraction(1 if q == 0 else 0)]
        row += [Fraction(2 * k ** (2 * q)) for k in range(1, r + 1)]
        row.append(Fraction(2 if q == 1 else 0))
        A.append(row)
    for c in range(n):
        piv = next(i for i in range(c, n) if A[i][c] != 0)
        A[c], A[piv] = A[piv], A[c]
        for i in range(n):
            if i != c and A[i][c] != 0:
                f = A[i][c] / A[c][c]
                A[i] = [a - f * b for a, b in zip(A[i], A[c])]
    v = [A[i][n] / A[i][i] for i in range(n)]
    return [v[abs(k)] for k in range(-r, r + 1)]


def weights(r: int) -> np.ndarray:
    return np.array([float(x) for x in weights_exact(r)])


def laplacian_unscaled(u: np.ndarray, r: int) -> np.ndarray:
    """sum_{k=-r..r} w_k (u(i+k, j) + u(i, j+k)) on a periodic grid stored as
    u[j, i], accumulated over k in ascending order (the pseudocode's order)."""
    w = weights(r)
    lap = np.zeros_like(u)
    for k in range(-r, r + 1):
        ux = np.roll(u, -k, axis=1)  # u(i + k, j)
        uy = np.roll(u, -k, axis=0)  # u(i, j + k)
        lap = lap + (w[r + k] * ux + w[r + k] * uy)
    return lap


def step(u_cur: np.ndarray, u_prev: np.ndarray, r: int, dt: float,
         dx: float) -> np.ndarray:
    """One leapfrog step: u_{n+1} from u_n (u_cur) and u_{n-1} (u_prev)."""
    u_cur = np.asarray(u_cur, dtype=np.float64)
    u_prev = np.asarray(u_prev, dtype=np.float64)
    c = (dt * dt) / (dx * dx)
    return 2.0 * u_cur - u_prev + c * laplacian_unscaled(u_cur, r)


def run(u_prev: np.ndarray, u_cur: np.ndarray, r: int, dt: float, dx: float,
        nsteps: int):
    """nsteps steps; returns (u_{n+K-1}, u_{n+K})."""
    a, b = np.asarray(u_prev, np.float64), np.asarray(u_cur, np.float64)
    for _ in range(nsteps):
        a, b = b, step(b, a, r, dt, dx)
    return a, b
