"""FP64 CPU oracle for the discontinuous-Galerkin volume term of the 2D
shallow-water equations (the paper's section 4.3).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the benchmark's CPU-baseline leg may import this module.  It shares no code
with the HIP product library and never imports it.

Equations (section 4.3.1): Q_t + F(Q)_x + G(Q)_y = S with Q = (h, hu, hv),
F = (hu, hu^2/h + g h^2/2, hu hv/h), G = (hv, hu hv/h, hv^2/h + g h^2/2),
S = (0, -g h B_x, -g h B_y), B the bathymetry.

Discretisation (section 4.3.2): conforming triangles, Q_H in P^N on each
element; the volume kernel is the element integral
    <F, dv/dx> + <G, dv/dy> + <S, v>   for every test function v in P^N,
here returned as nodal values after the inverse mass matrix (the form the
time stepper adds to): with the fluxes and source represented by their
nodal interpolants,
    rhs = Dxw F + Dyw G + S,   Dxw = M^-1 Dx^T M  (weak x-derivative),
and on an affine element Dxw = rx Drw + sx Dsw, Dyw = ry Drw + sy Dsw with
Drw = M^-1 Dr^T M, Dsw = M^-1 Ds^T M on the reference triangle.

Readings (the paper defers the nodal basis to the nodal-DG textbook it
cites): reference triangle with vertices (-1,-1), (1,-1), (-1,1); warp-and-
blend interpolation nodes (Warburton 2006) with the textbook's optimised
blending parameters; orthonormal (Dubiner / Koornwinder) modal basis for
the Vandermonde matrix; B_x, B_y the derivatives of the nodal interpolant of
B; affine elements with counterclockwise vertices.

Parity status: pinned in tests/test_oracle_dg.py by closed forms (N = 1, 2
nodes, edge nodes = Gauss-Lobatto points, symmetry), exact rational
integrals of monomials (mass matrix, weak derivatives), exact
differentiation of polynomials, affine-map identities, and the whole volume
term against collapsed-coordinate Gauss quadrature of polynomial states.
"""
from __future__ import annotations

import math

import numpy as np

# optimised blending parameters alpha(N), N = 1..15 (textbook table)
_ALPHA_OPT = [0.0000, 0.0000, 1.4152, 0.1001, 0.2751, 0.9800, 1.0999, 1.2832,
              1.3648, 1.4773, 1.4959, 1.5743, 1.5770, 1.6223, 1.6258]


def num_nodes(N: int) -> int:
    return (N + 1) * (N + 2) // 2


# ----------------------------------------------------------------------------
# 1D ingredients
# ----------------------------------------------------------------------------

def jacobi_p(x, alpha, beta, n):
    """Orthonormal Jacobi polynomial P_n^(alpha,beta) at x (weight
    (1-x)^alpha (1+x)^beta on [-1, 1]), by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    g0 = (2 ** (alpha + beta + 1) / (alpha + beta + 1) * math.gamma(alpha + 1)
          * math.gamma(beta + 1) / math.gamma(alpha + beta + 1))
    p_prev = np.zeros_like(x)
    p = np.full_like(x, 1.0 / math.sqrt(g0))
    if n == 0:
        return p
    g1 = (alpha + 1) * (beta + 1) / (alpha + beta + 3) * g0
    p_next = ((alpha + beta + 2) * x / 2 + (alpha - beta) / 2) / math.sqrt(g1)
    p_prev, p = p, p_next
    a_old = 2 / (2 + alpha + beta) * math.sqrt((alpha + 1) * (beta + 1)
                                               / (alpha + beta + 3))
    for i in range(1, n):
        h1 = 2 * i + alpha + beta
        a_new = 2 / (h1 + 2) * math.sqrt((i + 1) * (i + 1 + alpha + beta)
                                         * (i + 1 + alpha) * (i + 1 + beta)
                                         / (h1 + 1) / (h1 + 3))
        b_new = -(alpha ** 2 - beta ** 2) / h1 / (h1 + 2)
        p_new = (-a_old * p_prev + (x - b_new) * p) / a_new
        p_prev, p = p, p_new
        a_old = a_new
    return p


def grad_jacobi_p(x, alpha, beta, n):
    if n == 0:
        return np.zeros_like(np.asarray(x, dtype=np.float64))
    return math.sqrt(n * (n + alpha + beta + 1)) * jacobi_p(x, alpha + 1,
                                                            beta + 1, n - 1)


def gauss_lobatto(N):
    """Gauss-Lobatto points on [-1, 1]: endpoints and the roots of P_N'."""
    if N == 1:
        return np.array([-1.0, 1.0])
    c = np.zeros(N + 1)
    c[N] = 1.0
    inner = np.polynomial.legendre.legroots(np.polynomial.legendre.legder(c))
    return np.concatenate([[-1.0], np.sort(inner.real), [1.0]])


def _warp_factor(N, rout):
    """Interpolant, on equidistant nodes, of the displacement from the
    equidistant to the Gauss-Lobatto nodes, divided by (1 - r^2)."""
    rout = np.asarray(rout, dtype=np.float64)
    req = np.linspace(-1.0, 1.0, N + 1)
    disp = gauss_lobatto(N) - req
    warp = np.zeros_like(rout)
    for i in range(N + 1):
        li = np.ones_like(rout)
        for j in range(N + 1):
            if j != i:
                li = li * (rout - req[j]) / (req[i] - req[j])
        warp = warp + li * disp[i]
    inside = np.abs(rout) < 1.0 - 1e-10
    sf = np.where(inside, 1.0 - rout ** 2, 1.0)
    return np.where(inside, warp / sf, warp)


def nodes(N: int):
    """Warp-and-blend interpolation nodes on the reference triangle, (r, s)
    arrays of length Np, in the order n = 0..N (rows from the edge s = -1
    up), m = 0..N-n along each row."""
    alpha = _ALPHA_OPT[N - 1] if N <= 15 else 5.0 / 3.0
    L1, L3 = [], []
    for n in range(N + 1):
        for m in range(N + 1 - n):
            L1.append(n / N)
            L3.append(m / N)
    L1, L3 = np.array(L1), np.array(L3)
    L2 = 1.0 - L1 - L3
    x = -L2 + L3
    y = (-L2 - L3 + 2 * L1) / math.sqrt(3.0)
    b1, b2, b3 = 4 * L2 * L3, 4 * L1 * L3, 4 * L1 * L2
    w1 = b1 * _warp_factor(N, L3 - L2) * (1 + (alpha * L1) ** 2)
    w2 = b2 * _warp_factor(N, L1 - L3) * (1 + (alpha * L2) ** 2)
    w3 = b3 * _warp_factor(N, L2 - L1) * (1 + (alpha * L3) ** 2)
    c2, c3 = math.cos(2 * math.pi / 3), math.cos(4 * math.pi / 3)
    s2, s3 = math.sin(2 * math.pi / 3), math.sin(4 * math.pi / 3)
    x = x + w1 + c2 * w2 + c3 * w3
    y = y + s2 * w2 + s3 * w3
    # equilateral (x, y) -> reference (r, s) through barycentric coordinates
    l1 = (math.sqrt(3.0) * y + 1) / 3
    l2 = (-3 * x - math.sqrt(3.0) * y + 2) / 6
    l3 = (3 * x - math.sqrt(3.0) * y + 2) / 6
    return -l2 + l3 - l1, -l2 - l3 + l1


# ----------------------------------------------------------------------------
# orthonormal basis on the triangle, Vandermonde and operator matrices
# ----------------------------------------------------------------------------

def _collapse(r, s):
    a = np.where(np.abs(s - 1.0) > 1e-13, 2 * (1 + r) / (1 - s + 1e-300) - 1,
                 -1.0)
    return a, np.asarray(s, dtype=np.float64)


def basis(r, s, i, j):
    """psi_ij = sqrt(2) P_i(a) P_j^(2i+1,0)(b) (1-b)^i, orthonormal on the
    reference triangle (collapsed coordinates a, b)."""
    a, b = _collapse(r, s)
    return (math.sqrt(2.0) * jacobi_p(a, 0, 0, i)
            * jacobi_p(b, 2 * i + 1, 0, j) * (1 - b) ** i)


def grad_basis(r, s, i, j):
    a, b = _collapse(r, s)
    fa, dfa = jacobi_p(a, 0, 0, i), grad_jacobi_p(a, 0, 0, i)
    gb, dgb = jacobi_p(b, 2 * i + 1, 0, j), grad_jacobi_p(b, 2 * i + 1, 0, j)
    dr = dfa * gb
    if i > 0:
        dr = dr * (0.5 * (1 - b)) ** (i - 1)
    ds = dfa * (gb * (0.5 * (1 + a)))
    if i > 0:
        ds = ds * (0.5 * (1 - b)) ** (i - 1)
    tmp = dgb * (0.5 * (1 - b)) ** i
    if i > 0:
        tmp = tmp - 0.5 * i * gb * (0.5 * (1 - b)) ** (i - 1)
    ds = ds + fa * tmp
    scale = 2 ** (i + 0.5)
    return dr * scale, ds * scale


def _modes(N):
    return [(i, j) for i in range(N + 1) for j in range(N + 1 - i)]


def vandermonde(N, r, s):
    return np.stack([basis(r, s, i, j) for i, j in _modes(N)], axis=1)


def grad_vandermonde(N, r, s):
    g = [grad_basis(r, s, i, j) for i, j in _modes(N)]
    return (np.stack([x[0] for x in g], axis=1),
            np.stack([x[1] for x in g], axis=1))


def reference_operators(N):
    """Dict with nodes r, s and the matrices V, Dr, Ds, M (reference mass
    matrix (V V^T)^-1), Drw = M^-1 Dr^T M, Dsw = M^-1 Ds^T M."""
    r, s = nodes(N)
    V = vandermonde(N, r, s)
    Vr, Vs = grad_vandermonde(N, r, s)
    Vinv = np.linalg.inv(V)
    Dr, Ds = Vr @ Vinv, Vs @ Vinv
    M = np.linalg.inv(V @ V.T)
    Minv = V @ V.T
    return {"r": r, "s": s, "V": V, "Dr": Dr, "Ds": Ds, "M": M,
            "Drw": Minv @ Dr.T @ M, "Dsw": Minv @ Ds.T @ M}


# ----------------------------------------------------------------------------
# affine elements, shallow-water fluxes, the volume term
# ----------------------------------------------------------------------------

def geometric_factors(vx, vy, etov):
    """Per element (rx, sx, ry, sy, J) of the affine map from the reference
    triangle: x = -(r+s)/2 x1 + (1+r)/2 x2 + (1+s)/2 x3 (same for y)."""
    v = np.asarray(etov)
    x1, x2, x3 = vx[v[:, 0]], vx[v[:, 1]], vx[v[:, 2]]
    y1, y2, y3 = vy[v[:, 0]], vy[v[:, 1]], vy[v[:, 2]]
    xr, xs = (x2 - x1) / 2, (x3 - x1) / 2
    yr, ys = (y2 - y1) / 2, (y3 - y1) / 2
    J = xr * ys - xs * yr
    return ys / J, -yr / J, -xs / J, xr / J, J


def physical_nodes(ops, vx, vy, etov):
    v = np.asarray(etov)
    r, s = ops["r"], ops["s"]
    la, lb, lc = -(r + s) / 2, (1 + r) / 2, (1 + s) / 2
    X = (np.outer(vx[v[:, 0]], la) + np.outer(vx[v[:, 1]], lb)
         + np.outer(vx[v[:, 2]], lc))
    Y = (np.outer(vy[v[:, 0]], la) + np.outer(vy[v[:, 1]], lb)
         + np.outer(vy[v[:, 2]], lc))
    return X, Y


def bathymetry_gradient(ops, geo, B):
    """Nodal x- and y-derivatives of the nodal interpolant of B [E][Np]."""
    rx, sx, ry, sy, _ = geo
    Br, Bs = B @ ops["Dr"].T, B @ ops["Ds"].T
    return rx[:, None] * Br + sx[:, None] * Bs, ry[:, None] * Br + sy[:, None] * Bs


def fluxes(Q, g):
    """F, G, the nodal fluxes, from Q [E][3][Np]."""
    h, hu, hv = Q[:, 0], Q[:, 1], Q[:, 2]
    u, v = hu / h, hv / h
    F = np.stack([hu, hu * u + 0.5 * g * h * h, hu * v], axis=1)
    G = np.stack([hv, hv * u, hv * v + 0.5 * g * h * h], axis=1)
    return F, G


def volume_rhs(ops, geo, Q, Bx, By, g):
    """rhs [E][3][Np] = Dxw F + Dyw G + S on every element."""
    rx, sx, ry, sy, _ = geo
    F, G = fluxes(np.asarray(Q, dtype=np.float64), g)
    Fr = rx[:, None, None] * F + ry[:, None, None] * G
    Fs = sx[:, None, None] * F + sy[:, None, None] * G
    rhs = Fr @ ops["Drw"].T + Fs @ ops["Dsw"].T
    h = Q[:, 0]
    rhs[:, 1] += -g * h * Bx
    rhs[:, 2] += -g * h * By
    return rhs


def volume_flops(N: int) -> int:
    """Floating-point operations per element counted for the GFLOP/s metric:
    the two Np x Np products per component (2 Np^2 multiply-adds each, two
    flops per multiply-add) and the nodal work (fluxes, metric combinations,
    source), 32 per node."""
    Np = num_nodes(N)
    return 3 * 2 * 2 * Np * Np + 32 * Np
