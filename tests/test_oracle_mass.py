"""Pins of the oracle's mass term: the screened equation
-div(kappa grad u) + alpha u = f of section 4.2 (equation semPDE), whose weak
form (equation semOperator) adds (alpha u, v); GLL quadrature lumps it to the
diagonal alpha(X) w_i w_j w_k J (section 4.2.1, discrete orthogonality).

Each check fails on a plausible slip in H = alpha B or in where it enters
(missing J or weight, alpha applied twice, mass added per global instead of
per local node, mass missing from the Jacobi diagonal):
  1. affine closed form H = alpha w_i w_j w_k hx hy hz / 8 with the textbook
     GLL weights;
  2. sum of H integrates alpha(X) exactly (constant and linear alpha, on the
     affine cube and on the det J = 1 sine map);
  3. N = 1: the assembled operator is h times the 7-point stencil plus
     alpha h^3 on the diagonal;
  4. for u in Q_{N-1} on affine meshes, interior rows equal
     B (-Laplace u + alpha u) at the node, for constant and nodal alpha;
  5. brute force: element mass matrices from explicitly evaluated Lagrange
     basis values, assembled with the stiffness, equal the fast operator;
  6. without Dirichlet faces the operator is SPD for alpha > 0 and A 1 is
     the assembled alpha B;
  7. spectral convergence to the manufactured solution of the screened
     equation, and PCG agreeing with a sparse direct solve."""
import numpy as np
import pytest

from oracle import oracle as orc
from seminputs import uniform


def _dense_global(m):
    A = np.zeros((m.nG, m.nG))
    e = np.zeros(m.nG)
    for g in range(m.nG):
        e[g] = 1.0
        A[:, g] = orc.apply_global(m, e)
        e[g] = 0.0
    return A


def _global_coords(m):
    Xg = np.zeros((3, m.nG))
    Xg[:, m.l2g] = m.X
    return Xg


def test_mass_factor_affine_closed_form():
    # GLL weights for N = 3 (textbook): 1/6, 5/6, 5/6, 1/6
    w = np.array([1 / 6, 5 / 6, 5 / 6, 1 / 6])
    alpha, ex, ey, ez = 2.5, 2, 3, 2
    m = orc.mesh(3, ex, ey, ez, orc.MAP_AFFINE, alpha=alpha)
    hx, hy, hz = 1 / ex, 1 / ey, 1 / ez
    wq = (w[None, None, :] * w[None, :, None] * w[:, None, None]).reshape(-1)
    ref = np.tile(alpha * wq * hx * hy * hz / 8, m.E)
    assert np.max(np.abs(m.H - ref)) < 1e-14 * np.max(ref)


@pytest.mark.parametrize("N", [1, 3, 6])
@pytest.mark.parametrize("mapping", [orc.MAP_AFFINE, orc.MAP_SINE_X])
def test_mass_integrates_alpha(N, mapping):
    """Constant alpha: sum H = alpha |Omega| = alpha.  alpha(X) = 1 + X: the
    integral of 1 + x over the image is 3/2 on both meshes (det J = 1 for the
    sine map, whose shift integrates to zero by symmetry), and the
    quadrature is exact for this degree-N integrand."""
    m = orc.mesh(N, 3, 2, 3, mapping, alpha=0.75)
    assert abs(m.H.sum() - 0.75) < 1e-13
    m2 = orc.mesh(N, 3, 2, 3, mapping, alpha_nodal=1.0 + orc.coords(
        N, 3, 2, 3, mapping)[0])
    assert abs(m2.H.sum() - 1.5) < 1e-13


def test_n1_is_stencil_plus_lumped_mass():
    n, alpha = 4, 3.0
    m = orc.mesh(1, n, n, n, orc.MAP_AFFINE, dirichlet=0, alpha=alpha)
    A = _dense_global(m)
    h = 1.0 / n
    Gd = n + 1
    for gz in range(1, Gd - 1):
        for gy in range(1, Gd - 1):
            for gx in range(1, Gd - 1):
                g = gx + Gd * (gy + Gd * gz)
                row = A[g].copy()
                assert abs(row[g] - (6 * h + alpha * h ** 3)) < 1e-14
                for d in (1, Gd, Gd * Gd):
                    assert abs(row[g + d] + h) < 1e-14
                    assert abs(row[g - d] + h) < 1e-14
                    row[g + d] = row[g - d] = 0
                row[g] = 0
                assert np.max(np.abs(row)) < 1e-14


POLYS = [
    (lambda x, y, z: x ** 2, lambda x, y, z: -2.0 + 0 * x),
    (lambda x, y, z: x * y * z, lambda x, y, z: 0 * x),
    (lambda x, y, z: x ** 3 * y + z ** 2 * y, lambda x, y, z: -6 * x * y - 2 * y),
]


@pytest.mark.parametrize("k", range(len(POLYS)))
@pytest.mark.parametrize("nodal", [False, True])
def test_exact_on_polynomials_with_mass(k, nodal):
    """The lumped mass acts pointwise, so with u in Q_{N-1} on an affine mesh
    every interior row of the assembled Neumann operator equals
    B_b (-Laplace u + alpha u)(x_b), for constant and variable alpha."""
    N = 4
    u_f, lap_f = POLYS[k]
    X = orc.coords(N, 3, 2, 4, orc.MAP_AFFINE)
    if nodal:
        a_l = 1.0 + X[0] ** 2 + 0.5 * X[1] * X[2]
        m = orc.mesh(N, 3, 2, 4, orc.MAP_AFFINE, dirichlet=0, alpha_nodal=a_l)
    else:
        m = orc.mesh(N, 3, 2, 4, orc.MAP_AFFINE, dirichlet=0, alpha=2.0)
    Xg = _global_coords(m)
    a_g = 1.0 + Xg[0] ** 2 + 0.5 * Xg[1] * Xg[2] if nodal else 2.0
    u = u_f(*Xg)
    Au = orc.apply_global(m, u)
    Bg = orc.to_global(m, orc.gs(m, m.B))
    ref = Bg * (lap_f(*Xg) + a_g * u)
    interior = np.all((Xg > 1e-12) & (Xg < 1 - 1e-12), axis=0)
    scale = np.max(np.abs(orc.to_global(m, orc.ax_abs(m, orc.to_local(m, u)))))
    err = np.max(np.abs(Au[interior] - ref[interior]))
    assert err < 1e-13 * scale, (err, scale)


@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_brute_force_with_mass_2x2x2(N):
    m0 = orc.mesh(N, 2, 2, 2, orc.MAP_SINE_CYCLIC, dirichlet=0)
    a_l = orc.to_local(m0, 1.5 + uniform(m0.nG, seed=11))
    m = orc.mesh(N, 2, 2, 2, orc.MAP_SINE_CYCLIC, dirichlet=0, alpha_nodal=a_l)
    A = _dense_global(m)
    S = orc.assemble_sparse(m).toarray()
    assert np.max(np.abs(A - S)) < 1e-13 * np.max(np.abs(S))
    # the brute-force mass matrix is diagonal: GLL lumping is exact here
    Me = orc.brute_element_mass(N, m.xi, m.H[: m.n1 ** 3])
    off = Me - np.diag(np.diag(Me))
    assert np.max(np.abs(off)) < 1e-14 * np.max(np.abs(Me))
    assert np.max(np.abs(np.diag(Me) - m.H[: m.n1 ** 3])) < 1e-14 * np.max(m.H)


@pytest.mark.parametrize("N", [2, 4])
def test_diagonal_with_mass_matches_brute_force(N):
    m = orc.mesh(N, 2, 2, 2, orc.MAP_SINE_CYCLIC, dirichlet=1, alpha=4.0)
    S = orc.assemble_sparse(m).toarray()
    dinv = orc.jacobi_dinv_global(m)
    free = dinv != 0
    assert np.max(np.abs(1.0 / dinv[free] - np.diag(S)[free])) < \
        1e-13 * np.max(np.diag(S))


def test_neumann_with_mass_is_spd():
    alpha = 0.5
    m = orc.mesh(2, 2, 2, 2, orc.MAP_SINE_CYCLIC, dirichlet=0, alpha=alpha)
    A = _dense_global(m)
    assert np.max(np.abs(A - A.T)) < 1e-13 * np.max(np.abs(A))
    lam = np.linalg.eigvalsh(0.5 * (A + A.T))
    assert lam[0] > 0.1 * alpha * np.min(orc.to_global(m, orc.gs(m, m.B)))
    # the stiffness annihilates constants: A 1 is the assembled alpha B
    a1 = orc.apply_global(m, np.ones(m.nG))
    hb = orc.to_global(m, orc.gs(m, m.H))
    assert np.max(np.abs(a1 - hb)) < 1e-13 * np.max(np.abs(A))


def _screened_error(N, n, alpha):
    m = orc.mesh(N, n, n, n, orc.MAP_AFFINE, dirichlet=1, alpha=alpha)
    # f = (3 pi^2 + alpha) u* for u* = sin(pi x) sin(pi y) sin(pi z)
    f = orc.src_sine(m.X) * (1.0 + alpha / (3 * np.pi ** 2))
    b = orc.to_global(m, orc.rhs_local(m, f))
    x, st, it, _ = orc.pcg(m, b, 1e-13, 2000)
    assert st == 0
    Xg = _global_coords(m)
    ue = np.sin(np.pi * Xg[0]) * np.sin(np.pi * Xg[1]) * np.sin(np.pi * Xg[2])
    return np.max(np.abs(x - ue))


def test_screened_manufactured_p_convergence():
    errs = [_screened_error(N, 3, 20.0) for N in range(2, 9)]
    assert all(errs[i + 1] < 0.25 * errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-10


@pytest.mark.parametrize("dirichlet", [0, 1])
def test_pcg_with_mass_matches_sparse_direct_solve(dirichlet):
    import scipy.sparse.linalg as spla
    m = orc.mesh(3, 2, 3, 2, orc.MAP_SINE_CYCLIC, dirichlet=dirichlet,
                 alpha=1.0)
    b = orc.to_global(m, orc.rhs_local(m, 1.0 + m.X[0] * m.X[1]))
    x, st, it, _ = orc.pcg(m, b, 1e-13, 5000)
    assert st == 0
    S = orc.assemble_sparse(m, masked=bool(dirichlet)).tocsc()
    if dirichlet:
        free = np.ones(m.nG, bool)
        free[m.l2g[m.bmask.astype(bool)]] = False
        xs = np.zeros(m.nG)
        xs[free] = spla.spsolve(S[free][:, free], b[free])
    else:
        xs = spla.spsolve(S, b)
    assert np.max(np.abs(x - xs)) < 1e-10 * np.max(np.abs(xs))
