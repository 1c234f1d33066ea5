"""Pins of the oracle's solvers (paper section 4.2.2: the SEM system is
solved by preconditioned conjugate gradients): agreement with a sparse
direct solve of the brute-force assembled system, the convergence of the
manufactured-solution discretisation error in h and N, flexible CG, and the
right-hand-side assembly."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import oracle as orc
from seminputs import fourier_modes, grf_features


def _kappa():
    omega, b, sigma = grf_features(seed=7, M=64, ell=0.3, sigma=0.5)
    return omega, b, sigma


@pytest.mark.parametrize("N,ex,ey,ez", [(2, 3, 2, 2), (3, 2, 2, 2), (5, 2, 1, 2)])
def test_pcg_matches_sparse_direct_solve(N, ex, ey, ez):
    m = orc.mesh(N, ex, ey, ez, orc.MAP_SINE_CYCLIC, dirichlet=1,
                 kappa_params=_kappa())
    k, a, phi = fourier_modes(seed=0)
    b = orc.to_global(m, orc.rhs_local(m, orc.src_fourier(m.X, k, a, phi)))
    A = orc.assemble_sparse(m, masked=True)
    free = np.ones(m.nG, bool)
    free[m.l2g[m.bmask.astype(bool)]] = False
    x_ref = np.zeros(m.nG)
    Af = A[free][:, free].tocsc()
    x_ref[free] = spla.spsolve(Af, b[free])
    for jac in (True, False):
        x, st, it, hist = orc.pcg(m, b, 1e-13, 5000, jacobi=jac)
        assert st == 0
        cond = np.linalg.cond(Af.toarray())
        assert np.linalg.norm(x - x_ref) <= 1e-13 * cond * np.linalg.norm(x_ref)
        assert hist[-1] <= 1e-13
        assert orc.true_rel_residual(m, b, x) < 1e-12


def _manufactured_error(N, n):
    m = orc.mesh(N, n, n, n, orc.MAP_AFFINE, dirichlet=1)
    b = orc.to_global(m, orc.rhs_local(m, orc.src_sine(m.X)))
    x, st, it, _ = orc.pcg(m, b, 1e-13, 2000)
    assert st == 0
    Xg = np.zeros((3, m.nG))
    Xg[:, m.l2g] = m.X
    ue = np.sin(np.pi * Xg[0]) * np.sin(np.pi * Xg[1]) * np.sin(np.pi * Xg[2])
    return np.max(np.abs(x - ue))


def test_manufactured_p_convergence():
    """u = sin(pi x) sin(pi y) sin(pi z) on 4^3 elements: the nodal error
    falls exponentially in N (spectral convergence)."""
    errs = [_manufactured_error(N, 4) for N in range(2, 9)]
    assert all(errs[i + 1] < 0.2 * errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-12


@pytest.mark.parametrize("N", [1, 2, 3])
def test_manufactured_h_convergence(N):
    """Nodal error falls at least like h^(N+1) under uniform refinement."""
    e1, e2, e3 = (_manufactured_error(N, n) for n in (2, 4, 8))
    r1, r2 = np.log2(e1 / e2), np.log2(e2 / e3)
    assert r2 > N + 1 - 0.2, (r1, r2)


def test_rhs_assembly_integrates_constants():
    """With f = 1 the assembled load vector sums to the domain volume."""
    m = orc.mesh(4, 2, 3, 2, orc.MAP_SINE_CYCLIC, dirichlet=0)
    b = orc.to_global(m, orc.rhs_local(m, np.ones(m.nL)))
    assert abs(b.sum() - 1.0) < 1e-13


def test_fourier_source_is_smooth_sum_of_modes():
    k, a, phi = fourier_modes(seed=0)
    X = np.random.default_rng(0).uniform(0, 1, (3, 50))
    f = orc.src_fourier(X, k, a, phi)
    ref = sum(a[m] * np.cos(2 * np.pi * (k[m] @ X) + phi[m]) for m in range(8))
    np.testing.assert_allclose(f, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("N", [3, 5])
def test_fcg_with_fixed_jacobi_equals_pcg(N):
    """With a fixed SPD preconditioner, -(z_{k+1}, A p_k)/(p_k, A p_k) equals
    (z_{k+1}, r_{k+1})/(z_k, r_k) in exact arithmetic (A p_k = (r_k -
    r_{k+1})/alpha_k and (z_{k+1}, r_k) = 0), so flexible CG reproduces PCG."""
    m = orc.mesh(N, 3, 3, 2, orc.MAP_SINE_CYCLIC, dirichlet=1,
                 kappa_params=_kappa())
    k, a, phi = fourier_modes(seed=1)
    b = orc.to_global(m, orc.rhs_local(m, orc.src_fourier(m.X, k, a, phi)))
    dinv = orc.jacobi_dinv_global(m)
    x1, s1, i1, _ = orc.pcg(m, b, 1e-10, 2000)
    x2, s2, i2, _ = orc.fcg(m, b, lambda r: dinv * r, 1e-10, 2000)
    assert s1 == 0 and s2 == 0
    assert abs(i1 - i2) <= 2
    assert np.linalg.norm(x1 - x2) < 1e-8 * np.linalg.norm(x1)


def test_jacobi_reduces_iterations_on_variable_kappa():
    m = orc.mesh(3, 4, 4, 4, orc.MAP_AFFINE, dirichlet=1,
                 kappa_params=grf_features(seed=7, M=256, ell=0.1, sigma=1.0))
    k, a, phi = fourier_modes(seed=2)
    b = orc.to_global(m, orc.rhs_local(m, orc.src_fourier(m.X, k, a, phi)))
    _, s1, i_j, _ = orc.pcg(m, b, 1e-8, 5000, jacobi=True)
    _, s2, i_n, _ = orc.pcg(m, b, 1e-8, 5000, jacobi=False)
    assert s1 == 0 and s2 == 0 and i_j < i_n
