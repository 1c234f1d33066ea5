"""FP64 CPU oracle for the spectral-element Poisson operator (paper section 4.2).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the benchmark's CPU-baseline leg may import this module.  It shares no code
with the HIP product library and never imports it.

Two layers:

* ctypes wrappers over ``libsemoracle.so`` (plain C loops, see
  ``sem_oracle.c``): GLL nodes, derivative matrix, maps, geometry, the local
  operator ``w = D^T G D u``, gather-scatter, Jacobi diagonal, PCG and FCG;
* a brute-force layer in NumPy/SciPy that builds each dense element matrix
  from explicitly differentiated Lagrange polynomials (no sum
  factorisation, no derivative matrix) and assembles the global sparse
  matrix -- the independent check of the fast operator.

Parity status per function is recorded in the header of ``sem_oracle.h``
and pinned by ``tests/test_oracle_*.py``; the MLP part (``mlp_*``) is
pinned by finite differences; trained weights are "parity unpinned".
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libsemoracle.so")
_lib = None

MAP_AFFINE, MAP_SINE_X, MAP_SINE_CYCLIC = 0, 1, 2

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i64 = C.c_int64


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            import importlib.util
            spec = importlib.util.spec_from_file_location(
                "build_oracle", os.path.join(HERE, "build_oracle.py"))
            mod = importlib.util.module_from_spec(spec)
            spec.loader.exec_module(mod)
            mod.build()
        _lib = C.CDLL(_LIB_PATH)
        L = _lib
        L.orc_num_threads.argtypes = []
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_gll.argtypes = [C.c_int, _dp, _dp]
        L.orc_gll.restype = C.c_int
        L.orc_dmat.argtypes = [C.c_int, _dp, _dp]
        L.orc_num_global.argtypes = [C.c_int] * 5
        L.orc_num_global.restype = _i64
        L.orc_maps.argtypes = [C.c_int] * 6 + [_ip, _ip, _ip, _ip, _up]
        L.orc_coords.argtypes = [C.c_int] * 5 + [_dp, _dp]
        L.orc_geom.argtypes = [C.c_int, _i64, _dp, _dp, _dp, C.c_void_p, _dp,
                               _dp, C.POINTER(C.c_double)]
        L.orc_ax.argtypes = [C.c_int, _i64, _dp, _dp, _dp, _dp]
        L.orc_ax_abs.argtypes = [C.c_int, _i64, _dp, _dp, _dp, _dp]
        L.orc_gs.argtypes = [_i64, _i64, _ip, _up, _dp, _dp]
        L.orc_diag.argtypes = [C.c_int, _i64, _dp, _dp, _dp]
        L.orc_src_fourier.argtypes = [_i64, _dp, C.c_int, _dp, _dp, _dp, _dp]
        L.orc_src_sine.argtypes = [_i64, _dp, _dp]
        L.orc_kappa_rff.argtypes = [_i64, _dp, C.c_int, _dp, _dp, C.c_double,
                                    _dp]
        L.orc_apply_global.argtypes = [C.c_int, _i64, _i64, _ip, _up, _dp, _dp,
                                       C.c_void_p, _dp, _dp]
        L.orc_pcg.argtypes = [C.c_int, _i64, _i64, _ip, _up, _dp, _dp,
                              C.c_void_p, C.c_void_p, _dp, _dp, C.c_double,
                              C.c_int, C.POINTER(C.c_int), _dp]
        L.orc_pcg.restype = C.c_int
        L.orc_fcg.argtypes = [C.c_int, _i64, _i64, _ip, _up, _dp, _dp,
                              C.c_void_p, C.c_void_p, C.c_void_p, _dp, _dp,
                              C.c_double, C.c_int, C.POINTER(C.c_int), _dp]
        L.orc_fcg.restype = C.c_int
    return _lib


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ----------------------------------------------------------------------------
# Reference element (GLL nodes, weights, derivative matrix)
# ----------------------------------------------------------------------------

def gll(N: int):
    xi = np.zeros(N + 1)
    w = np.zeros(N + 1)
    if lib().orc_gll(N, xi, w) < 0:
        raise ValueError(f"GLL Newton failed for N={N}")
    return xi, w


def dmat(N: int, xi=None):
    if xi is None:
        xi, _ = gll(N)
    D = np.zeros((N + 1) * (N + 1))
    lib().orc_dmat(N, _f64(xi), D)
    return D.reshape(N + 1, N + 1)


# ----------------------------------------------------------------------------
# Mesh
# ----------------------------------------------------------------------------

@dataclass
class Mesh:
    N: int
    ex: int
    ey: int
    ez: int
    dirichlet: int
    mapping: int
    xi: np.ndarray
    w: np.ndarray
    D: np.ndarray
    l2g: np.ndarray
    perm: np.ndarray
    offsets: np.ndarray
    mult: np.ndarray
    bmask: np.ndarray
    X: np.ndarray        # (3, nL)
    G: np.ndarray        # (E, 6, n1^3)
    B: np.ndarray        # (nL,)
    minJ: float
    kappa: np.ndarray | None
    # lumped mass term of the weak form (section 4.2.1): H = alpha(X) B per
    # local node, or None when alpha = 0
    H: np.ndarray | None = None
    periodic: int = 0    # bit 1 x, 2 y, 4 z

    @property
    def n1(self):
        return self.N + 1

    @property
    def E(self):
        return self.ex * self.ey * self.ez

    @property
    def nL(self):
        return self.E * self.n1 ** 3

    @property
    def nG(self):
        return int(self.offsets.shape[0] - 1)


def maps(N, ex, ey, ez, dirichlet=1, periodic=0):
    """Distinct global-local numbering; ``periodic`` bit 1 x, 2 y, 4 z
    identifies the faces at 0 and 1 of that direction (no Dirichlet mask
    there)."""
    n1 = N + 1
    nL = ex * ey * ez * n1 ** 3
    nG = int(lib().orc_num_global(N, ex, ey, ez, int(periodic)))
    l2g = np.zeros(nL, np.int32)
    perm = np.zeros(nL, np.int32)
    offsets = np.zeros(nG + 1, np.int32)
    mult = np.zeros(nL, np.int32)
    bmask = np.zeros(nL, np.uint8)
    lib().orc_maps(N, ex, ey, ez, int(dirichlet), int(periodic), l2g, perm,
                   offsets, mult, bmask)
    return l2g, perm, offsets, mult, bmask


def coords(N, ex, ey, ez, mapping, xi=None):
    if xi is None:
        xi, _ = gll(N)
    nL = ex * ey * ez * (N + 1) ** 3
    X = np.zeros(3 * nL)
    lib().orc_coords(N, ex, ey, ez, int(mapping), _f64(xi), X)
    return X.reshape(3, nL)


def kappa_rff(X, omega, b, sigma):
    """kappa = exp(g), g a random-Fourier-feature Gaussian field."""
    X = _f64(X)
    n = X.shape[1]
    out = np.zeros(n)
    omega = _f64(omega).reshape(-1, 3)
    lib().orc_kappa_rff(n, X.reshape(-1), omega.shape[0], omega.reshape(-1),
                        _f64(b), float(sigma), out)
    return out


def geom(N, E, w, D, X, kappa=None):
    n3 = (N + 1) ** 3
    G = np.zeros(E * 6 * n3)
    B = np.zeros(E * n3)
    mj = C.c_double(0)
    kp = None
    if kappa is not None:
        kappa = _f64(kappa)
        kp = kappa.ctypes.data_as(C.c_void_p)
    lib().orc_geom(N, E, _f64(w), _f64(D).reshape(-1), _f64(X).reshape(-1), kp,
                   G, B, C.byref(mj))
    return G.reshape(E, 6, n3), B, mj.value


def mesh(N, ex, ey, ez, mapping=MAP_AFFINE, dirichlet=1, kappa_params=None,
         alpha=0.0, alpha_nodal=None, periodic=0):
    """Build everything the operator needs.  ``kappa_params`` is
    ``(omega[M,3], b[M], sigma)`` for kappa = exp(GRF) or None (kappa = 1).
    The mass coefficient alpha(X) of the screened equation is the constant
    ``alpha`` or, when given, the nodal array ``alpha_nodal`` (E-vector).
    ``periodic`` (bit 1 x, 2 y, 4 z) makes those directions periodic: each
    element keeps its own node positions (the copies of a node on the
    identified faces sit at 0 and at 1)."""
    xi, w = gll(N)
    D = dmat(N, xi)
    l2g, perm, offsets, mult, bmask = maps(N, ex, ey, ez, dirichlet, periodic)
    X = coords(N, ex, ey, ez, mapping, xi)
    kappa = None
    if kappa_params is not None:
        kappa = kappa_rff(X, *kappa_params)
    G, B, mj = geom(N, ex * ey * ez, w, D, X, kappa)
    H = None
    if alpha_nodal is not None:
        H = _f64(alpha_nodal).reshape(-1) * B
    elif alpha != 0.0:
        H = float(alpha) * B
    return Mesh(N, ex, ey, ez, int(dirichlet), int(mapping), xi, w, D, l2g,
                perm, offsets, mult, bmask, X, G, B, mj, kappa, H, int(periodic))


def _hptr(m: Mesh):
    """C pointer to the mass factor (None without a mass term)."""
    if m.H is None:
        return None
    return _f64(m.H).ctypes.data_as(C.c_void_p)


# ----------------------------------------------------------------------------
# Operator, gather-scatter, diagonal, sources
# ----------------------------------------------------------------------------

def ax(m: Mesh, u, E=None):
    """Unassembled local operator w_L = A_L u_L (all elements, or the first
    ``E`` elements of ``u`` when E is given)."""
    E = m.E if E is None else E
    u = _f64(u).reshape(-1)
    assert u.shape[0] == E * m.n1 ** 3
    w = np.zeros_like(u)
    lib().orc_ax(m.N, E, _f64(m.D).reshape(-1), _f64(m.G[:E]).reshape(-1), u, w)
    if m.H is not None:
        w += m.H[: u.shape[0]] * u
    return w


def ax_raw(N, D, G, u):
    """Operator on raw arrays: G (E,6,n1^3), u (E*n1^3)."""
    G = _f64(G)
    E = G.shape[0]
    u = _f64(u).reshape(-1)
    w = np.zeros_like(u)
    lib().orc_ax(N, E, _f64(D).reshape(-1), G.reshape(-1), u, w)
    return w


def ax_abs(m: Mesh, u):
    u = _f64(u).reshape(-1)
    w = np.zeros_like(u)
    lib().orc_ax_abs(m.N, m.E, _f64(m.D).reshape(-1), _f64(m.G).reshape(-1), u,
                     w)
    if m.H is not None:
        w += np.abs(m.H) * np.abs(u)
    return w


def gs(m: Mesh, v):
    v = _f64(v).reshape(-1).copy()
    acc = np.zeros(m.nG)
    lib().orc_gs(m.nL, m.nG, m.l2g, m.bmask, v, acc)
    return v


def local_diag(m: Mesh):
    d = np.zeros(m.nL)
    lib().orc_diag(m.N, m.E, _f64(m.D).reshape(-1), _f64(m.G).reshape(-1), d)
    if m.H is not None:
        d += m.H
    return d


def jacobi_dinv_global(m: Mesh):
    """Inverse of the assembled diagonal on unique nodes (0 on Dirichlet
    nodes), the diagonal summed in ascending local order (the gs
    order), so the values are reproducible bit for bit."""
    d = local_diag(m)
    v = d.copy()
    acc = np.zeros(m.nG)
    # pass 1 of gs only (no mask): sums in ascending l
    lib().orc_gs(m.nL, m.nG, m.l2g, np.zeros(m.nL, np.uint8), v, acc)
    dg = np.zeros(m.nG)
    dg[m.l2g] = v
    masked = np.zeros(m.nG, bool)
    masked[m.l2g[m.bmask.astype(bool)]] = True
    return np.where(masked, 0.0, 1.0 / np.where(dg == 0, 1.0, dg))


def src_fourier(X, k, a, phi):
    X = _f64(X)
    n = X.shape[1]
    f = np.zeros(n)
    k = _f64(k).reshape(-1, 3)
    lib().orc_src_fourier(n, X.reshape(-1), k.shape[0], k.reshape(-1), _f64(a),
                          _f64(phi), f)
    return f


def src_sine(X):
    X = _f64(X)
    n = X.shape[1]
    f = np.zeros(n)
    lib().orc_src_sine(n, X.reshape(-1), f)
    return f


def rhs_local(m: Mesh, f):
    """b_L = mask o Q Q^T (B o f): the assembled load vector, E-vector form."""
    return gs(m, m.B * _f64(f))


def to_global(m: Mesh, v_local):
    """Unique vector from a continuous E-vector (any copy)."""
    out = np.zeros(m.nG)
    out[m.l2g] = v_local
    return out


def to_local(m: Mesh, v_global):
    return _f64(v_global)[m.l2g]


def apply_global(m: Mesh, x):
    y = np.zeros(m.nG)
    lib().orc_apply_global(m.N, m.E, m.nG, m.l2g, m.bmask,
                           _f64(m.D).reshape(-1), _f64(m.G).reshape(-1),
                           _hptr(m), _f64(x), y)
    return y


def pcg(m: Mesh, b_global, rtol, maxit, jacobi=True, x0=None):
    """Jacobi-PCG (or plain CG) on unique vectors.  Returns
    (x, status, iters, hist)."""
    x = np.zeros(m.nG) if x0 is None else _f64(x0).copy()
    hist = np.zeros(maxit + 1)
    it = C.c_int(0)
    dinv = None
    dv = None
    if jacobi:
        dinv = jacobi_dinv_global(m)
        dv = dinv.ctypes.data_as(C.c_void_p)
    st = lib().orc_pcg(m.N, m.E, m.nG, m.l2g, m.bmask, _f64(m.D).reshape(-1),
                       _f64(m.G).reshape(-1), _hptr(m), dv, _f64(b_global), x,
                       float(rtol), int(maxit), C.byref(it), hist)
    return x, st, it.value, hist[: it.value + 1]


_PREC_FN = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.POINTER(C.c_double),
                       C.c_void_p)


def fcg(m: Mesh, b_global, precond, rtol, maxit, x0=None):
    """Flexible CG with a Python preconditioner ``precond(r) -> z`` acting on
    unique vectors.  Returns (x, status, iters, hist)."""
    nG = m.nG
    x = np.zeros(nG) if x0 is None else _f64(x0).copy()
    hist = np.zeros(maxit + 1)
    it = C.c_int(0)

    def cb(rp, zp, ctx):
        r = np.ctypeslib.as_array(rp, shape=(nG,))
        z = np.ctypeslib.as_array(zp, shape=(nG,))
        z[:] = precond(r.copy())

    fn = _PREC_FN(cb)
    st = lib().orc_fcg(m.N, m.E, nG, m.l2g, m.bmask, _f64(m.D).reshape(-1),
                       _f64(m.G).reshape(-1), _hptr(m), C.cast(fn, C.c_void_p),
                       None,
                       _f64(b_global), x, float(rtol), int(maxit),
                       C.byref(it), hist)
    return x, st, it.value, hist[: it.value + 1]


def true_rel_residual(m: Mesh, b_global, x_global):
    r = _f64(b_global) - apply_global(m, x_global)
    return float(np.linalg.norm(r) / np.linalg.norm(b_global))


# ----------------------------------------------------------------------------
# Brute force: dense element matrices from explicit Lagrange derivatives
# ----------------------------------------------------------------------------

def lagrange_derivs_at_nodes(xi):
    """L[a][m] = l_a'(xi_m) from the monomial coefficients of each Lagrange
    polynomial (numpy.polynomial), independent of the closed-form D."""
    n1 = len(xi)
    out = np.zeros((n1, n1))
    for a in range(n1):
        others = np.delete(xi, a)
        c = np.polynomial.polynomial.polyfromroots(others)
        c = c / np.polynomial.polynomial.polyval(xi[a], c)
        dc = np.polynomial.polynomial.polyder(c)
        out[a] = np.polynomial.polynomial.polyval(xi, dc)
    return out


def brute_element_matrix(N, xi, Ge):
    """(A_e)_{pq} = sum over quadrature nodes nu of
    sum_ab G_ab(nu) d_a phi_p(nu) d_b phi_q(nu), with phi_p = l_i l_j l_k and
    G_ab the weighted metric (w J kappa grad r_a . grad r_b) at nu."""
    n1 = N + 1
    n3 = n1 ** 3
    L = lagrange_derivs_at_nodes(np.asarray(xi))  # L[a][m] = l_a'(xi_m)
    I = np.eye(n1)                                 # l_a(xi_m) = delta
    # gradient matrices: grad[d][nu, p] = d_d phi_p at node nu
    # node nu = (m, n, o) with index m + n1 n + n1^2 o; p = (i, j, k) likewise
    # phi_p(nu) = l_i(m) l_j(n) l_k(o)
    # kron order: index = m + n1*n + n1^2*o  ->  np.kron(O, N, M)
    Dr = np.kron(I, np.kron(I, L.T))   # [nu, p] = l_i'(xi_m) d_jn d_ko
    Ds = np.kron(I, np.kron(L.T, I))
    Dt = np.kron(L.T, np.kron(I, I))
    grads = [Dr, Ds, Dt]
    Gfull = np.zeros((3, 3, n3))
    pairs = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    for q, (a, b) in enumerate(pairs):
        Gfull[a, b] = Ge[q]
        Gfull[b, a] = Ge[q]
    A = np.zeros((n3, n3))
    for a in range(3):
        for b in range(3):
            A += grads[a].T @ (Gfull[a, b][:, None] * grads[b])
    return A


def lagrange_values_at_nodes(xi):
    """V[a][m] = l_a(xi_m), each Lagrange polynomial evaluated from its
    monomial coefficients (the identity up to rounding)."""
    n1 = len(xi)
    out = np.zeros((n1, n1))
    for a in range(n1):
        c = np.polynomial.polynomial.polyfromroots(np.delete(xi, a))
        c = c / np.polynomial.polynomial.polyval(xi[a], c)
        out[a] = np.polynomial.polynomial.polyval(xi, c)
    return out


def brute_element_mass(N, xi, ae_wJ):
    """(M_e)_{pq} = sum over quadrature nodes nu of alpha w J (nu) phi_p(nu)
    phi_q(nu): the mass operator of the weak form under GLL quadrature, with
    the basis values evaluated explicitly (its diagonal form is the lumping
    the paper derives from discrete orthogonality, not assumed here).
    ``ae_wJ`` holds alpha w_i w_j w_k J at the element's nodes."""
    V = lagrange_values_at_nodes(np.asarray(xi))
    Phi = np.kron(V.T, np.kron(V.T, V.T))  # [nu, p] = phi_p(nu)
    return Phi.T @ (np.asarray(ae_wJ)[:, None] * Phi)


def assemble_sparse(m: Mesh, masked=False):
    """Global sparse operator (stiffness, plus the mass term when the mesh has
    one) from brute-force element matrices."""
    import scipy.sparse as sp
    n3 = m.n1 ** 3
    rows, cols, vals = [], [], []
    for e in range(m.E):
        Ae = brute_element_matrix(m.N, m.xi, m.G[e])
        if m.H is not None:
            Ae = Ae + brute_element_mass(m.N, m.xi, m.H[e * n3:(e + 1) * n3])
        g = m.l2g[e * n3:(e + 1) * n3]
        rows.append(np.repeat(g, n3))
        cols.append(np.tile(g, n3))
        vals.append(Ae.reshape(-1))
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows),
                                              np.concatenate(cols))),
                      shape=(m.nG, m.nG)).tocsr()
    if masked:
        keep = np.ones(m.nG)
        keep[m.l2g[m.bmask.astype(bool)]] = 0
        Mk = sp.diags(keep)
        A = (Mk @ A @ Mk).tocsr()
    return A
