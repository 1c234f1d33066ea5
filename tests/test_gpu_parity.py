"""GPU parity of the HIP path (through the C ABI) against the FP64 CPU oracle.

Bars (tolerances written here; each follows from the arithmetic it checks):
  * maps (l2g, perm, offsets, mult, mask) and FP64 gather-scatter: bit-exact;
  * FP64 sem_ax: ||w_gpu - w_oracle||_inf / ||w_oracle||_inf <= 1e-12 on
    random continuous and discontinuous inputs, and componentwise
    |dw| <= 1e-12 (|A||u|) on smooth inputs;
  * geometry, mass, Jacobi diagonal, right-hand side: <= 1e-13 relative;
  * FP32 / BF16 sem_ax: error against the FP64 oracle reported, bounded;
  * PCG / refinement: solutions agree with the oracle's PCG solution.
Meshes span several workgroups with a ragged last one, every order 1..8.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from seminputs import fourier_modes, grf_features, uniform

from gpu_util import Pair, bf16_round, export, to_dev, to_host, torch

pytestmark = pytest.mark.gpu

AFF, SX, CYC = orc.MAP_AFFINE, orc.MAP_SINE_X, orc.MAP_SINE_CYCLIC

MESHES = [
    (1, 3, 2, 3, AFF), (2, 2, 3, 2, CYC), (3, 5, 3, 3, CYC),
    (4, 4, 4, 4, AFF), (5, 3, 3, 2, CYC), (6, 2, 2, 3, SX),
    (7, 3, 3, 5, CYC), (8, 2, 3, 2, CYC), (7, 1, 1, 1, CYC),
    (8, 2, 1, 2, CYC),  # 4 elements: ragged last workgroup of 3 at N = 8
]


def _kappa():
    return grf_features(seed=7, M=64, ell=0.3, sigma=0.5)


@pytest.fixture(scope="module")
def sem():
    from paper_1403_0968_amd import sem as s
    s.lib()
    return s


@pytest.fixture(scope="module", params=MESHES,
                ids=lambda p: f"N{p[0]}_{p[1]}x{p[2]}x{p[3]}_map{p[4]}")
def pair(request, sem):
    N, ex, ey, ez, mp = request.param
    kap = _kappa() if mp == CYC else None
    p = Pair(sem, N, ex, ey, ez, mapping=mp, dirichlet=1, kappa=kap)
    print(f"[gpu] mesh N={N} {ex}x{ey}x{ez} map={mp}", flush=True)
    yield p
    p.close()


def test_maps_bit_exact(sem, pair):
    m = pair.m
    t = torch()
    assert (pair.E, pair.nL, pair.nG) == (m.E, m.nL, m.nG)
    np.testing.assert_array_equal(export(sem, pair.h, sem.SEM_ARR_L2G, m.nL, t.int32), m.l2g)
    np.testing.assert_array_equal(export(sem, pair.h, sem.SEM_ARR_PERM, m.nL, t.int32), m.perm)
    np.testing.assert_array_equal(
        export(sem, pair.h, sem.SEM_ARR_OFFSETS, m.nG + 1, t.int32), m.offsets)
    np.testing.assert_array_equal(export(sem, pair.h, sem.SEM_ARR_MULT, m.nL, t.int32), m.mult)
    np.testing.assert_array_equal(export(sem, pair.h, sem.SEM_ARR_MASK, m.nL, t.uint8), m.bmask)


def test_geometry_matches_oracle(sem, pair):
    m = pair.m
    t = torch()
    X = export(sem, pair.h, sem.SEM_ARR_COORDS, 3 * m.nL, t.float64).reshape(3, -1)
    np.testing.assert_allclose(X, m.X, rtol=0, atol=1e-15)
    G = export(sem, pair.h, sem.SEM_ARR_GEOM, m.G.size, t.float64).reshape(m.G.shape)
    assert np.max(np.abs(G - m.G)) <= 1e-13 * np.max(np.abs(m.G))
    B = export(sem, pair.h, sem.SEM_ARR_MASS, m.nL, t.float64)
    assert np.max(np.abs(B - m.B)) <= 1e-13 * np.max(np.abs(m.B))
    d = export(sem, pair.h, sem.SEM_ARR_DIAG, m.nL, t.float64)
    dref = orc.local_diag(m)
    assert np.max(np.abs(d - dref)) <= 1e-13 * np.max(np.abs(dref))
    di = export(sem, pair.h, sem.SEM_ARR_DINV, m.nG, t.float64)
    diref = orc.jacobi_dinv_global(m)
    np.testing.assert_array_equal(di == 0, diref == 0)
    assert np.max(np.abs(di - diref)) <= 1e-13 * np.max(np.abs(diref))


def _ax_gpu(sem, h, u, prec):
    t = torch()
    if prec == sem.SEM_FP64:
        ud, wd = to_dev(u, t.float64), t.empty(len(u), dtype=t.float64, device="cuda")
    elif prec == sem.SEM_FP32:
        ud, wd = to_dev(u, t.float32), t.empty(len(u), dtype=t.float32, device="cuda")
    else:
        _, u16 = bf16_round(u)
        ud = to_dev(u16.view(np.int16), t.int16)
        wd = t.empty(len(u), dtype=t.float32, device="cuda")
    sem.sem_ax(h, prec, ud, wd)
    t.cuda.synchronize()
    return to_host(wd).astype(np.float64)


def test_ax_fp64_random(sem, pair):
    m = pair.m
    for kind in ("continuous", "discontinuous"):
        u = (orc.to_local(m, uniform(m.nG, seed=11)) if kind == "continuous"
             else uniform(m.nL, seed=12))
        w = _ax_gpu(sem, pair.h, u, sem.SEM_FP64)
        ref = orc.ax(m, u)
        err = np.max(np.abs(w - ref)) / np.max(np.abs(ref))
        print(f"[ax fp64 {kind}] rel err {err:.3e}")
        assert err <= 1e-12, (kind, err)


def test_ax_fp64_smooth_componentwise(sem, pair):
    m = pair.m
    x, y, z = m.X
    u = np.sin(2 * x + 1) * np.cos(3 * y) * np.exp(z)
    w = _ax_gpu(sem, pair.h, u, sem.SEM_FP64)
    ref = orc.ax(m, u)
    bound = orc.ax_abs(m, u)
    assert np.all(np.abs(w - ref) <= 1e-12 * bound + 1e-300)


def test_ax_low_precision_error_reported(sem, pair):
    m = pair.m
    u = uniform(m.nL, seed=13)
    ref = orc.ax(m, u)
    w32 = _ax_gpu(sem, pair.h, u, sem.SEM_FP32)
    e32 = np.max(np.abs(w32 - ref)) / np.max(np.abs(ref))
    ub, _ = bf16_round(u)
    refb = orc.ax(m, ub)
    w16 = _ax_gpu(sem, pair.h, u, sem.SEM_BF16)
    e16 = np.max(np.abs(w16 - refb)) / np.max(np.abs(refb))
    print(f"[ax fp32] rel err {e32:.3e}  [ax bf16 G, same bf16 u] rel err {e16:.3e}")
    assert e32 <= 2e-6
    assert e16 <= 2e-2


def test_gs_bit_exact(sem, pair):
    m = pair.m
    t = torch()
    rng = np.random.default_rng(5)
    v = rng.choice([1e16, -1e16, 1.0, 3.0, -7.0, 0.1], size=m.nL) + uniform(m.nL, 6)
    # negative zeros, on single-copy and on shared nodes: every sum starts
    # from +0.0, so the result holds +0.0 wherever all copies are -0.0
    v[::5] = -0.0
    v[m.perm[m.offsets[m.l2g[m.nL // 2]]:m.offsets[m.l2g[m.nL // 2] + 1]]] = -0.0
    vd = to_dev(v)
    sem.sem_gs(pair.h, sem.SEM_FP64, vd)
    t.cuda.synchronize()
    got = to_host(vd)
    ref = orc.gs(m, v)
    np.testing.assert_array_equal(got.view(np.uint64), ref.view(np.uint64))
    v32 = to_dev(v.astype(np.float32), t.float32)
    sem.sem_gs(pair.h, sem.SEM_FP32, v32)
    t.cuda.synchronize()
    ref32 = orc.gs(m, v.astype(np.float32).astype(np.float64))
    got32 = to_host(v32).astype(np.float64)
    assert np.max(np.abs(got32 - ref32)) <= 1e-6 * np.max(np.abs(ref32))


def test_rhs_and_jacobi_match_oracle(sem, pair):
    m = pair.m
    t = torch()
    k, a, phi = fourier_modes(seed=0)
    b = t.empty(m.nL, dtype=t.float64, device="cuda")
    sem.sem_rhs(pair.h, b, sem.SEM_SRC_FOURIER, (k, a, phi))
    t.cuda.synchronize()
    ref = orc.rhs_local(m, orc.src_fourier(m.X, k, a, phi))
    got = to_host(b)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    z = t.empty_like(b)
    sem.sem_precond_apply(pair.h, sem.SEM_PC_JACOBI, sem.SEM_FP64, b, z)
    t.cuda.synchronize()
    zref = orc.jacobi_dinv_global(m)[m.l2g] * ref
    assert np.max(np.abs(to_host(z) - zref)) <= 1e-13 * np.max(np.abs(zref))


def test_determinism(sem, pair):
    m = pair.m
    t = torch()
    u = to_dev(uniform(m.nL, seed=21))
    w1 = t.empty_like(u)
    w2 = t.empty_like(u)
    sem.sem_ax(pair.h, sem.SEM_FP64, u, w1)
    sem.sem_ax(pair.h, sem.SEM_FP64, u, w2)
    sem.sem_gs(pair.h, sem.SEM_FP64, w1)
    sem.sem_gs(pair.h, sem.SEM_FP64, w2)
    t.cuda.synchronize()
    assert t.equal(w1, w2)


def test_ax_matrix_core_against_oracle(sem, pair):
    """Matrix-core BF16 operator (split derivative matrix) against the
    oracle applied to the same BF16-rounded input: the remaining error is
    the BF16 storage of G and of the fluxes (~2^-9 relative each)."""
    m = pair.m
    u = uniform(m.nL, seed=14)
    ub, _ = bf16_round(u)
    refb = orc.ax(m, ub)
    wm = _ax_gpu(sem, pair.h, u, sem.SEM_BF16_MFMA)
    em = np.max(np.abs(wm - refb)) / np.max(np.abs(refb))
    wv = _ax_gpu(sem, pair.h, u, sem.SEM_BF16)
    ev = np.max(np.abs(wv - refb)) / np.max(np.abs(refb))
    print(f"[ax bf16 N={m.N}] matrix cores {em:.3e}, VALU {ev:.3e}")
    assert em <= 2e-2


def test_ax_matrix_core_split_derivative(sem, pair):
    """A constant is differentiated to zero exactly, so A_L 1 = 0: with the
    two-term BF16 split of D the residue is at the split's 2^-16 level, with
    D rounded to BF16 it is at 2^-9 (the error refinement cannot remove)."""
    m = pair.m
    one = np.ones(m.nL)
    scale = np.max(orc.ax_abs(m, one))
    ws = _ax_gpu(sem, pair.h, one, sem.SEM_BF16_MFMA)
    wp = _ax_gpu(sem, pair.h, one, sem.SEM_BF16_PLAIN_D)
    wv = _ax_gpu(sem, pair.h, one, sem.SEM_BF16)
    es, ep, ev = (np.max(np.abs(w)) / scale for w in (ws, wp, wv))
    print(f"[A 1, N={m.N}] split {es:.2e}, plain {ep:.2e}, VALU FP32-D {ev:.2e}")
    assert es <= 1e-4
    if m.N < 2:
        # N = 1: D = [[-1/2, 1/2], [-1/2, 1/2]] is exact in BF16, so its low
        # term vanishes (up to the host's rounding of D) and both forms agree:
        # A 1 = 0 to the split's level with D rounded as well
        assert ep <= 1e-4
        assert np.max(np.abs(ws - wp)) <= 1e-6 * scale
    else:
        assert ep >= 10 * es


def test_ax_matrix_core_transposed_split(sem, pair):
    """The transposed contractions sum to zero over each element for any
    input: sum_i (D^T f)_i = f . (D 1) = 0 for every flux f, so the element
    sums of w vanish whatever the BF16 rounding of u, G and the fluxes.
    With the split derivative matrix the residue is at the split's 2^-16
    level; with D rounded to BF16 (whose rows no longer sum to zero) at
    2^-9 -- this exercises the transposed stage, where A 1 (zero fluxes)
    cannot."""
    m = pair.m
    u = uniform(m.nL, seed=15)
    n3 = m.n1 ** 3
    scale = orc.ax_abs(m, np.abs(bf16_round(u)[0])).reshape(m.E, n3).sum(1)
    wfs = _ax_gpu(sem, pair.h, u, sem.SEM_BF16_MFMA)
    wfp = _ax_gpu(sem, pair.h, u, sem.SEM_BF16_PLAIN_D)
    ws = wfs.reshape(m.E, n3).sum(1)
    wp = wfp.reshape(m.E, n3).sum(1)
    es = float(np.max(np.abs(ws) / scale))
    ep = float(np.max(np.abs(wp) / scale))
    print(f"[element sums of w, N={m.N}] split {es:.2e}, plain {ep:.2e}")
    assert es <= 1e-4
    if m.N < 3:
        # at N <= 2 every entry of D is exact in BF16: the split's low term
        # vanishes (up to the host's rounding of D) and both forms agree
        assert np.max(np.abs(wfs - wfp)) <= 1e-6 * np.max(np.abs(wfp))
    else:
        assert ep >= 10 * es
